"""Serving (vopp_server_*): every planning request of every episode gives the
same result whether the episode is served alone or in a mix of concurrent
episodes, and the same as the plain single-request path (vopp_plan, then
vopp_env_step and vopp_belief_update between steps)."""

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27191_amd import vopp
    vopp.lib()
    return vopp


def episodes(n):
    rng = np.random.default_rng(42)
    out = []
    for i in range(n):
        depth = int(rng.integers(2, 6))
        n_p = int(rng.integers(200, 2500))
        if i % 2 == 0:
            inst = I.tabular_sparse(int(rng.integers(0, 999)), int(rng.integers(16, 120)),
                                    int(rng.integers(2, 7)), int(rng.integers(2, 9)), 4,
                                    with_heuristic=True)
            parts = (np.arange(n_p) % inst["nS"]).astype(np.int32)
            state = int(rng.integers(0, inst["nS"]))
            bel = parts
        else:
            inst = I.nav2d(int(rng.integers(0, 999)), 6, heuristic=1)
            bel = I.nav_belief(int(rng.integers(0, 999)), n_p, 0.5, 1.5)
            state = (1.0, 1.2)
        out.append(dict(inst=inst, belief=bel, n_p=n_p, budget=depth, depth=depth,
                        seed=int(rng.integers(1, 2 ** 40)), env_seed=int(rng.integers(1, 2 ** 40)),
                        state=state, steps=4))
    return out


def plain_episode(V, ep):
    import torch
    pom = V.Pomdp.from_instance(ep["inst"])
    parts = torch.as_tensor(V.particles_host(ep["inst"], ep["belief"]), device="cuda")
    if ep["inst"]["kind"] == "tabular":
        state = torch.tensor([ep["state"]], dtype=torch.int32, device="cuda")
    else:
        state = torch.tensor(ep["state"], dtype=torch.float32, device="cuda")
    out = []
    for t in range(ep["steps"]):
        prm = V.params(ep["n_p"], seed=ep["seed"], step=t)
        r = V.plan(pom, parts, ep["n_p"], ep["budget"], ep["depth"], prm)
        out.append((r.action, r.v_root, r.particle_steps))
        if t + 1 < ep["steps"]:
            obs, _, _ = V.env_step(pom, state, r.action, ep["env_seed"], t)
            V.belief_update(pom, parts, ep["n_p"], r.action, obs, ep["seed"], t)
    pom.close()
    return out


def serve(V, eps, max_active=64, budget=64 << 30, phases_per_tick=1):
    srv = V.Server(hbm_budget_bytes=budget, max_active=max_active,
                   phases_per_tick=phases_per_tick)
    poms = [V.Pomdp.from_instance(ep["inst"]) for ep in eps]
    ids = []
    for pom, ep in zip(poms, eps):
        ids.append(srv.submit(pom, V.particles_host(ep["inst"], ep["belief"]), ep["budget"],
                              ep["depth"], V.params(ep["n_p"], seed=ep["seed"]), ep["state"],
                              ep["env_seed"], ep["steps"]))
    res = srv.run_until_idle()
    by = {}
    for r in res:
        assert r["status"] == 0
        assert r["done_s"] >= r["arrival_s"]
        by[(r["episode"], r["step"])] = (r["action"], r["v_root"], r["particle_steps"])
    srv.close()
    for p in poms:
        p.close()
    return [[by[(i, t)] for t in range(ep["steps"])] for i, ep in zip(ids, eps)]


def test_served_mix_equals_alone_and_plain(V):
    eps = episodes(8)
    mixed = serve(V, eps)
    for ep, got in zip(eps, mixed):
        assert got == plain_episode(V, ep)
    alone = serve(V, eps[3:4])
    assert alone[0] == mixed[3]
    # Several phases per tick: the same results.
    for ppt in (5, 64):
        assert serve(V, eps, phases_per_tick=ppt) == mixed


def test_admission_by_budget_and_slots(V):
    import torch
    eps = episodes(6)
    # Two slots: later episodes wait for free slots and still match.
    small = serve(V, eps, max_active=2)
    for ep, got in zip(eps, small):
        assert got == plain_episode(V, ep)
    # A budget that fits one footprint at a time.
    pom = V.Pomdp.from_instance(eps[0]["inst"])
    fp = V.footprint(pom, V.params(eps[0]["n_p"]), eps[0]["budget"], eps[0]["depth"])
    pom.close()
    one = serve(V, eps[:1] * 3, budget=int(fp * 1.5))
    assert one[0] == one[1] == one[2]


def test_oversized_episode_rejected(V):
    eps = episodes(1)
    srv = V.Server(hbm_budget_bytes=4096, max_active=4)
    pom = V.Pomdp.from_instance(eps[0]["inst"])
    with pytest.raises(V.VoppError) as e:
        srv.submit(pom, V.particles_host(eps[0]["inst"], eps[0]["belief"]), 2, 2,
                   V.params(eps[0]["n_p"]), eps[0]["state"], 1, 2)
    assert e.value.status == V.VOPP_E_NOMEM
    srv.close()
    pom.close()


def test_episode_chain_matches_oracle(V, orc):
    # One tabular and one navigation episode of the mix, step by step against
    # the oracle's own chain (plan, true-environment step, SIR belief update):
    # every plan meets the parity bar of tests/drawcheck.py with no flagged
    # draw decided differently, the environment gives the same observation,
    # and the updated particles are equal bit for bit.  The served requests of
    # the same episodes equal this plain chain (test above), so they meet the
    # bar too.
    import torch
    from tests.drawcheck import (assert_tree_parity, check_draws, gpu_forced_plan,
                                 oracle_plan)
    eps = episodes(4)[:2]
    served = serve(V, eps)
    for ep, got in zip(eps, served):
        inst = ep["inst"]
        tab = inst["kind"] == "tabular"
        pom = V.Pomdp.from_instance(inst)
        parts = torch.as_tensor(V.particles_host(inst, ep["belief"]), device="cuda")
        state = torch.tensor([ep["state"]] if tab else ep["state"],
                             dtype=torch.int32 if tab else torch.float32, device="cuda")
        o_parts = ep["belief"] if tab else (ep["belief"][0], ep["belief"][1])
        o_state = ep["state"]
        ws = V.Workspace(pom, V.params(ep["n_p"]), ep["budget"], ep["depth"])
        try:
            for t in range(ep["steps"]):
                o = oracle_plan(orc, inst, o_parts, ep["n_p"], ep["budget"], ep["depth"],
                                seed=ep["seed"], step=t)
                r, tree, act, obs = gpu_forced_plan(V, pom, ws, inst, parts, ep["n_p"],
                                                    ep["n_p"], ep["budget"], ep["depth"], o,
                                                    seed=ep["seed"], step=t)
                follow, _, _ = check_draws(o, act, obs)
                assert follow == 0
                assert_tree_parity(r, tree, o, inst["nA"])
                assert r.action == o.action
                assert got[t] == (r.action, r.v_root, r.particle_steps)
                if t + 1 == ep["steps"]:
                    break
                o_state, o_obs, _, _ = orc.env_step(inst, o_state, o.action, ep["env_seed"], t)
                g_obs, _, _ = V.env_step(pom, state, r.action, ep["env_seed"], t)
                assert g_obs == o_obs
                o_parts, _ = orc.belief_update(inst, o_parts, o.action, o_obs, ep["seed"], t)
                V.belief_update(pom, parts, ep["n_p"], r.action, g_obs, ep["seed"], t)
                host = parts.cpu().numpy()
                if tab:
                    assert np.array_equal(host, o_parts)
                else:
                    n = ep["n_p"]
                    assert np.array_equal(host[:n].view(np.uint32),
                                          np.asarray(o_parts[0], np.float32).view(np.uint32))
                    assert np.array_equal(host[n:].view(np.uint32),
                                          np.asarray(o_parts[1], np.float32).view(np.uint32))
        finally:
            ws.close()
            pom.close()
