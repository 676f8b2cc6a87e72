"""Parity of the HIP planner with the oracle at MARS-sized action sets
(|A| = 625 and 3025; rows of more than 64 actions are drawn from memory and
swept by one wavefront per belief).

Every plan is held to the protocol of tests/drawcheck.py.  Iteration 1 draws
only from initial rows (double-precision running sums on both sides), so it
is exact at the benchmark sizes.  Later iterations draw from rows the kernel
keeps in single precision, with single-precision weights summed by quads in
double precision.  The benchmark shapes (mars625 and mars3025 at n_p 16,384,
K 4, depth 4) are held to the full bar.
"""

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests.drawcheck import (assert_tree_parity as assert_parity, check_draws, forced_parity,
                             gpu_forced_plan, oracle_plan)
from tests.test_gpu_parity import gpu_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27191_amd import vopp
    vopp.lib()
    return vopp


def run_gpu(V, inst, bel, n_p, K, depth, seed, schedule=0):
    pom = V.Pomdp.from_instance(inst)
    try:
        prm = V.params(n_p, seed=seed, schedule=schedule)
        ws = V.Workspace(pom, prm, K, depth)
        b = V.belief_tensor(inst, bel)
        res = V.plan(pom, b, b.numel(), K, depth, prm, ws=ws)
        tree = V.tree_dump(ws, pom.nA, res.n_beliefs, res.n_actions)
        ws.close()
    finally:
        pom.close()
    return res, tree


@pytest.mark.parametrize("name", ["mars625", "mars3025"])
def test_first_iteration_full_size(V, orc, name):
    inst, bel, p = I.workload(name, seed=0)
    n_p, depth = p["n_particles"], p["depth"]
    st = forced_parity(V, orc, inst, bel, n_p, 1, depth, seed=3, schedule=1)
    assert st["flagged"] == 0


@pytest.mark.parametrize("name", ["mars625", "mars3025"])
def test_full_size_plan(V, orc, name):
    """The benchmark shapes, every iteration: every draw, the tree, the values."""
    inst, bel, p = I.workload(name, seed=0)
    n_p, K, depth = p["n_particles"], p["budget"], p["depth"]
    st = forced_parity(V, orc, inst, bel, n_p, K, depth, seed=1, max_flag_frac=0.2)
    print(f"[parity] {name} full size: draws {st['draws']} flagged {st['flagged']} "
          f"followed {st['follow']}", flush=True)
    gpu_invariants(st["res"], st["tree"], n_p, K, depth, 0)


# 65 actions: the shortest long row; 1500, 3025 and 4096: the sweeps that hold
# 8, 12 and 16 quads of the row per lane.
@pytest.mark.parametrize("nS,A,n_p,K,depth", [(256, 625, 1024, 3, 3), (128, 3025, 768, 3, 3),
                                             (256, 625, 2048, 4, 4), (128, 65, 1024, 3, 3),
                                             (64, 1500, 768, 3, 3), (64, 4096, 512, 3, 3)])
def test_reduced_plan(V, orc, nS, A, n_p, K, depth):
    inst = I.mars_like(1, nS, A)
    bel = I.tabular_belief(inst)
    forced_parity(V, orc, inst, bel, n_p, K, depth, seed=1, max_flag_frac=0.2)


def test_wide_reference_policy(V, orc):
    # A non-uniform pi0 over 625 actions: iteration 1 draws from the initial
    # row's double-precision running sums on both sides.
    inst = I.mars_like(2, 128, 625)
    bel = I.tabular_belief(inst)
    pi0 = np.random.default_rng(3).uniform(0.5, 2.0, size=625)
    # The root row of 625 non-uniform entries has 624 boundaries, so the
    # screen flags many root draws; both sides draw them in double precision.
    st = forced_parity(V, orc, inst, bel, 1024, 1, 3, seed=1, pi0=pi0, max_flag_frac=0.2)
    assert st["follow"] == 0
    forced_parity(V, orc, inst, bel, 1024, 2, 3, seed=2, pi0=pi0, max_flag_frac=0.2)


def test_wide_limits(V):
    inst = I.mars_like(5, 8, 4096, nO=9)
    pom = V.Pomdp.from_instance(inst)
    pom.close()
    with pytest.raises(V.VoppError):
        V.Pomdp.from_instance(I.mars_like(5, 8, 4097, nO=9))
    with pytest.raises(V.VoppError):             # 2049+ actions leave 14 observation bits
        V.Pomdp.from_instance(I.mars_like(5, 1, 2049, nO=16385, n_succ=1))


def test_wide_anytime_and_reroot(V, orc):
    # The anytime plan and a kept subtree with 625 actions: the anytime plan
    # with ample time equals the plain plan, and a plan from the kept subtree
    # matches the oracle's plan from its own kept subtree.
    from tests.test_oracle_reroot import branches
    inst = I.mars_like(3, 128, 625)
    bel = I.tabular_belief(inst)
    sd = 1
    o1 = oracle_plan(orc, inst, bel, 1024, 3, 3, seed=sd, keep=True)
    a, ob = branches(o1, 625, 1)[0]
    h, _ = orc.reroot(o1, a, ob, 625)
    o2 = oracle_plan(orc, inst, bel, 1024, 2, 3, seed=sd + 100, start=h)
    pom = V.Pomdp.from_instance(inst)
    b = V.belief_tensor(inst, bel)
    p1, p2 = V.params(1024, seed=sd), V.params(1024, seed=sd + 100)
    A_ws, B_ws, C_ws = V.Workspace(pom, p1, 3, 3), V.Workspace(pom, p2, 2, 3), \
        V.Workspace(pom, p1, 3, 3)
    try:
        r1, t1, act, obs = gpu_forced_plan(V, pom, A_ws, inst, b, b.numel(), 1024, 3, 3, o1,
                                           seed=sd)
        check_draws(o1, act, obs)
        assert_parity(r1, t1, o1, 625)
        plain = V.plan(pom, b, b.numel(), 3, 3, p1, ws=C_ws)
        q, k = V.plan_anytime(pom, b, b.numel(), 3, 3, 1e6, p1, ws=C_ws)
        assert k == 3 and np.array_equal(q.values, plain.values)
        assert V.reroot(pom, A_ws, a, ob, p2, 2, 3, B_ws) == len(
            orc.reroot(o1, a, ob, 625)[1]["b_parent"])
        r2, t2, act, obs = gpu_forced_plan(V, pom, B_ws, inst, b, b.numel(), 1024, 2, 3, o2,
                                           seed=sd + 100)
        check_draws(o2, act, obs)
        assert_parity(r2, t2, o2, 625)
    finally:
        for w in (A_ws, B_ws, C_ws):
            w.close()
        pom.close()


def test_wide_anytime_stops_early_and_equals_plain_plan(V):
    # 625 actions: an anytime plan stopped after one iteration, and one
    # stopped about a third of the way, equal the plain plan at the realised
    # K' bit for bit (the claim pass and every later phase of an iteration
    # that does not run return at once).  The fixed-point shift is at its
    # cap for every K here (rewards scaled by 0.05), so the two plans sum on
    # the same grid.
    inst = I.mars_like(4, 128, 625, reward_scale=0.05)
    bel = I.tabular_belief(inst)
    kmax, depth = 8, 3
    pom = V.Pomdp.from_instance(inst)
    b = V.belief_tensor(inst, bel)
    prm = V.params(1024, seed=5)
    ws = V.Workspace(pom, prm, kmax, depth)

    def plain(K):
        r = V.plan(pom, b, b.numel(), K, depth, prm, ws=ws)
        return r, V.tree_dump(ws, 625, r.n_beliefs, r.n_actions)

    def anytime(ms):
        r, k = V.plan_anytime(pom, b, b.numel(), kmax, depth, ms, prm, ws=ws)
        return r, k, V.tree_dump(ws, 625, r.n_beliefs, r.n_actions)

    def same(a, ta, c, tc):
        assert a.action == c.action and a.v_root == c.v_root
        assert np.array_equal(a.values, c.values)
        assert (a.particle_steps, a.n_beliefs, a.n_actions) == \
            (c.particle_steps, c.n_beliefs, c.n_actions)
        for key in ta:
            assert np.array_equal(ta[key], tc[key]), key

    try:
        full, kf, _ = anytime(1e6)
        assert kf == kmax
        r, k, t = anytime(1e-6)
        assert k == 1
        same(r, t, *plain(1))
        r, k, t = anytime(max(full.device_ms / 3.0, 0.05))
        assert 1 <= k <= kmax
        same(r, t, *plain(k))
    finally:
        ws.close()
        pom.close()
