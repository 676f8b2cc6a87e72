"""Batched planning (vopp_batch_*): every instance's result must be bit-identical
to a plain vopp_plan call with the same inputs, in every mode (the persistent
launch over a device queue, the per-phase launches replayed from their hipGraph
or issued one by one), on every replay, and for every launch shape the
autotuner tries."""

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests.drawcheck import forced_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27191_amd import vopp
    vopp.lib()
    return vopp


def small_mix(seed, n):
    """A reduced mix: tabular and navigation, uneven n_p / depth / budget."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        depth = int(rng.integers(2, 7))
        K = int(rng.integers(1, depth + 1))
        n_p = int(rng.integers(100, 3000))
        sched = int(rng.integers(0, 2))
        if i % 2 == 0:
            inst = I.tabular_sparse(int(rng.integers(0, 1000)), int(rng.integers(20, 200)),
                                    int(rng.integers(2, 9)), int(rng.integers(2, 12)), 4,
                                    with_heuristic=bool(i % 4 == 0))
            bel = I.tabular_belief(inst)
        else:
            inst = I.nav2d(int(rng.integers(0, 1000)), int(rng.integers(4, 12)),
                           heuristic=int(i % 3 == 0))
            bel = I.nav_belief(int(rng.integers(0, 1000)), 500,
                               *( (7.0, 8.5) if i % 5 == 1 else (0.5, 1.5) ))
        out.append((inst, bel, dict(n_particles=n_p, budget=K, depth=depth, eta=1.0,
                                    seed=int(rng.integers(1, 2 ** 40)), schedule=sched)))
    return out


def build(V, mix):
    items, keep = [], []
    for inst, bel, p in mix:
        pom = V.Pomdp.from_instance(inst)
        belt = V.belief_tensor(inst, bel)
        nb = belt.numel() if inst["kind"] == "tabular" else belt.numel() // 2
        prm = V.params(p["n_particles"], eta=p["eta"], seed=p["seed"],
                       schedule=p["schedule"])
        items.append((pom, belt, nb, p["budget"], p["depth"], prm))
        keep.append((pom, belt))
    return items, keep


def plain(V, items):
    out = []
    for pom, belt, nb, K, depth, prm in items:
        out.append(V.plan(pom, belt, nb, K, depth, prm))
    return out


def same(a, b):
    assert a.action == b.action
    assert np.array_equal(a.values, b.values)
    assert a.v_root == b.v_root
    assert (a.particle_steps, a.n_beliefs, a.n_actions) == (b.particle_steps, b.n_beliefs,
                                                            b.n_actions)


def test_batch_equals_plain_plans(V):
    items, keep = build(V, small_mix(1, 14))
    ref = plain(V, items)
    batch = V.Batch(items)
    assert batch.num_launches > 10
    for mode in (V.BATCH_PERSISTENT, V.BATCH_GRAPH, V.BATCH_EAGER, V.BATCH_PERSISTENT):
        res, ms = batch.run(mode=mode)
        assert ms > 0
        for a, b in zip(res, ref):
            same(a, b)
    batch.close()


@pytest.mark.parametrize("tuning", [(1, 1, 1, 1, 1), (7, 3, 1, 3, 5), (4096, 4096, 0, 1, 1),
                                    (16, 16, 0, 64, 1000)])
def test_persistent_launch_shapes(V, tuning):
    # One tile per sweep and one block per CU (each tile loops over many chunks
    # of record positions, and few blocks serve many instances), odd tile
    # counts, and large ones: the same results.
    items, keep = build(V, small_mix(5, 9))
    ref = plain(V, items)
    batch = V.Batch(items, tuning=tuning)
    for _ in range(2):
        res, _ = batch.run(mode=V.BATCH_PERSISTENT)
        for a, b in zip(res, ref):
            same(a, b)
    batch.close()


def test_graph_replays_with_new_requests(V):
    import torch
    mix = small_mix(2, 10)
    items, keep = build(V, mix)
    batch = V.Batch(items)
    for rep in range(3):
        # Eager work and synchronisation between replays.
        x = torch.randn(1000, device="cuda")
        _ = (x * 2).sum().item()
        new_items = []
        for i, (pom, belt, nb, K, depth, prm) in enumerate(items):
            seed = 1000 * rep + 17 * i + 3
            batch.set_request(i, belt, nb, seed, step=rep)
            new_items.append((pom, belt, nb, K, depth,
                              V.params(prm.n_particles, eta=prm.eta, seed=seed,
                                       schedule=prm.schedule, step=rep)))
        res, _ = batch.run(mode=V.BATCH_PERSISTENT)
        per_phase, _ = batch.run(mode=V.BATCH_GRAPH)
        eager, _ = batch.run(mode=V.BATCH_EAGER)
        ref = plain(V, new_items)
        for a, b, c, d in zip(res, per_phase, eager, ref):
            same(a, d)
            same(b, d)
            same(c, d)
    batch.close()


def oracle_checked(V, orc, inst, bel, n_p, K, depth, seed):
    """The plain plan of one instance held to the oracle bar (tests/drawcheck.py)
    with no flagged draw decided differently, so the unforced plan -- and any
    plan bit-identical to it -- meets the bar too."""
    st = forced_parity(V, orc, inst, bel, n_p, K, depth, seed=seed)
    assert st["follow"] == 0
    return st


@pytest.mark.parametrize("tuning", [None, (1, 1)])
def test_batch_instances_match_oracle(V, orc, tuning):
    # One tabular and one navigation instance inside a mix, each equal to its
    # oracle-checked plain plan.  tuning (1, 1) runs every accumulate and
    # backup sweep of the batch on one block, so each block loops over many
    # chunks of record positions (the sweeps' grid-stride path).
    tab = I.tabular_sparse(5, 300, 5, 7, 4, with_heuristic=True)
    tab_bel = I.tabular_belief(tab)
    nav = I.nav2d(7, 6, heuristic=1)
    nav_bel = I.nav_belief(2, 900)
    st_t = oracle_checked(V, orc, tab, tab_bel, 3000, 4, 4, 3)
    st_n = oracle_checked(V, orc, nav, nav_bel, 2600, 4, 5, 4)
    mix = small_mix(3, 5)
    items, keep = build(V, mix)
    for at, (inst, bel, n_p, K, depth, sd) in ((2, (tab, tab_bel, 3000, 4, 4, 3)),
                                               (4, (nav, nav_bel, 2600, 4, 5, 4))):
        pom = V.Pomdp.from_instance(inst)
        belt = V.belief_tensor(inst, bel)
        nb = belt.numel() if inst["kind"] == "tabular" else belt.numel() // 2
        items.insert(at, (pom, belt, nb, K, depth, V.params(n_p, seed=sd)))
        keep.append((pom, belt))
    ref = plain(V, items)
    batch = V.Batch(items, tuning=tuning)
    for mode in (V.BATCH_PERSISTENT, V.BATCH_GRAPH):
        res, _ = batch.run(mode=mode)
        for a, b in zip(res, ref):
            same(a, b)
        for r, st in ((res[2], st_t), (res[4], st_n)):
            same(r, st["res"])
    batch.close()


def test_autotune_keeps_results(V):
    items, keep = build(V, small_mix(4, 8))
    ref = plain(V, items)
    batch = V.Batch(items)
    assert batch.auto_mode == V.BATCH_PERSISTENT
    chosen = batch.autotune(reps=1)
    assert chosen[2] >= 0 and chosen[3] in (1, 4) and chosen[4] in (1, 2, 4, 8)
    # Block caps of the per-phase graph: 256 each, or the plain plan's.
    assert (chosen[0], chosen[1]) in ((256, 256), (4096, 2048))
    assert batch.auto_mode in (V.BATCH_GRAPH, V.BATCH_PERSISTENT)
    for mode in (V.BATCH_AUTO, V.BATCH_GRAPH, V.BATCH_PERSISTENT):
        res, _ = batch.run(mode=mode)
        for a, b in zip(res, ref):
            same(a, b)
    batch.close()


def test_batch_rejects_large_action_sets(V):
    inst = I.tabular_dense(0, 4, 20, 2)
    pom = V.Pomdp.from_instance(inst)
    belt = V.belief_tensor(inst, I.tabular_belief(inst))
    with pytest.raises(V.VoppError) as e:
        V.Batch([(pom, belt, 4, 2, 2, V.params(64))])
    assert e.value.status == V.VOPP_E_INVALID
