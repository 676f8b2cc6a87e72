"""The anytime planning step (Alg. 1 with a wall-clock budget) through the C
ABI: the iteration count K' is decided on the device at the end of each
iteration, and the plan must be the plain K'-iteration plan.

The tabular workload here (n_p = 1024, K <= 32, |R| < 1, gamma = 0.95) keeps
the fixed-point resolution of the sums at its finest setting for every K, so
the anytime plan and the plain plan at K' agree bit for bit.  The plain plan
at K' is held to the oracle parity bar of tests/drawcheck.py; with no flagged
draw decided differently (follow count 0) it is the unforced plan, so the
anytime plan meets the bar too.
"""

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests.drawcheck import (assert_tree_parity as assert_parity, check_draws, gpu_forced_plan,
                             oracle_plan)

pytestmark = pytest.mark.gpu

N_P, DEPTH, KMAX, SEED = 1024, 4, 32, 18


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27191_amd import vopp
    vopp.lib()
    return vopp


@pytest.fixture(scope="module")
def setup(V):
    inst, bel, _ = I.workload("tabular16", seed=0)
    pom = V.Pomdp.from_instance(inst)
    prm = V.params(N_P, seed=SEED)
    ws = V.Workspace(pom, prm, KMAX, DEPTH)
    b = V.belief_tensor(inst, bel)
    yield inst, bel, pom, prm, ws, b
    ws.close()
    pom.close()


def plain(V, setup, K):
    inst, bel, pom, prm, ws, b = setup
    res = V.plan(pom, b, b.numel(), K, DEPTH, prm, ws=ws)
    return res, V.tree_dump(ws, pom.nA, res.n_beliefs, res.n_actions)


def anytime(V, setup, time_ms, kmax=KMAX):
    inst, bel, pom, prm, ws, b = setup
    res, k = V.plan_anytime(pom, b, b.numel(), kmax, DEPTH, time_ms, prm, ws=ws)
    return res, k, V.tree_dump(ws, pom.nA, res.n_beliefs, res.n_actions)


def same(r0, t0, r1, t1):
    assert r0.action == r1.action
    assert np.array_equal(r0.values, r1.values)
    assert r0.v_root == r1.v_root
    assert (r0.particle_steps, r0.n_beliefs, r0.n_actions) == \
        (r1.particle_steps, r1.n_beliefs, r1.n_actions)
    for k in t0:
        assert np.array_equal(t0[k], t1[k]), k


def test_tiny_budget_runs_one_iteration(V, setup):
    r, k, t = anytime(V, setup, 1e-6)
    assert k == 1
    same(r, t, *plain(V, setup, 1))


def test_ample_budget_runs_the_cap(V, setup):
    r, k, t = anytime(V, setup, 1e6)
    assert k == KMAX
    same(r, t, *plain(V, setup, KMAX))


def test_cap_below_workspace_size(V, setup):
    r, k, t = anytime(V, setup, 1e6, kmax=7)
    assert k == 7
    same(r, t, *plain(V, setup, 7))


def test_budget_stops_midway_and_equals_plain_plan(V, setup):
    # Time the full plan, then give about a third of it.
    full, _, _ = anytime(V, setup, 1e6)
    budget = max(full.device_ms / 3.0, 0.05)
    r, k, t = anytime(V, setup, budget)
    assert 1 <= k <= KMAX
    if k < KMAX:
        # It stopped because the budget was spent after iteration k.
        assert r.device_ms >= budget
    same(r, t, *plain(V, setup, k))
    # Level counts describe the K'-iteration tree.
    counts = V.level_counts(setup[4])
    assert len(counts) == sum(min(i, DEPTH) for i in range(1, k + 1))


def test_anytime_matches_oracle(V, orc, setup):
    inst, bel = setup[0], setup[1]
    full, _, _ = anytime(V, setup, 1e6)
    r, k, t = anytime(V, setup, max(full.device_ms / 2.0, 0.05))
    o = oracle_plan(orc, inst, bel, N_P, k, DEPTH, seed=SEED, schedule=0)
    _, _, pom, prm, ws, b = setup
    rf, tf, act, obs = gpu_forced_plan(V, pom, ws, inst, b, b.numel(), N_P, k, DEPTH, o,
                                       seed=SEED)
    follow, _, _ = check_draws(o, act, obs)
    assert_parity(rf, tf, o, 3)
    assert follow == 0
    same(r, t, rf, tf)


def test_plain_plan_after_anytime_plan(V, setup):
    # The workspace keeps no anytime state that changes a later plain plan.
    r0, t0 = plain(V, setup, 5)
    anytime(V, setup, 1e-6)
    anytime(V, setup, 1e6)
    r1, t1 = plain(V, setup, 5)
    same(r0, t0, r1, t1)


def test_bad_time_budget_rejected(V, setup):
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(V.VoppError):
            anytime(V, setup, bad)
