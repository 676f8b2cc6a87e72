"""Pins of the serial CPU oracle against what the method and mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, an independent replay, the exact
reference-based Bellman recursion, soft value iteration, the expected-count
limit of Alg. 1-3, and invariants.  The ``mutate`` flag plants known mistakes
in the oracle to show that the pins catch them.
"""

import math
import os

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests import refimpl as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- Philox -----------------------------------------------------------------

def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, out in _kat_rows():
        assert orc.philox(ctr, key).tolist() == out
        assert list(R.philox(ctr, key)) == out


def test_philox_matches_independent_python(orc):
    rng = np.random.default_rng(7)
    for _ in range(300):
        c = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        assert orc.philox(c, k).tolist() == list(R.philox(c, k))


# --- threshold sampler ----------------------------------------------------------

def test_thresholds_match_probabilities(orc):
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 8, 32, 100):
        p = rng.dirichlet(0.5 * np.ones(n)).astype(np.float32)
        thr = orc.thresholds(p).astype(np.int64)
        assert thr[-1] == 2 ** 31
        assert np.all(np.diff(thr) >= 0)
        got = np.diff(np.concatenate([[0], thr])) / 2.0 ** 31
        want = p.astype(np.float64) / p.astype(np.float64).sum()
        assert np.max(np.abs(got - want)) <= 2.0 ** -31 + 1e-15
        assert thr.tolist() == R.thresholds(p).tolist()


def test_pick_boundaries_and_zero_mass(orc):
    p = np.array([0.25, 0.0, 0.5, 0.0, 0.25], np.float32)
    thr = orc.thresholds(p)
    assert thr.tolist() == [2 ** 29, 2 ** 29, 3 * 2 ** 29, 3 * 2 ** 29, 2 ** 31]
    # u = x >> 1: the first u of each outcome and the last u of the previous.
    for j, lo in ((0, 0), (2, 2 ** 29), (4, 3 * 2 ** 29)):
        assert orc.pick(thr, 2 * lo) == j
        assert orc.pick(thr, 2 * lo + 1) == j
    assert orc.pick(thr, 2 * (2 ** 29) - 1) == 0
    assert orc.pick(thr, 2 * (3 * 2 ** 29) - 1) == 2
    assert orc.pick(thr, 0xFFFFFFFF) == 4
    # Zero-mass outcomes are never drawn.
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2 ** 32, size=2000):
        assert orc.pick(thr, int(x)) in (0, 2, 4)


def test_root_draw_counts_closed_form():
    # idx = (x*M) >> 32 hits index i exactly ceil((i+1)2^32/M) - ceil(i 2^32/M)
    # times; check the formula on a brute-force count over a 2^20 sub-grid
    # scaled to 32 bits (x = j << 12).
    for M in (3, 7, 16, 1000):
        counts = np.bincount(((np.arange(2 ** 20, dtype=np.uint64) << np.uint64(12))
                              * np.uint64(M)) >> np.uint64(32), minlength=M)
        want = R.root_probs(M) * 2 ** 20
        assert np.max(np.abs(counts - want)) <= 1.0


# --- action sampling (Eq. 6) ---------------------------------------------------

def test_uniform_row_draw_is_floor_u_times_A(orc):
    # With every preference equal, the softmax of Eq. (6) is uniform and the
    # inverse-CDF draw is floor(u |A|) for u = (x0 >> 8) 2^-24, at every
    # belief; such a draw is never a near tie.
    rng = np.random.default_rng(1)
    xs = list(rng.integers(0, 2 ** 32, size=3000)) + [0, 0xFFFFFFFF, 0x80000000]
    for A in (1, 2, 3, 4, 5, 6, 8, 64):
        psi = np.full(A, -math.log(A))
        for x in xs:
            a, margin, near = orc.sample_action(psi, 1.0, int(x), 2.0 ** -12, 1e-6)
            assert a == R.uniform_row_action(int(x), A) == ((int(x) >> 8) * A) >> 24
            assert margin == 1.0 and not near
    # u |A| = 5 - 2^-23 for |A| = 6 lies just below the boundary at 5: the
    # exact draw is 4 (a single-precision product would round it up to 5).
    k = (5 * 2 ** 23 - 1) // 3
    x = k << 8
    assert ((x >> 8) * 6) >> 24 == 4
    assert orc.sample_action(np.zeros(6), 1.0, x)[0] == 4


def test_two_action_draw_closed_form(orc):
    # Psi = (0, ln 3 / eta): weights (1/3, 1), so action 0 is drawn exactly
    # when u < 1/4, i.e. x0 >> 8 < 2^22.  Draws next to that boundary are
    # near ties under the screen; draws far from it are not.
    for eta in (0.5, 1.0, 2.0):
        psi = np.array([0.0, math.log(3.0) / eta])
        for q, want in ((0, 0), (1, 0), (2 ** 22 - 1, 0), (2 ** 22 + 1, 1),
                        (2 ** 23, 1), (2 ** 24 - 1, 1)):
            a, margin, near = orc.sample_action(psi, eta, q << 8, 2.0 ** -12, 0.0)
            assert a == want
            assert near == (q in (2 ** 22 - 1, 2 ** 22 + 1))
            exact = abs(q / 2.0 ** 24 * 4.0 / 3.0 - 1.0 / 3.0) / (4.0 / 3.0)
            assert margin == pytest.approx(exact, rel=1e-9, abs=1e-15)


def test_softmax_draw_frequencies(orc):
    # Sampled frequencies follow softmax(eta psi) (chi-square, 4 df).
    psi = np.array([0.3, -1.0, 0.0, 0.7, -0.2])
    eta = 2.0
    p = np.exp(eta * (psi - psi.max()))
    p /= p.sum()
    rng = np.random.default_rng(5)
    n = 20000
    cnt = np.zeros(5)
    for x in rng.integers(0, 2 ** 32, size=n):
        cnt[orc.sample_action(psi, eta, int(x))[0]] += 1
    chi2 = (((cnt - n * p) ** 2) / (n * p)).sum()
    assert chi2 < 20.0          # p ~ 5e-4 for 4 degrees of freedom


# --- generative models --------------------------------------------------------

def test_nav_fp32_arithmetic_matches_independent_numpy(orc):
    inst = I.nav2d(3, 8, heuristic=1)
    ref = R.Nav(inst)
    rng = np.random.default_rng(11)
    for i in range(3000):
        x, y = rng.uniform(-0.5, 10.5, size=2).astype(np.float32)
        if i % 7 == 0:
            x, y = np.float32(9.0), np.float32(9.2)
        a = int(rng.integers(0, 4))
        w1, w2 = (int(v) for v in rng.integers(0, 2 ** 32, size=2))
        got = orc.nav_step(inst, x, y, a, w1, w2)
        (nx, ny), key, r, term = ref.step((x, y), a, (0, w1, w2, 0))
        assert got == (float(nx), float(ny), key, r, int(term))


def test_gauss_table_antisymmetric():
    g = I.gauss_quantile_table()
    assert g.dtype == np.float32 and g.size == 4096
    assert np.array_equal(g, -g[::-1])
    assert abs(float(g.astype(np.float64).mean())) == 0.0
    assert abs(float((g.astype(np.float64) ** 2).mean()) - 1.0) < 1e-3


# --- iteration-1 tree: independent replay -------------------------------------

def _compare_tree(res, rep):
    b = rep["b_rows"]
    a = rep["a_rows"]
    assert len(res.b_parent) == len(b)
    assert len(res.a_parent) == len(a)
    assert res.b_parent.tolist() == [r["parent"] for r in b]
    assert res.b_obs.tolist() == [r["obs"] for r in b]
    assert res.b_depth.tolist() == [r["depth"] for r in b]
    assert res.a_parent.tolist() == [r["parent"] for r in a]
    assert res.a_act.tolist() == [r["act"] for r in a]
    assert res.a_N.tolist() == [r["N"] for r in a]
    assert np.array_equal(res.a_C, np.array([r["C"] for r in a]))
    assert res.particle_steps == rep["steps"]


@pytest.mark.parametrize("depth", [1, 2, 4])
def test_first_iteration_tree_tabular(orc, depth):
    inst = I.tabular_dense(0, 16, 3, 4, with_heuristic=True)
    bel = I.tabular_belief(inst)
    res = orc.plan(inst, bel, 512, 1, depth, eta=1.0, seed=9, schedule=1, step=3)
    rep = R.replay_first(inst, bel, 512, depth, seed=9, step=3)
    _compare_tree(res, rep)
    # Leaf counts of this iteration.
    for bl, (c, _) in rep["leaves"].items():
        assert res.b_N[bl] == c


def test_first_iteration_tree_sparse(orc):
    inst = I.tabular_sparse(2, 64, 5, 7, 4, with_heuristic=True)
    bel = I.tabular_belief(inst)
    res = orc.plan(inst, bel, 700, 1, 3, eta=0.7, seed=2 ** 40 + 5, schedule=1)
    rep = R.replay_first(inst, bel, 700, 3, seed=2 ** 40 + 5)
    _compare_tree(res, rep)


def test_first_iteration_tree_nav(orc):
    inst = I.nav2d(1, 6, heuristic=1)
    # Start near the goal so that some episodes terminate.
    bx, by = I.nav_belief(4, 300, 7.5, 8.5)
    res = orc.plan(inst, (bx, by), 400, 1, 3, eta=1.0, seed=77, schedule=1)
    rep = R.replay_first(inst, (bx, by), 400, 3, seed=77)
    _compare_tree(res, rep)
    assert any(r["N"] > 0 for r in rep["a_rows"])
    n_leaf = sum(c for c, _ in rep["leaves"].values())
    assert n_leaf < 400   # some episodes reached the goal and were filtered


# --- one iteration of values: closed form on the replayed tree -----------------

@pytest.mark.parametrize("kind", ["tabular", "nav"])
def test_k1_values_match_backup_on_replay(orc, kind):
    if kind == "tabular":
        inst = I.tabular_dense(4, 16, 3, 4, with_heuristic=True)
        bel = I.tabular_belief(inst)
    else:
        inst = I.nav2d(2, 8, heuristic=1)
        bel = I.nav_belief(5, 500, 6.5, 8.5)
    eta = 1.3
    res = orc.plan(inst, bel, 600, 1, 3, eta=eta, seed=4, schedule=1)
    rep = R.replay_first(inst, bel, 600, 3, seed=4)
    psi, V, Nb = R.k1_values(rep, eta)
    np.testing.assert_allclose(res.psi, psi, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(res.b_V, V, rtol=1e-12, atol=1e-12)
    assert res.b_N.tolist() == Nb.tolist()


def test_depth1_closed_form(orc):
    # K = 1, depth 1: Psi(root, a) = Psi0 + C_a/N_a + gamma * mean_h(a) for each
    # sampled action, V = L_eta Psi (Eq. 3-5 with L_eta Psi0 = 0).
    inst = I.tabular_dense(6, 16, 4, 4, with_heuristic=True)
    bel = I.tabular_belief(inst)
    eta, n = 0.8, 2000
    res = orc.plan(inst, bel, n, 1, 1, eta=eta, seed=12)
    mdl = R.Tabular(inst)
    C = np.zeros(4)
    N = np.zeros(4)
    Hs = np.zeros(4)
    for ep in range(n):
        w = R.draw(12, ep, 1, 0, 1, 0)
        s = (w[0] * 16) >> 32
        w = R.draw(12, ep, 2, 0, 1, 0)
        a = min(((w[0] >> 8) * 4) >> 24, 3)     # root draw: exact
        sn, o, r, _ = mdl.step(s, a, w)
        C[a] += r
        N[a] += 1
        Hs[a] += mdl.h(sn)
    psi0 = -math.log(4) / eta
    want = np.where(N > 0, psi0 + C / np.maximum(N, 1) + inst["gamma"] * Hs / np.maximum(N, 1), psi0)
    np.testing.assert_allclose(res.psi_root, want, rtol=0, atol=1e-12)
    v = R.lse(want, eta)
    assert abs(res.v_root - v) < 1e-12
    # L_eta update identity: L(Psi_new) = (1/eta) log sum_a pi_old(a) e^{eta Q_a}.
    Q = want - psi0
    assert abs(res.v_root - math.log(np.mean(np.exp(eta * Q))) / eta) < 1e-12


# --- statistical pins: exact recursion, soft VI, expected-count limit --------

def _tiny(seed, nS=3, nA=2, nO=2, heur=True):
    return I.tabular_dense(seed, nS, nA, nO, gamma=0.9, with_heuristic=heur)


def _oracle_root(orc, inst, bel, n_p, K, depth, eta, schedule, seeds, mutate=0):
    vs, ps = [], []
    for sd in seeds:
        r = orc.plan(inst, bel, n_p, K, depth, eta=eta, seed=sd,
                     schedule=schedule, mutate=mutate)
        vs.append(r.v_root)
        ps.append(r.psi_root)
    return np.array(vs), np.array(ps)


def _within(samples, target, k=4.5, floor=2e-3):
    m = samples.mean(axis=0)
    se = samples.std(axis=0, ddof=1) / math.sqrt(samples.shape[0])
    return np.all(np.abs(m - target) <= k * se + floor), m, se


@pytest.mark.parametrize("seed,depth", [(0, 2), (1, 3)])
def test_k1_converges_to_reference_bellman(orc, seed, depth):
    inst = _tiny(seed)
    bel = I.tabular_belief(inst)
    b0 = R.root_probs(bel.size)
    eta = 1.5
    exact = R.ref_bellman(inst, b0, depth, eta)
    v, _ = _oracle_root(orc, inst, bel, 2 ** 15, 1, depth, eta, 1, range(1, 13))
    ok, m, se = _within(v, exact)
    assert ok, (m, exact, se)
    # A planted mistake (gamma dropped from Q) must be caught.
    vm, _ = _oracle_root(orc, inst, bel, 2 ** 15, 1, depth, eta, 1, range(1, 13),
                         mutate=1)
    assert not _within(vm, exact)[0]


def test_fully_observed_matches_soft_value_iteration(orc):
    inst = I.tabular_fully_observed(3, 3, 2, gamma=0.9)
    bel = I.tabular_belief(inst)
    b0 = R.root_probs(bel.size)
    eta = 2.0
    exact = R.soft_vi(inst, b0, 3, eta)
    assert abs(exact - R.ref_bellman(inst, b0, 3, eta)) < 1e-12
    v, _ = _oracle_root(orc, inst, bel, 2 ** 15, 1, 3, eta, 1, range(20, 32))
    ok, m, se = _within(v, exact)
    assert ok, (m, exact, se)


@pytest.mark.parametrize("K,depth,schedule", [(3, 3, 0), (3, 2, 1), (4, 2, 0)])
def test_iterations_converge_to_expected_count_limit(orc, K, depth, schedule):
    inst = _tiny(2)
    bel = I.tabular_belief(inst)
    b0 = R.root_probs(bel.size)
    eta = 1.0
    psi_f, v_f = R.fluid_plan(inst, b0, K, depth, eta, schedule)
    v, psi = _oracle_root(orc, inst, bel, 2 ** 15, K, depth, eta, schedule,
                          range(40, 52))
    ok_v, m, se = _within(v, v_f)
    ok_p, mp, sep = _within(psi, psi_f)
    assert ok_v, (m, v_f, se)
    assert ok_p, (mp, psi_f, sep)
    # A planted mistake (V_curr left out of the preference update) is caught.
    vm, psim = _oracle_root(orc, inst, bel, 2 ** 15, K, depth, eta, schedule,
                            range(40, 52), mutate=2)
    assert not (_within(vm, v_f)[0] and _within(psim, psi_f)[0])


# --- invariants ------------------------------------------------------------------

def _invariants(res, inst, n_p, K, depth, schedule, h_zero):
    A = inst["nA"]
    Ds = [depth if schedule == 1 else min(k, depth) for k in range(1, K + 1)]
    nb, na = len(res.b_parent), len(res.a_parent)
    assert nb <= 1 + n_p * sum(Ds) and na <= n_p * sum(Ds)
    root_acts = np.nonzero(res.a_parent == 0)[0]
    assert res.a_N[root_acts].sum() == K * n_p
    assert np.all(res.a_N >= 1)
    # Children visit counts never exceed the parent action's visits.
    kid = np.zeros(na, np.int64)
    np.add.at(kid, res.b_parent[1:], res.b_N[1:])
    assert np.all(kid <= res.a_N)
    # Each (belief, action) pair and each (action node, obs) pair is unique.
    assert len(set(zip(res.a_parent.tolist(), res.a_act.tolist()))) == na
    assert len(set(zip(res.b_parent[1:].tolist(), res.b_obs[1:].tolist()))) == nb - 1
    # Depth bookkeeping: a belief is one level below its parent action.
    adepth = res.b_depth[res.a_parent]
    assert np.all(res.b_depth[1:] == adepth[res.b_parent[1:]] + 1)
    # Softmax weights of every row sum to one.
    z = np.exp(res.psi - res.psi.max(axis=1, keepdims=True))
    assert np.allclose((z / z.sum(axis=1, keepdims=True)).sum(axis=1), 1.0, atol=1e-12)
    if h_zero:
        g = inst["gamma"]
        rmax = float(np.max(np.abs(inst["reward"]))) if inst["kind"] == "tabular" else 201.0
        rem = depth - res.b_depth
        bound = rmax * (1 - g ** rem) / (1 - g)
        assert np.all(np.abs(res.b_V) <= bound + 1e-9)
        assert np.all(np.abs(res.b_V) <= rmax / (1 - g) + 1e-9)


@pytest.mark.parametrize("seed", range(1, 5))
def test_invariants_tabular16(orc, seed):
    inst, bel, p = I.workload("tabular16", seed=0)
    for schedule in (0, 1):
        res = orc.plan(inst, bel, p["n_particles"], p["budget"], p["depth"],
                       eta=1.0, seed=seed, schedule=schedule)
        _invariants(res, inst, p["n_particles"], p["budget"], p["depth"],
                    schedule, True)


def test_invariants_nav_and_sparse(orc):
    inst = I.nav2d(0, 8)
    bel = I.nav_belief(1, 4096)
    res = orc.plan(inst, bel, 2048, 5, 5, eta=1.0, seed=3)
    _invariants(res, inst, 2048, 5, 5, 0, True)
    inst = I.tabular_sparse(0, 256, 8, 32, 8)
    bel = I.tabular_belief(inst)
    res = orc.plan(inst, bel, 4096, 6, 6, eta=1.0, seed=3)
    _invariants(res, inst, 4096, 6, 6, 0, True)
