"""Oracle pins at MARS-sized action sets (|A| = 625 and 3025, Sec. IV): the
draw of Eq. (6) over thousands of actions (flat rows in closed form, other
rows by frequency), the depth-1 closed form of Eq. (3)-(5), and the tree
invariants of a deeper plan.
"""

import numpy as np
import pytest
from scipy import stats

from paper_2510_27191_amd import instances as I
from tests import refimpl as R


@pytest.mark.parametrize("A", [625, 3025])
def test_flat_row_draw(orc, A):
    # Every weight is exp(0) = 1, the running sums are the integers 1..A, and
    # the draw is floor(u * A) with u = (x0 >> 8) / 2^24.
    rng = np.random.default_rng(A)
    eta = 1.0
    row = np.full(A, -np.log(A) / eta)
    for x0 in rng.integers(0, 2 ** 32, size=4000, dtype=np.uint64):
        x0 = int(x0)
        want = ((x0 >> 8) * A) >> 24
        a, margin, near = orc.sample_action(row, eta, x0, 2.0 ** -12, 1e-4)
        assert a == want and margin == 1.0 and not near


def test_long_row_exact_draw(orc):
    # A hand-made long row: two actions hold all but exp(-40) of the mass
    # each; the other 98 weigh exp(-40) ~ 4e-18.  By Eq. (6), t = u * P_last
    # with P_last = 2 + 98 e^-40, so any u >= 2^-24 below 1/2 draws 17 and any
    # u above 1/2 draws 63.  u = 0 gives t = 0 < P_0 = e^-40: action 0, a draw
    # that sits on a boundary and is screened as a near tie.
    A, eta = 100, 1.0
    row = np.full(A, -40.0)
    row[17] = row[63] = 0.0
    for q in (1, 2, 2 ** 22, 2 ** 23 - 1, 2 ** 23 + 1, 2 ** 24 - 1):
        a, _, near = orc.sample_action(row, eta, q << 8, 2.0 ** -12, 1e-5)
        assert a == (17 if q < 2 ** 23 else 63)
        # (u near 0 or 1 lies next to the boundaries that the light actions
        # pile up at 0 and P_last: near ties as well)
        if q in (2 ** 22, 2 ** 23 - 1, 2 ** 23 + 1):
            assert near == (q != 2 ** 22)
    a, _, near = orc.sample_action(row, eta, 0, 2.0 ** -12, 1e-5)
    assert a == 0 and near


def test_softmax_draw_frequencies_625(orc):
    rng = np.random.default_rng(9)
    A, eta, n = 625, 1.0, 120000
    row = rng.normal(0.0, 1.5, size=A)
    p = np.exp(eta * (row - row.max()))
    p /= p.sum()
    counts = np.zeros(A)
    for x0 in rng.integers(0, 2 ** 32, size=n, dtype=np.uint64):
        counts[orc.sample_action(row, eta, int(x0))[0]] += 1
    # Bins: the 40 likeliest actions one by one, the rest pooled.
    order = np.argsort(-p)
    top = order[:40]
    obs = np.append(counts[top], counts[order[40:]].sum())
    exp = np.append(p[top], p[order[40:]].sum()) * n
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, df=len(obs) - 1) > 1e-4


def test_depth1_closed_form_625(orc):
    # K = 1, depth 1, flat root row: Psi(root, a) = Psi0 + C_a/N_a for each
    # sampled action (zero heuristic), V = L_eta Psi.
    inst = I.mars_like(4, 64, 625)
    bel = I.tabular_belief(inst)
    A, eta, n = 625, 0.7, 3000
    res = orc.plan(inst, bel, n, 1, 1, eta=eta, seed=5)
    mdl = R.Tabular(inst)
    C = np.zeros(A)
    N = np.zeros(A)
    for ep in range(n):
        w = R.draw(5, ep, 1, 0, 1, 0)
        s = (w[0] * 64) >> 32
        w = R.draw(5, ep, 2, 0, 1, 0)
        a = min(((w[0] >> 8) * A) >> 24, A - 1)
        _, _, r, _ = mdl.step(s, a, w)
        C[a] += r
        N[a] += 1
    psi = np.full(A, -np.log(A) / eta)
    vis = N > 0
    psi[vis] += C[vis] / N[vis]
    np.testing.assert_allclose(res.psi_root, psi, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(res.v_root, R.lse(psi, eta), rtol=1e-12, atol=1e-12)
    assert sorted(res.a_act[res.a_parent == 0].tolist()) == np.nonzero(vis)[0].tolist()


def test_tree_invariants_3025(orc):
    inst = I.mars_like(6, 128, 3025)
    bel = I.tabular_belief(inst)
    n_p, K, depth = 600, 3, 3
    res = orc.plan(inst, bel, n_p, K, depth, seed=2)
    root = res.a_parent == 0
    assert res.a_N[root].sum() == K * n_p
    key = res.a_parent.astype(np.int64) * 4096 + res.a_act
    assert np.unique(key).size == key.size
    kid = np.zeros(len(res.a_parent), np.int64)
    np.add.at(kid, res.b_parent[1:], res.b_N[1:])
    assert np.all(kid <= res.a_N)
    # Non-sensing actions observe NULL only.
    sense = (res.a_act % 25) >= 20
    obs_of = np.zeros(len(res.a_parent), np.int64)
    np.maximum.at(obs_of, res.b_parent[1:], res.b_obs[1:])
    assert np.all(obs_of[~sense] == 0)
    vmax = 10.0 / (1.0 - inst["gamma"])
    assert np.all(np.abs(res.psi_root) < vmax + np.log(3025))
