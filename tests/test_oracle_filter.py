"""Pins of the oracle's true-environment step and SIR belief update."""

import math

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests import refimpl as R


def deterministic_instance():
    """T(s, a) = (s + a + 1) mod 4 with certainty; Z(s', a, o) = [o == s']."""
    nS, nA = 4, 2
    rowptr = np.arange(nS * nA + 1, dtype=np.int32)
    col = np.array([(s + a + 1) % nS for s in range(nS) for a in range(nA)], np.int32)
    tprob = np.ones(nS * nA, np.float32)
    Z = np.zeros((nS, nA, nS), np.float32)
    for s in range(nS):
        Z[s, :, s] = 1.0
    return dict(kind="tabular", nS=nS, nA=nA, nO=nS, rowptr=rowptr, col=col,
                tprob=tprob, zprob=Z.reshape(-1), reward=np.zeros(nS * nA, np.float32),
                heur=None, gamma=0.9)


def test_deterministic_model_gives_known_posterior(orc):
    inst = deterministic_instance()
    parts = np.array([0, 1, 2, 3] * 50, np.int32)
    new, tot = orc.belief_update(inst, parts, 1, 3, seed=5, step=2)
    # Only particles that moved to state 3 (from state 1 under a = 1) explain o = 3.
    assert np.all(new == 3)
    assert tot == 50 * 2 ** 31
    # An observation no particle can explain: weights all zero, moved set kept.
    parts = np.array([0] * 10, np.int32)
    new, tot = orc.belief_update(inst, parts, 0, 3, seed=5, step=2)
    assert tot == 0 and np.all(new == 1)


def test_matches_independent_replay(orc):
    inst = I.tabular_dense(3, 6, 3, 4)
    parts = np.arange(40, dtype=np.int32) % 6
    new, tot = orc.belief_update(inst, parts, 2, 1, seed=2 ** 35 + 9, step=7)
    ref, rtot = R.pf_update(inst, list(parts), 2, 1, 2 ** 35 + 9, 7)
    assert tot == rtot and new.tolist() == ref
    nav = I.nav2d(1, 6)
    bx, by = I.nav_belief(2, 30, 3.0, 5.0)
    s, obs, _, _ = orc.env_step(nav, (float(bx[0]), float(by[0])), 1, seed=4, step=0)
    (nx, ny), tot = orc.belief_update(nav, (bx, by), 1, obs, seed=11, step=3)
    ref, rtot = R.pf_update(nav, [(np.float32(a), np.float32(b)) for a, b in zip(bx, by)],
                            1, obs, 11, 3)
    assert tot == rtot > 0
    assert nx.tolist() == [float(p[0]) for p in ref]
    assert ny.tolist() == [float(p[1]) for p in ref]


def test_posterior_matches_bayes_filter(orc):
    # Frequencies of the resampled particles follow the exact Bayes posterior
    # b'(s') ~ sum_s b(s) T(s, a, s') Z(s', a, o)  (chi-square, 5 dof).
    inst = I.tabular_dense(8, 6, 2, 3)
    mdl = R.Tabular(inst)
    b0 = np.full(6, 1 / 6)
    a, o = 1, 2
    post = (b0 @ mdl.T[:, a, :]) * mdl.Zp[:, a, o]
    post /= post.sum()
    n = 60000
    parts = np.arange(n, dtype=np.int32) % 6
    new, tot = orc.belief_update(inst, parts, a, o, seed=3, step=1)
    cnt = np.bincount(new, minlength=6).astype(np.float64)
    m = post > 0
    chi2 = (((cnt[m] - n * post[m]) ** 2) / (n * post[m])).sum()
    assert chi2 < 30.0, (cnt / n, post)
    assert cnt[~m].sum() == 0


def test_env_step_is_the_model_on_its_own_stream(orc):
    inst = I.tabular_dense(2, 10, 3, 4)
    s = 4
    for t in range(5):
        s2, obs, r, term = orc.env_step(inst, s, t % 3, seed=77, step=t)
        ref = R.env_step(inst, s, t % 3, 77, t)
        assert (s2, obs, r, bool(term)) == (ref[0], ref[1], ref[2], ref[3])
        s = s2
    nav = I.nav2d(3, 8)
    st = (1.0, 1.0)
    for t in range(5):
        st2, obs, r, term = orc.env_step(nav, st, t % 4, seed=5, step=t)
        (nx, ny), o2, r2, term2 = R.env_step(nav, (np.float32(st[0]), np.float32(st[1])),
                                             t % 4, 5, t)
        assert st2 == (float(nx), float(ny)) and obs == o2 and r == r2
        st = st2


def test_nav_cell_counts_cover_the_table():
    # For any position, the cell counts over all cells sum to 4096 per axis.
    nav = I.nav2d(0, 4)
    mdl = R.Nav(nav)
    f = np.float32
    for v in (f(0.3), f(5.0), f(9.7)):
        sd = f(0.05) + f(0.5) * abs(f(v - f(5.0)))
        cells = {}
        for j in range(4096):
            k = mdl._axis(f(v + f(sd * mdl.g[j])))
            cells[k] = cells.get(k, 0) + 1
        assert sum(cells.values()) == 4096
        for k, c in list(cells.items())[:3]:
            assert R.nav_cell_count(mdl, v, sd, k) == c
