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


# --- navigation likelihood (the SIR weight of the navigation model) -----------

def test_nav_likelihood_sums_to_one_over_cells(orc):
    # Every (x-noise, y-noise) index pair of the observation lands in exactly
    # one grid cell, so the likelihood counts over all cells sum to 4096^2 at
    # any position: near the clamped border of the grid too.
    nav = I.nav2d(0, 4)
    small = dict(nav, key_lo=2, key_n=12)       # cells [1, 7) per axis, clamped
    for inst, pos in ((nav, (5.0, 5.0)), (small, (0.3, 9.7)), (small, (6.0, 3.2))):
        n = inst["key_n"]
        tot = sum(orc.nav_obs_weight(inst, pos[0], pos[1], o) for o in range(n * n))
        assert tot == 4096 * 4096


def _axis_cells(inst, v):
    """Grid cell per axis of fp32 values v (floor, clamp), as the model keys
    its observations."""
    f = np.float32
    c = np.floor(v * f(inst["inv_bin"])).astype(np.float32)
    c = np.clip(c, f(inst["key_lo"]), f(inst["key_lo"] + inst["key_n"] - 1))
    return c.astype(np.int64) - inst["key_lo"]


def _posterior_one_axis(inst, pos, a, o):
    """Bayes posterior of the moved position along the axis that moves freely,
    for a particle at pos pushed into a wall by action a (so the other axis is
    clamped to the wall whatever its noise): enumerate the 4096 motion-noise
    values of the free axis and, for each, the 4096 x 4096 observation-noise
    pairs, as the model draws them (fp32 throughout)."""
    f = np.float32
    g = np.asarray(inst["gauss"], np.float32)
    lo, hi = f(inst["lo"]), f(inst["hi"])
    sm = f(inst["sigma_move"])
    step = f(inst["step"])
    x0, y0 = f(pos[0]), f(pos[1])
    dx = {0: f(0), 1: step, 2: f(0), 3: -step}[a]
    dy = {0: step, 1: f(0), 2: -step, 3: f(0)}[a]
    nx = np.clip((x0 + dx) + sm * g, lo, hi).astype(np.float32)   # x-noise index i
    ny = np.clip((y0 + dy) + sm * g, lo, hi).astype(np.float32)   # y-noise index i'
    free_x = a in (0, 2)
    if free_x:
        assert np.all(ny == ny[0])
        xs, ys = nx, np.full(4096, ny[0], np.float32)
    else:
        assert np.all(nx == nx[0])
        xs, ys = np.full(4096, nx[0], np.float32), ny
    sd = (f(inst["sigma_obs0"]) +
          f(inst["sigma_obs_slope"]) * np.abs(xs - f(inst["obs_center_x"]))).astype(np.float32)
    kn = inst["key_n"]
    kx, ky = o // kn, o % kn
    like = np.zeros(4096)
    for i in range(4096):
        ox = (xs[i] + (sd[i] * g).astype(np.float32)).astype(np.float32)
        oy = (ys[i] + (sd[i] * g).astype(np.float32)).astype(np.float32)
        like[i] = (np.count_nonzero(_axis_cells(inst, ox) == kx) *
                   np.count_nonzero(_axis_cells(inst, oy) == ky))
    return (xs if free_x else ys), like / like.sum()


@pytest.mark.parametrize("pos,a", [((4.3, 10.0), 0), ((10.0, 6.1), 1)])
def test_nav_resampling_follows_bayes_posterior(orc, pos, a):
    # Particles at one position pushed into a wall: the moved position varies
    # along one axis only, and its posterior given the observation is the
    # prior over the 4096 motion-noise values times the likelihood of the
    # observed cell, enumerated over the observation noise.  One resampled
    # particle per filter run (independent runs by seed) must follow it
    # (chi-square over 8 equal-mass bins; self-normalised weights over n = 48
    # particles bias each bin by about 1/n of its mass, below the test's
    # resolution).
    inst = I.nav2d(1, 4)
    n, runs = 48, 1500
    free, post = None, None
    # The observation: the cell of the unperturbed move.
    f = np.float32
    tgt = (f(min(max(pos[0] + (1.0 if a == 1 else -1.0 if a == 3 else 0.0), 0.0), 10.0)),
           f(min(max(pos[1] + (1.0 if a == 0 else -1.0 if a == 2 else 0.0), 0.0), 10.0)))
    o = int(_axis_cells(inst, np.array([tgt[0]], np.float32))[0] * inst["key_n"] +
            _axis_cells(inst, np.array([tgt[1]], np.float32))[0])
    free, post = _posterior_one_axis(inst, pos, a, o)
    # Bin edges at the posterior's octiles over the sorted values.
    order = np.argsort(free, kind="stable")
    cdf = np.cumsum(post[order])
    edges = [free[order][np.searchsorted(cdf, q)] for q in np.arange(1, 8) / 8]
    def bin_of(v):
        return int(np.searchsorted(np.asarray(edges, np.float32), np.float32(v), side="right"))
    mass = np.zeros(8)
    for v, p in zip(free, post):
        mass[bin_of(v)] += p
    cnt = np.zeros(8)
    bx = np.full(n, pos[0], np.float32)
    by = np.full(n, pos[1], np.float32)
    for r in range(runs):
        (nx, ny), tot = orc.belief_update(inst, (bx, by), a, o, seed=1000 + r, step=r % 7)
        assert tot > 0
        cnt[bin_of(nx[0] if a in (0, 2) else ny[0])] += 1
    m = mass > 0
    chi2 = (((cnt[m] - runs * mass[m]) ** 2) / (runs * mass[m])).sum()
    from scipy import stats
    assert stats.chi2.sf(chi2, df=int(m.sum()) - 1) > 1e-4, (cnt, runs * mass)
