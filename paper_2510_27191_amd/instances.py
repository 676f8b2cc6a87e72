"""Seeded synthetic POMDP instances and belief particle sets.

This module only draws random numbers and lays them out as arrays.  It holds
none of the planner's arithmetic (no thresholds, no sampling rules, no
values), so both the GPU path and the serial CPU oracle can take their inputs
from it.

Instance families (the workloads the planner is measured on):

* ``tabular_dense``  - a small random tabular POMDP: every transition row
  T[s, a, :] and observation row Z[s', a, :] is a Dirichlet(0.5) draw,
  rewards R[s, a] ~ U[-1, 1] (fp32).  Transitions are stored in CSR form with
  every state listed as a successor.
* ``tabular_sparse`` - a large sparse tabular POMDP: each (s, a) has
  ``n_succ`` distinct successors with Dirichlet(0.5) weights (CSR, int32
  columns / fp32 weights), dense Dirichlet(0.5) observation rows.
* ``nav2d``          - a continuous 2-D navigation POMDP on [0, 10]^2 with four
  unit moves, Gaussian motion noise, position observations whose noise grows
  away from x = 5 and are binned on a 0.5 grid to form tree keys, a goal disk
  and seed-placed obstacle disks.

The paper represents continuous spaces by a fixed finite set chosen a priori
(Sec. III-B); here the Gaussian noise is a fixed 4096-entry quantile table that
is part of the instance, and observations are keyed by their grid cell.

Array conventions (shared by every consumer):

tabular dict: ``kind='tabular'``, ``nS, nA, nO`` ints, ``rowptr`` int32
[nS*nA+1], ``col`` int32 [nnz] (successor states, ascending inside a row),
``tprob`` float32 [nnz], ``zprob`` float32 [nS*nA*nO] indexed [s'][a][o],
``reward`` float32 [nS*nA] indexed [s][a], ``heur`` float32 [nS] or None,
``gamma`` float.

nav dict: ``kind='nav'`` plus the scalar fields listed in ``NAV_FIELDS``,
``disks`` float32 [n, 2] (centres), ``gauss`` float32 [4096].
"""

from __future__ import annotations

import math

import numpy as np

NAV_FIELDS = (
    "lo", "hi", "step", "sigma_move", "sigma_obs0", "sigma_obs_slope",
    "obs_center_x", "inv_bin", "key_lo", "key_n", "goal_x", "goal_y",
    "goal_r2", "disk_r2", "r_step", "r_goal", "r_hit", "heuristic", "gamma",
)

GAUSS_TABLE_SIZE = 4096


def gauss_quantile_table(n: int = GAUSS_TABLE_SIZE) -> np.ndarray:
    """Standard-normal quantiles at the cell centres (j + 0.5) / n, fp32.

    A uniform 12-bit index into this table is a discretised N(0, 1) draw.
    The table is antisymmetric (entry j = -entry n-1-j), so its mean is 0.
    """
    from scipy.special import ndtri

    q = ndtri((np.arange(n, dtype=np.float64) + 0.5) / n)
    half = q[n // 2:].astype(np.float32)
    # Enforce exact antisymmetry in fp32.
    return np.concatenate([-half[::-1], half]).astype(np.float32)


def tabular_dense(seed: int, nS: int = 16, nA: int = 3, nO: int = 4,
                  gamma: float = 0.95, alpha: float = 0.5,
                  with_heuristic: bool = False) -> dict:
    """Random dense tabular POMDP (T, Z rows ~ Dirichlet(alpha), R ~ U[-1,1])."""
    rng = np.random.default_rng(seed)
    T = rng.dirichlet(alpha * np.ones(nS), size=(nS, nA)).astype(np.float32)
    Z = rng.dirichlet(alpha * np.ones(nO), size=(nS, nA)).astype(np.float32)
    R = rng.uniform(-1.0, 1.0, size=(nS, nA)).astype(np.float32)
    heur = (rng.uniform(-1.0, 1.0, size=nS).astype(np.float32)
            if with_heuristic else None)
    rowptr = (np.arange(nS * nA + 1, dtype=np.int64) * nS).astype(np.int32)
    col = np.tile(np.arange(nS, dtype=np.int32), nS * nA)
    return dict(kind="tabular", nS=nS, nA=nA, nO=nO, rowptr=rowptr, col=col,
                tprob=T.reshape(-1).copy(), zprob=Z.reshape(-1).copy(),
                reward=R.reshape(-1).copy(), heur=heur, gamma=float(gamma))


def tabular_sparse(seed: int, nS: int = 4096, nA: int = 8, nO: int = 32,
                   n_succ: int = 8, gamma: float = 0.95, alpha: float = 0.5,
                   with_heuristic: bool = False) -> dict:
    """Random sparse tabular POMDP: ``n_succ`` distinct successors per (s, a)."""
    rng = np.random.default_rng(seed)
    k = min(n_succ, nS)
    rows = nS * nA
    col = _distinct_rows(rng, rows, nS, k)
    tp = rng.dirichlet(alpha * np.ones(k), size=rows).astype(np.float32)
    Z = rng.dirichlet(alpha * np.ones(nO), size=(nS, nA)).astype(np.float32)
    R = rng.uniform(-1.0, 1.0, size=(nS, nA)).astype(np.float32)
    heur = (rng.uniform(-1.0, 1.0, size=nS).astype(np.float32)
            if with_heuristic else None)
    rowptr = (np.arange(rows + 1, dtype=np.int64) * k).astype(np.int32)
    return dict(kind="tabular", nS=nS, nA=nA, nO=nO, rowptr=rowptr,
                col=col.reshape(-1).copy(), tprob=tp.reshape(-1).copy(),
                zprob=Z.reshape(-1).copy(), reward=R.reshape(-1).copy(),
                heur=heur, gamma=float(gamma))


def mars_like(seed: int, nS: int = 2048, nA: int = 625, nO: int = 9, n_succ: int = 4,
              gamma: float = 0.983, alpha: float = 0.5, reward_scale: float = 1.0) -> dict:
    """Synthetic tabular POMDP shaped like Multi-Agent RockSample: |A| = (5+m)^2
    joint actions (625 for m = 20, 3025 for m = 50), |O| = 9 with a NULL
    observation 0, gamma = 0.983.

    Each (s, a) has ``n_succ`` successors with Dirichlet(alpha) weights.  One
    action in five of each block of 25 senses: its observation row is
    Dirichlet(alpha) over the 9 observations; every other action observes NULL.
    Rewards are -0.1 per step, and +-10 (either sign) for 2% of the (s, a)
    pairs, like sampling a good or a bad rock; ``reward_scale`` multiplies both.
    """
    rng = np.random.default_rng(seed)
    k = min(n_succ, nS)
    rows = nS * nA
    col = _distinct_rows(rng, rows, nS, k)
    tp = rng.dirichlet(alpha * np.ones(k), size=rows).astype(np.float32)
    Z = np.zeros((nS, nA, nO), np.float32)
    Z[:, :, 0] = 1.0
    sense = np.nonzero(np.arange(nA) % 25 >= 20)[0]
    Z[:, sense, :] = rng.dirichlet(alpha * np.ones(nO), size=(nS, sense.size)).astype(np.float32)
    R = np.full((nS, nA), -0.1, np.float32)
    hit = rng.random((nS, nA)) < 0.02
    R[hit] = np.where(rng.random(int(hit.sum())) < 0.5, 10.0, -10.0).astype(np.float32)
    R = (R * np.float32(reward_scale)).astype(np.float32)
    rowptr = (np.arange(rows + 1, dtype=np.int64) * k).astype(np.int32)
    return dict(kind="tabular", nS=nS, nA=nA, nO=nO, rowptr=rowptr,
                col=col.reshape(-1).copy(), tprob=tp.reshape(-1).copy(),
                zprob=Z.reshape(-1).copy(), reward=R.reshape(-1).copy(),
                heur=None, gamma=float(gamma))


def _distinct_rows(rng, rows: int, n: int, k: int) -> np.ndarray:
    """rows x k distinct integers from [0, n) per row, sorted; uniform over
    k-subsets (rows with a repeated value are drawn again)."""
    if k == n:
        return np.tile(np.arange(n, dtype=np.int32), (rows, 1))
    out = np.sort(rng.integers(0, n, size=(rows, k)), axis=1)
    bad = np.nonzero((np.diff(out, axis=1) == 0).any(axis=1))[0]
    while bad.size:
        redo = np.sort(rng.integers(0, n, size=(bad.size, k)), axis=1)
        out[bad] = redo
        ok = ~(np.diff(redo, axis=1) == 0).any(axis=1)
        bad = bad[~ok]
    return out.astype(np.int32)


def nav2d(seed: int, n_disks: int = 8, gamma: float = 0.95,
          heuristic: int = 0) -> dict:
    """2-D navigation POMDP with ``n_disks`` seed-placed radius-1 obstacles.

    Obstacle centres are uniform in [1, 9]^2, rejected when closer than 2 to
    the goal (9, 9) or to the start corner (1, 1).
    """
    rng = np.random.default_rng(seed)
    centres = []
    while len(centres) < n_disks:
        c = rng.uniform(1.0, 9.0, size=2)
        if math.hypot(c[0] - 9.0, c[1] - 9.0) < 2.0:
            continue
        if math.hypot(c[0] - 1.0, c[1] - 1.0) < 2.0:
            continue
        centres.append(c)
    disks = np.asarray(centres, dtype=np.float32).reshape(-1, 2)
    return dict(kind="nav", lo=0.0, hi=10.0, step=1.0, sigma_move=0.1,
                sigma_obs0=0.05, sigma_obs_slope=0.5, obs_center_x=5.0,
                inv_bin=2.0, key_lo=-32, key_n=128, goal_x=9.0, goal_y=9.0,
                goal_r2=0.25, disk_r2=1.0, r_step=-1.0, r_goal=100.0,
                r_hit=-100.0, heuristic=int(heuristic), gamma=float(gamma),
                disks=disks, gauss=gauss_quantile_table(), nA=4)


def tabular_belief(inst: dict) -> np.ndarray:
    """One particle per state: the uniform belief over S."""
    return np.arange(inst["nS"], dtype=np.int32)


def nav_belief(seed: int, n: int, lo: float = 0.5, hi: float = 1.5):
    """``n`` particles with x, y ~ U[lo, hi] (fp32), returned as (x, y)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=n).astype(np.float32)
    y = rng.uniform(lo, hi, size=n).astype(np.float32)
    return x, y


def tabular_fully_observed(seed: int, nS: int = 3, nA: int = 2,
                           gamma: float = 0.9) -> dict:
    """A tabular POMDP whose observation is the next state (Z = identity)."""
    inst = tabular_dense(seed, nS=nS, nA=nA, nO=nS, gamma=gamma,
                         with_heuristic=True)
    Z = np.zeros((nS, nA, nS), dtype=np.float32)
    for s in range(nS):
        Z[s, :, s] = 1.0
    inst["zprob"] = Z.reshape(-1).copy()
    return inst


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------

def workload(name: str, seed: int = 0):
    """Return (instance, belief, plan dict) for a named workload.

    ``plan`` carries n_particles, budget (iterations), depth, eta.
    """
    if name == "tabular16":          # |S|=16 |A|=3 |O|=4, n_p=1024, depth 4
        inst = tabular_dense(seed, 16, 3, 4)
        return inst, tabular_belief(inst), dict(n_particles=1024, budget=4,
                                                depth=4, eta=1.0)
    if name == "nav2d":              # n_p=2^16, depth 10
        inst = nav2d(seed, 8)
        return inst, nav_belief(seed + 1000, 65536), dict(
            n_particles=65536, budget=10, depth=10, eta=1.0)
    if name == "mars625":            # |S|=2048 |A|=625 |O|=9, n_p=2^14, depth 4
        inst = mars_like(seed, 2048, 625)
        return inst, tabular_belief(inst), dict(n_particles=16384, budget=4,
                                                depth=4, eta=1.0)
    if name == "mars3025":           # |S|=512 |A|=3025 |O|=9, n_p=2^14, depth 4
        inst = mars_like(seed, 512, 3025)
        return inst, tabular_belief(inst), dict(n_particles=16384, budget=4,
                                                depth=4, eta=1.0)
    if name == "sparse4096":         # |S|=4096 |A|=8 |O|=32, n_p=2^18, depth 8
        inst = tabular_sparse(seed, 4096, 8, 32, 8)
        return inst, tabular_belief(inst), dict(n_particles=262144, budget=8,
                                                depth=8, eta=1.0)
    raise KeyError(name)


def batch_mix(seed: int = 0, n: int = 256, max_np_log2: float = 16.0):
    """The mixed batch: alternating tabular and navigation instances.

    Tabular: |S| log-uniform in [64, 4096], |A| in {3..8}, |O| in {4..32},
    min(8, |S|) successors per (s, a).  Navigation: 4..16 obstacles.
    Depth uniform in {4..12}, budget = depth, n_p = round(2^U[10, 16]).
    Returns a list of (instance, belief, plan) triples.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        depth = int(rng.integers(4, 13))
        n_p = int(round(2.0 ** rng.uniform(10.0, max_np_log2)))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        if i % 2 == 0:
            nS = int(round(math.exp(rng.uniform(math.log(64), math.log(4096)))))
            nA = int(rng.integers(3, 9))
            nO = int(rng.integers(4, 33))
            inst = tabular_sparse(sub, nS, nA, nO, min(8, nS))
            bel = tabular_belief(inst)
        else:
            inst = nav2d(sub, int(rng.integers(4, 17)))
            bel = nav_belief(sub + 1, n_p)
        out.append((inst, bel, dict(n_particles=n_p, budget=depth,
                                    depth=depth, eta=1.0, seed=sub)))
    return out
