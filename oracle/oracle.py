"""ctypes wrapper around the serial CPU oracle (``vopp_oracle.cpp``).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  The product path
never does.

``build()`` compiles ``liboracle.so`` with g++ (-O2, contraction off, so every
double and single precision operation rounds once); ``load()`` loads it,
building it first only when no library exists yet.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vopp_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build() -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", LIB + ".tmp", SRC]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class OrcTabular(C.Structure):
    _fields_ = [("nS", C.c_int32), ("nA", C.c_int32), ("nO", C.c_int32),
                ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("tprob", C.c_void_p), ("zprob", C.c_void_p),
                ("reward", C.c_void_p), ("heur", C.c_void_p),
                ("gamma", C.c_double)]


class OrcNav(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "lo", "hi", "step", "sigma_move", "sigma_obs0", "sigma_obs_slope",
        "obs_center_x", "inv_bin")] + [
        ("key_lo", C.c_int32), ("key_n", C.c_int32)] + [
        (n, C.c_float) for n in ("goal_x", "goal_y", "goal_r2", "disk_r2",
                                 "r_step", "r_goal", "r_hit")] + [
        ("heuristic", C.c_int32), ("n_disks", C.c_int32),
        ("disks", C.c_void_p), ("gauss", C.c_void_p), ("gamma", C.c_double)]


class OrcParams(C.Structure):
    _fields_ = [("n_particles", C.c_int32), ("budget", C.c_int32),
                ("depth", C.c_int32), ("schedule", C.c_int32),
                ("eta", C.c_double), ("seed", C.c_uint64),
                ("step", C.c_uint32), ("tau", C.c_double),
                ("tau_abs", C.c_double), ("tau_psi", C.c_double),
                ("trace", C.c_int32), ("mutate", C.c_int32),
                ("pi0", C.c_void_p), ("start", C.c_void_p)]


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    vp = C.c_void_p
    lib.orc_plan_tabular.restype = vp
    lib.orc_plan_tabular.argtypes = [C.POINTER(OrcTabular), vp, C.c_int32,
                                     C.POINTER(OrcParams)]
    lib.orc_plan_nav.restype = vp
    lib.orc_plan_nav.argtypes = [C.POINTER(OrcNav), vp, vp, C.c_int32,
                                 C.POINTER(OrcParams)]
    lib.orc_result_info.argtypes = [vp, vp, vp, vp]
    lib.orc_result_tree.argtypes = [vp] * 11
    lib.orc_result_trace.argtypes = [vp] * 4
    lib.orc_result_draws.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
    lib.orc_nav_obs_weight.argtypes = [C.POINTER(OrcNav), C.c_float, C.c_float, C.c_int32]
    lib.orc_nav_obs_weight.restype = C.c_uint64
    lib.orc_result_free.argtypes = [vp]
    lib.orc_reroot.restype = vp
    lib.orc_reroot.argtypes = [vp, C.c_int32, C.c_int32]
    lib.orc_philox.argtypes = [C.c_uint32] * 6 + [vp]
    lib.orc_thresholds.argtypes = [vp, C.c_int32, vp]
    lib.orc_pick.argtypes = [vp, C.c_int32, C.c_uint32]
    lib.orc_pick.restype = C.c_int32
    lib.orc_sample_action.argtypes = [vp, C.c_int32, C.c_double, C.c_uint32,
                                      C.c_double, C.c_double, C.c_double, vp, vp]
    lib.orc_sample_action.restype = C.c_int32
    lib.orc_nav_step.argtypes = [C.POINTER(OrcNav), C.c_float, C.c_float,
                                 C.c_int32, C.c_uint32, C.c_uint32] + [vp] * 5
    lib.orc_env_step_tabular.argtypes = [C.POINTER(OrcTabular), vp, C.c_int32,
                                         C.c_uint64, C.c_uint32, vp, vp, vp]
    lib.orc_env_step_nav.argtypes = [C.POINTER(OrcNav), vp, vp, C.c_int32,
                                     C.c_uint64, C.c_uint32, vp, vp, vp]
    lib.orc_pf_update_tabular.argtypes = [C.POINTER(OrcTabular), vp, C.c_int32,
                                          C.c_int32, C.c_int32, C.c_uint64, C.c_uint32]
    lib.orc_pf_update_tabular.restype = C.c_uint64
    lib.orc_pf_update_nav.argtypes = [C.POINTER(OrcNav), vp, vp, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_uint64, C.c_uint32]
    lib.orc_pf_update_nav.restype = C.c_uint64
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c32(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class _Keep:
    """Holds numpy arrays alive while a ctypes struct points at them."""

    def __init__(self):
        self.arrs = []

    def __call__(self, a, dt):
        if a is None:
            return None
        a = _c32(a, dt)
        self.arrs.append(a)
        return _ptr(a)


def tabular_struct(inst, keep):
    return OrcTabular(inst["nS"], inst["nA"], inst["nO"],
                      keep(inst["rowptr"], np.int32), keep(inst["col"], np.int32),
                      keep(inst["tprob"], np.float32),
                      keep(inst["zprob"], np.float32),
                      keep(inst["reward"], np.float32),
                      keep(inst.get("heur"), np.float32), inst["gamma"])


def nav_struct(inst, keep):
    disks = _c32(inst["disks"], np.float32).reshape(-1)
    return OrcNav(inst["lo"], inst["hi"], inst["step"], inst["sigma_move"],
                  inst["sigma_obs0"], inst["sigma_obs_slope"],
                  inst["obs_center_x"], inst["inv_bin"], inst["key_lo"],
                  inst["key_n"], inst["goal_x"], inst["goal_y"],
                  inst["goal_r2"], inst["disk_r2"], inst["r_step"],
                  inst["r_goal"], inst["r_hit"], inst["heuristic"],
                  disks.size // 2, keep(disks, np.float32),
                  keep(inst["gauss"], np.float32), inst["gamma"])


@dataclass
class OracleResult:
    action: int
    v_root: float
    psi_root: np.ndarray
    particle_steps: int
    n_draws: int
    near_ties: int
    min_margin: float
    b_parent: np.ndarray
    b_obs: np.ndarray
    b_depth: np.ndarray
    psi: np.ndarray
    b_V: np.ndarray
    b_N: np.ndarray
    a_parent: np.ndarray
    a_act: np.ndarray
    a_C: np.ndarray
    a_N: np.ndarray
    trace: dict | None = None
    draws: dict | None = None
    handle: "Handle | None" = None


class Handle:
    """Owns an oracle result (a finished plan or a re-rooted tree)."""

    def __init__(self, h):
        self.h = h

    def __del__(self):
        if self.h:
            load().orc_result_free(self.h)
            self.h = None


def _tree_arrays(h, A):
    lib = load()
    info = np.zeros(8, np.int64)
    mm = np.zeros(1, np.float64)
    vr = np.zeros(1, np.float64)
    lib.orc_result_info(h, _ptr(info), _ptr(mm), _ptr(vr))
    nb, na = int(info[0]), int(info[1])
    out = dict(b_parent=np.zeros(nb, np.int32), b_obs=np.zeros(nb, np.int32),
               b_depth=np.zeros(nb, np.int32),
               psi=np.zeros((nb, A), np.float64),
               b_V=np.zeros(nb, np.float64), b_N=np.zeros(nb, np.int64),
               a_parent=np.zeros(na, np.int32), a_act=np.zeros(na, np.int32),
               a_C=np.zeros(na, np.float64), a_N=np.zeros(na, np.int64))
    lib.orc_result_tree(h, *[_ptr(out[k]) for k in (
        "b_parent", "b_obs", "b_depth", "psi", "b_V", "b_N", "a_parent",
        "a_act", "a_C", "a_N")])
    return info, mm, vr, out


def reroot(result, a, o, A):
    """Tree re-rooting between real steps: the subtree of ``result``'s tree
    (kept with ``plan(..., keep=True)``) under action a and observation o.
    Returns (Handle, tree arrays); the arrays are empty when the tree has no
    belief for (a, o), and a plan started from the handle then starts fresh."""
    h = load().orc_reroot(result.handle.h, int(a), int(o))
    hd = Handle(h)
    _, _, _, out = _tree_arrays(h, A)
    return hd, out


def step_base(budget, depth, schedule):
    """First level step of each iteration: [0, D_1, D_1 + D_2, ...] (K + 1)."""
    out = [0]
    for k in range(1, budget + 1):
        out.append(out[-1] + (depth if schedule == 1 else min(k, depth)))
    return np.asarray(out, np.int32)


def plan(inst, belief, n_particles, budget, depth, eta=1.0, seed=1,
         schedule=0, step=0, tau=2.0 ** -12, tau_abs=0.0, tau_psi=0.0, trace=False,
         draws=False, mutate=0, pi0=None, start=None, keep=False):
    """Run one serial planning step and return the full tree.  pi0: reference
    policy weights over the actions (positive; normalised), or None: uniform.
    start: a Handle from ``reroot`` to plan from its tree.  keep: keep the
    result's handle (``.handle``) for re-rooting.  tau, tau_abs, tau_psi:
    near-tie screen of the draws (|t - P_j| <= (tau + tau_psi * eta *
    max |Psi|) * P_last + tau_abs).  trace: the
    per-draw rows; draws: the same as dense arrays by (level step, episode)
    (``act`` -1 where no draw; ``flags`` bit 0 drawn, 1 terminal, 2 near tie)."""
    lib = load()
    hold = _Keep()
    pi = None
    if pi0 is not None:
        pi = np.ascontiguousarray(pi0, np.float64)
        assert pi.shape == (inst["nA"],) and np.all(pi > 0)
        hold.arrs.append(pi)
    prm = OrcParams(n_particles, budget, depth, schedule, eta, seed, step,
                    tau, tau_abs, tau_psi, 1 if (trace or draws) else 0, mutate,
                    None if pi is None else pi.ctypes.data,
                    None if start is None else start.h)
    if inst["kind"] == "tabular":
        m = tabular_struct(inst, hold)
        bel = _c32(belief, np.int32)
        h = lib.orc_plan_tabular(C.byref(m), _ptr(bel), bel.size, C.byref(prm))
    else:
        m = nav_struct(inst, hold)
        bx = _c32(belief[0], np.float32)
        by = _c32(belief[1], np.float32)
        h = lib.orc_plan_nav(C.byref(m), _ptr(bx), _ptr(by), bx.size,
                             C.byref(prm))
    hd = Handle(h)
    try:
        info, mm, vr, out = _tree_arrays(h, inst["nA"])
        tr = None
        if trace:
            n = int(info[6])
            ints = np.zeros((n, 8), np.int32)
            r = np.zeros(n, np.float32)
            mg = np.zeros(n, np.float64)
            lib.orc_result_trace(h, _ptr(ints), _ptr(r), _ptr(mg))
            tr = dict(k=ints[:, 0], d=ints[:, 1], ep=ints[:, 2], b=ints[:, 3],
                      a=ints[:, 4], obs=ints[:, 5], term=ints[:, 6],
                      an=ints[:, 7], r=r, margin=mg)
        dr = None
        if draws:
            sb = step_base(budget, depth, schedule)
            n = int(sb[-1]) * n_particles
            dr = dict(act=np.full(n, -1, np.int16), obs=np.zeros(n, np.int32),
                      flags=np.zeros(n, np.uint8), step_base=sb)
            lib.orc_result_draws(h, _ptr(sb), n_particles, _ptr(dr["act"]),
                                 _ptr(dr["obs"]), _ptr(dr["flags"]))
        return OracleResult(action=int(info[2]), v_root=float(vr[0]),
                            psi_root=out["psi"][0].copy(),
                            particle_steps=int(info[3]), n_draws=int(info[4]),
                            near_ties=int(info[5]), min_margin=float(mm[0]),
                            trace=tr, draws=dr, handle=hd if keep else None, **out)
    finally:
        if not keep:
            del hd


# Building blocks for the pins -------------------------------------------------

def philox(counter, key):
    lib = load()
    out = np.zeros(4, np.uint32)
    lib.orc_philox(*[int(c) & 0xFFFFFFFF for c in counter],
                   int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF, _ptr(out))
    return out


def thresholds(p):
    lib = load()
    p = _c32(p, np.float32)
    out = np.zeros(p.size, np.uint32)
    lib.orc_thresholds(_ptr(p), p.size, _ptr(out))
    return out


def pick(thr, x):
    lib = load()
    thr = _c32(thr, np.uint32)
    return int(lib.orc_pick(_ptr(thr), thr.size, int(x) & 0xFFFFFFFF))


def sample_action(psi, eta, x0, tau=0.0, tau_abs=0.0, tau_psi=0.0):
    """Eq. (6) draw: (action, margin, near tie under the screen)."""
    lib = load()
    psi = _c32(psi, np.float64)
    mg = np.zeros(1, np.float64)
    nr = np.zeros(1, np.int32)
    a = lib.orc_sample_action(_ptr(psi), psi.size, eta, int(x0) & 0xFFFFFFFF,
                              float(tau), float(tau_abs), float(tau_psi), _ptr(mg),
                              _ptr(nr))
    return int(a), float(mg[0]), bool(nr[0])


def nav_obs_weight(inst, x, y, o):
    """Navigation likelihood of observation key o at (x, y), units of 2^-24."""
    lib = load()
    keep = _Keep()
    m = nav_struct(inst, keep)
    return int(lib.orc_nav_obs_weight(C.byref(m), float(x), float(y), int(o)))


def nav_step(inst, x, y, a, w1, w2):
    lib = load()
    keep = _Keep()
    m = nav_struct(inst, keep)
    nx = np.zeros(1, np.float32)
    ny = np.zeros(1, np.float32)
    key = np.zeros(1, np.int32)
    r = np.zeros(1, np.float32)
    term = np.zeros(1, np.int32)
    lib.orc_nav_step(C.byref(m), float(x), float(y), int(a), int(w1), int(w2),
                     _ptr(nx), _ptr(ny), _ptr(key), _ptr(r), _ptr(term))
    return float(nx[0]), float(ny[0]), int(key[0]), float(r[0]), int(term[0])


def env_step(inst, state, a, seed, step):
    """One true-environment step.  state: int (tabular) or (x, y)."""
    lib = load()
    keep = _Keep()
    obs = np.zeros(1, np.int32)
    r = np.zeros(1, np.float32)
    term = np.zeros(1, np.int32)
    if inst["kind"] == "tabular":
        m = tabular_struct(inst, keep)
        s = np.array([state], np.int32)
        lib.orc_env_step_tabular(C.byref(m), _ptr(s), int(a), int(seed), int(step),
                                 _ptr(obs), _ptr(r), _ptr(term))
        return int(s[0]), int(obs[0]), float(r[0]), int(term[0])
    m = nav_struct(inst, keep)
    x = np.array([state[0]], np.float32)
    y = np.array([state[1]], np.float32)
    lib.orc_env_step_nav(C.byref(m), _ptr(x), _ptr(y), int(a), int(seed), int(step),
                         _ptr(obs), _ptr(r), _ptr(term))
    return (float(x[0]), float(y[0])), int(obs[0]), float(r[0]), int(term[0])


def belief_update(inst, particles, a, o, seed, step):
    """SIR update.  particles: int32 array (tabular) or (x, y) float32 arrays.
    Returns (new particles, integer weight total)."""
    lib = load()
    keep = _Keep()
    if inst["kind"] == "tabular":
        m = tabular_struct(inst, keep)
        p = np.array(particles, np.int32)
        tot = lib.orc_pf_update_tabular(C.byref(m), _ptr(p), p.size, int(a), int(o),
                                        int(seed), int(step))
        return p, int(tot)
    m = nav_struct(inst, keep)
    x = np.array(particles[0], np.float32)
    y = np.array(particles[1], np.float32)
    tot = lib.orc_pf_update_nav(C.byref(m), _ptr(x), _ptr(y), x.size, int(a), int(o),
                                int(seed), int(step))
    return (x, y), int(tot)
