"""Thin ctypes binding of the C ABI in ``include/vopp.h``.

Argument marshalling only: every step of a plan runs in the HIP library
``libvopp.so``.  PyTorch provides device memory (belief particles) and
streams.  Importing this module raises if the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvopp.so")

VOPP_OK = 0
VOPP_E_INVALID = -1
VOPP_E_NOMEM = -2
VOPP_E_DEVICE = -3
VOPP_E_BUSY = -4
VOPP_E_INTERNAL = -5
SCHEDULE_DEEPEN = 0
SCHEDULE_FIXED = 1

EXPORTS = (
    "vopp_last_error", "vopp_version", "vopp_pomdp_tabular", "vopp_pomdp_nav2d",
    "vopp_pomdp_num_actions", "vopp_pomdp_set_reference_policy", "vopp_pomdp_free",
    "vopp_plan_footprint",
    "vopp_workspace_create", "vopp_workspace_free", "vopp_plan", "vopp_plan_anytime",
    "vopp_reroot",
    "vopp_tree_dump", "vopp_level_counts", "vopp_profile_enable", "vopp_profile_reset",
    "vopp_profile_read", "vopp_batch_create", "vopp_batch_footprint",
    "vopp_batch_set_request", "vopp_batch_run", "vopp_batch_autotune",
    "vopp_batch_num_launches", "vopp_batch_auto_mode", "vopp_batch_free", "vopp_plan_batch",
    "vopp_env_step", "vopp_belief_update", "vopp_server_create",
    "vopp_server_submit", "vopp_server_tick", "vopp_server_poll",
    "vopp_server_episode_state", "vopp_server_free",
)
MAX_ACTIONS = 64

KERNEL_KINDS = ("forward", "accumulate", "backup_leaf", "backup_level", "backup_root",
                "setup", "select")


class VoppError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vopp status {status}: {msg}")
        self.status = status


class vopp_tabular_desc(C.Structure):
    _fields_ = [("nS", C.c_int32), ("nA", C.c_int32), ("nO", C.c_int32),
                ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("tprob", C.c_void_p), ("zprob", C.c_void_p),
                ("reward", C.c_void_p), ("heur", C.c_void_p),
                ("gamma", C.c_double)]


class vopp_nav2d_desc(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "lo", "hi", "step", "sigma_move", "sigma_obs0", "sigma_obs_slope",
        "obs_center_x", "inv_bin")] + [
        ("key_lo", C.c_int32), ("key_n", C.c_int32)] + [
        (n, C.c_float) for n in ("goal_x", "goal_y", "goal_r2", "disk_r2",
                                 "r_step", "r_goal", "r_hit")] + [
        ("heuristic", C.c_int32), ("n_disks", C.c_int32),
        ("disks", C.c_void_p), ("gauss", C.c_void_p), ("gamma", C.c_double)]


class vopp_params(C.Structure):
    _fields_ = [("n_particles", C.c_int32), ("schedule", C.c_int32),
                ("eta", C.c_double), ("seed", C.c_uint64), ("step", C.c_uint32)]


class vopp_stats(C.Structure):
    _fields_ = [("particle_steps", C.c_int64), ("n_beliefs", C.c_int64),
                ("n_actions", C.c_int64), ("device_ms", C.c_double),
                ("near_ties", C.c_int64), ("sweep_visits", C.c_int64),
                ("sweep_internal", C.c_int64), ("sweep_nodes", C.c_int64),
                ("insert_reprobes", C.c_int64)]


class vopp_request(C.Structure):
    _fields_ = [("pomdp", C.c_void_p), ("belief_particles", C.c_void_p),
                ("n_belief", C.c_int32), ("budget", C.c_int32), ("depth", C.c_int32),
                ("params", vopp_params)]


class vopp_result(C.Structure):
    _fields_ = [("action", C.c_int32), ("status", C.c_int32), ("v_root", C.c_double),
                ("particle_steps", C.c_int64), ("n_beliefs", C.c_int64),
                ("n_actions", C.c_int64), ("values", C.c_double * MAX_ACTIONS)]


class vopp_tuning(C.Structure):
    _fields_ = [("accum_cap", C.c_int32), ("backup_cap", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("forward_group", C.c_int32),
                ("sweep_group", C.c_int32)]


BATCH_EAGER, BATCH_GRAPH, BATCH_PERSISTENT, BATCH_AUTO = 0, 1, 2, 3


class vopp_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_active", C.c_int32),
                ("max_inflight", C.c_int32), ("phases_per_tick", C.c_int32)]


class vopp_episode_desc(C.Structure):
    _fields_ = [("pomdp", C.c_void_p), ("init_particles", C.c_void_p),
                ("n_particles", C.c_int32), ("budget", C.c_int32), ("depth", C.c_int32),
                ("params", vopp_params), ("true_state", C.c_void_p),
                ("env_seed", C.c_uint64), ("n_steps", C.c_int32)]


class vopp_served(C.Structure):
    _fields_ = [("episode", C.c_int32), ("step", C.c_int32), ("action", C.c_int32),
                ("status", C.c_int32), ("v_root", C.c_double),
                ("particle_steps", C.c_int64), ("arrival_s", C.c_double),
                ("done_s", C.c_double)]


_lib = None


def lib():
    """Load libvopp.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run python -m paper_2510_27191_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i32, st = C.c_void_p, C.c_int32, C.c_int
    L.vopp_last_error.restype = C.c_char_p
    L.vopp_version.restype = C.c_char_p
    L.vopp_pomdp_tabular.argtypes = [C.POINTER(vopp_tabular_desc), C.POINTER(vp)]
    L.vopp_pomdp_tabular.restype = st
    L.vopp_pomdp_nav2d.argtypes = [C.POINTER(vopp_nav2d_desc), C.POINTER(vp)]
    L.vopp_pomdp_nav2d.restype = st
    L.vopp_pomdp_num_actions.argtypes = [vp]
    L.vopp_pomdp_num_actions.restype = i32
    L.vopp_pomdp_set_reference_policy.argtypes = [vp, C.POINTER(C.c_double)]
    L.vopp_pomdp_set_reference_policy.restype = st
    L.vopp_pomdp_free.argtypes = [vp]
    L.vopp_pomdp_free.restype = None
    L.vopp_plan_footprint.argtypes = [vp, C.POINTER(vopp_params), i32, i32]
    L.vopp_plan_footprint.restype = C.c_size_t
    L.vopp_workspace_create.argtypes = [vp, C.POINTER(vopp_params), i32, i32,
                                        C.POINTER(vp)]
    L.vopp_workspace_create.restype = st
    L.vopp_workspace_free.argtypes = [vp]
    L.vopp_workspace_free.restype = None
    L.vopp_plan.argtypes = [vp, vp, i32, i32, i32, C.POINTER(vopp_params), vp, vp,
                            C.POINTER(i32), vp, vp, C.POINTER(vopp_stats)]
    L.vopp_plan.restype = st
    L.vopp_plan_trace.argtypes = [vp, vp, i32, i32, i32, C.POINTER(vopp_params), vp, vp,
                                  C.POINTER(i32), vp, vp, C.POINTER(vopp_stats), vp, vp,
                                  vp, C.c_int64]
    L.vopp_plan_trace.restype = st
    L.vopp_plan_noalloc.argtypes = [vp, vp, i32, i32, i32, C.POINTER(vopp_params), vp, vp]
    L.vopp_plan_noalloc.restype = st
    L.vopp_plan_anytime.argtypes = [vp, vp, i32, i32, i32, C.c_double, C.POINTER(vopp_params),
                                    vp, vp, C.POINTER(i32), vp, vp, C.POINTER(vopp_stats),
                                    C.POINTER(i32)]
    L.vopp_plan_anytime.restype = st
    L.vopp_reroot.argtypes = [vp, vp, i32, i32, C.POINTER(vopp_params), i32, i32, vp, vp,
                              C.POINTER(C.c_int64)]
    L.vopp_reroot.restype = st
    L.vopp_tree_dump.argtypes = [vp] * 11
    L.vopp_tree_dump.restype = st
    L.vopp_level_counts.argtypes = [vp, vp, i32, C.POINTER(i32)]
    L.vopp_level_counts.restype = st
    L.vopp_profile_enable.argtypes = [vp, i32]
    L.vopp_profile_enable.restype = st
    L.vopp_profile_reset.argtypes = [vp]
    L.vopp_profile_reset.restype = st
    L.vopp_profile_read.argtypes = [vp, vp, vp]
    L.vopp_profile_read.restype = st
    L.vopp_batch_create.argtypes = [vp, i32, C.POINTER(vopp_tuning), C.POINTER(vp)]
    L.vopp_batch_create.restype = st
    L.vopp_batch_footprint.argtypes = [vp, i32]
    L.vopp_batch_footprint.restype = C.c_size_t
    L.vopp_batch_set_request.argtypes = [vp, i32, vp, i32, C.c_uint64, C.c_uint32]
    L.vopp_batch_set_request.restype = st
    L.vopp_batch_run.argtypes = [vp, vp, i32, vp, vp]
    L.vopp_batch_run.restype = st
    L.vopp_batch_autotune.argtypes = [vp, vp, i32, C.POINTER(vopp_tuning)]
    L.vopp_batch_autotune.restype = st
    L.vopp_batch_num_launches.argtypes = [vp]
    L.vopp_batch_num_launches.restype = i32
    L.vopp_batch_auto_mode.argtypes = [vp]
    L.vopp_batch_auto_mode.restype = i32
    L.vopp_batch_free.argtypes = [vp]
    L.vopp_batch_free.restype = None
    L.vopp_plan_batch.argtypes = [vp, i32, vp, vp]
    L.vopp_plan_batch.restype = st
    L.vopp_env_step.argtypes = [vp, vp, i32, C.c_uint64, C.c_uint32, vp, vp, vp, vp]
    L.vopp_env_step.restype = st
    L.vopp_belief_update.argtypes = [vp, vp, i32, i32, i32, C.c_uint64, C.c_uint32, vp, vp]
    L.vopp_belief_update.restype = st
    L.vopp_server_create.argtypes = [C.POINTER(vopp_server_config), C.POINTER(vp)]
    L.vopp_server_create.restype = st
    L.vopp_server_submit.argtypes = [vp, C.POINTER(vopp_episode_desc), C.POINTER(i32)]
    L.vopp_server_submit.restype = st
    L.vopp_server_tick.argtypes = [vp, C.POINTER(i32)]
    L.vopp_server_tick.restype = st
    L.vopp_server_poll.argtypes = [vp, vp, i32]
    L.vopp_server_poll.restype = i32
    L.vopp_server_episode_state.argtypes = [vp, i32, vp, C.POINTER(i32)]
    L.vopp_server_episode_state.restype = st
    L.vopp_server_free.argtypes = [vp]
    L.vopp_server_free.restype = None
    _lib = L
    return L


def _check(status):
    if status != VOPP_OK:
        raise VoppError(status, lib().vopp_last_error().decode())


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _arr(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Pomdp:
    """A model handle (vopp_pomdp_tabular / vopp_pomdp_nav2d)."""

    def __init__(self, handle, kind, nA):
        self.handle = C.c_void_p(handle)
        self.kind = kind
        self.nA = nA

    @classmethod
    def from_instance(cls, inst):
        L = lib()
        h = C.c_void_p()
        if inst["kind"] == "tabular":
            keep = [_arr(inst["rowptr"], np.int32), _arr(inst["col"], np.int32),
                    _arr(inst["tprob"], np.float32), _arr(inst["zprob"], np.float32),
                    _arr(inst["reward"], np.float32)]
            heur = inst.get("heur")
            heur = None if heur is None else _arr(heur, np.float32)
            d = vopp_tabular_desc(inst["nS"], inst["nA"], inst["nO"],
                                  *[_p(a) for a in keep], _p(heur), inst["gamma"])
            _check(L.vopp_pomdp_tabular(C.byref(d), C.byref(h)))
            return cls(h.value, "tabular", inst["nA"])
        disks = _arr(inst["disks"], np.float32).reshape(-1)
        gauss = _arr(inst["gauss"], np.float32)
        d = vopp_nav2d_desc(inst["lo"], inst["hi"], inst["step"], inst["sigma_move"],
                            inst["sigma_obs0"], inst["sigma_obs_slope"],
                            inst["obs_center_x"], inst["inv_bin"], inst["key_lo"],
                            inst["key_n"], inst["goal_x"], inst["goal_y"],
                            inst["goal_r2"], inst["disk_r2"], inst["r_step"],
                            inst["r_goal"], inst["r_hit"], inst["heuristic"],
                            disks.size // 2, _p(disks), _p(gauss), inst["gamma"])
        _check(L.vopp_pomdp_nav2d(C.byref(d), C.byref(h)))
        return cls(h.value, "nav", 4)

    def set_reference_policy(self, pi0):
        """vopp_pomdp_set_reference_policy: pi0 of |A| positive weights, or None
        for the uniform policy."""
        if pi0 is None:
            _check(lib().vopp_pomdp_set_reference_policy(self.handle, None))
            return
        a = _arr(pi0, np.float64).reshape(-1)
        if a.size != self.nA:
            raise ValueError(f"reference policy has {a.size} entries, the model {self.nA} actions")
        _check(lib().vopp_pomdp_set_reference_policy(
            self.handle, a.ctypes.data_as(C.POINTER(C.c_double))))

    def close(self):
        if self.handle:
            lib().vopp_pomdp_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params(n_particles, eta=1.0, seed=1, schedule=SCHEDULE_DEEPEN, step=0):
    return vopp_params(int(n_particles), int(schedule), float(eta),
                       int(seed) & (2 ** 64 - 1), int(step) & 0xFFFFFFFF)


class Workspace:
    def __init__(self, pomdp, prm, budget, depth):
        h = C.c_void_p()
        _check(lib().vopp_workspace_create(pomdp.handle, C.byref(prm), int(budget),
                                           int(depth), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().vopp_workspace_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(pomdp, prm, budget, depth):
    return int(lib().vopp_plan_footprint(pomdp.handle, C.byref(prm), int(budget),
                                         int(depth)))


@dataclass
class PlanResult:
    action: int
    values: np.ndarray
    v_root: float
    particle_steps: int
    n_beliefs: int
    n_actions: int
    device_ms: float
    near_ties: int = 0
    sweep: tuple = (0, 0, 0)      # level sweeps: belief, internal, action-node visits
    insert_reprobes: int = 0      # inserts whose slot another key took first


def _sweep(st):
    return (int(st.sweep_visits), int(st.sweep_internal), int(st.sweep_nodes))


def belief_tensor(inst, belief, device="cuda"):
    """Device tensor of belief particles in the layout vopp_plan expects."""
    import torch
    if inst["kind"] == "tabular":
        return torch.as_tensor(_arr(belief, np.int32), device=device)
    x, y = belief
    return torch.as_tensor(np.concatenate([_arr(x, np.float32), _arr(y, np.float32)]),
                           device=device)


def plan(pomdp, belief_dev, n_belief, budget, depth, prm, ws=None, stream=None):
    """vopp_plan on a device tensor of belief particles."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    act = C.c_int32(-1)
    vals = np.zeros(pomdp.nA, np.float64)
    vroot = np.zeros(1, np.float64)
    st = vopp_stats()
    _check(lib().vopp_plan(pomdp.handle, C.c_void_p(belief_dev.data_ptr()),
                           int(n_belief), int(budget), int(depth), C.byref(prm),
                           ws.handle if ws is not None else None,
                           C.c_void_p(stream.cuda_stream), C.byref(act), _p(vals),
                           _p(vroot), C.byref(st)))
    return PlanResult(int(act.value), vals, float(vroot[0]), int(st.particle_steps),
                      int(st.n_beliefs), int(st.n_actions), float(st.device_ms),
                      int(st.near_ties), _sweep(st), int(st.insert_reprobes))


def plan_trace(pomdp, belief_dev, n_belief, budget, depth, prm, ws=None, stream=None,
               force=None):
    """vopp_plan_trace: returns (PlanResult, act, obs), with act (int16, the
    kernel's own decisions) and obs (int32) of shape [level steps, n_particles]
    on the host (-1 where an episode had terminated).  force: None, or an
    int16 array of the same size whose entries >= 0 replace the kernel's
    decision at that draw."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    steps = sum(depth if prm.schedule == 1 else min(k, depth) for k in range(1, budget + 1))
    n = steps * prm.n_particles
    act_d = torch.empty(n, dtype=torch.int16, device=belief_dev.device)
    obs_d = torch.empty(n, dtype=torch.int32, device=belief_dev.device)
    force_d = None
    if force is not None:
        f = np.ascontiguousarray(np.asarray(force, np.int16).reshape(-1))
        if f.size != n:
            raise ValueError(f"force holds {f.size} entries, the plan has {n} draws")
        force_d = torch.as_tensor(f, device=belief_dev.device)
    act = C.c_int32(-1)
    vals = np.zeros(pomdp.nA, np.float64)
    vroot = np.zeros(1, np.float64)
    st = vopp_stats()
    _check(lib().vopp_plan_trace(pomdp.handle, C.c_void_p(belief_dev.data_ptr()),
                                 int(n_belief), int(budget), int(depth), C.byref(prm),
                                 ws.handle if ws is not None else None,
                                 C.c_void_p(stream.cuda_stream), C.byref(act), _p(vals),
                                 _p(vroot), C.byref(st), C.c_void_p(act_d.data_ptr()),
                                 C.c_void_p(obs_d.data_ptr()),
                                 None if force_d is None else C.c_void_p(force_d.data_ptr()),
                                 C.c_int64(n)))
    res = PlanResult(int(act.value), vals, float(vroot[0]), int(st.particle_steps),
                     int(st.n_beliefs), int(st.n_actions), float(st.device_ms),
                     int(st.near_ties), _sweep(st), int(st.insert_reprobes))
    shape = (steps, prm.n_particles)
    return (res, act_d.cpu().numpy().reshape(shape), obs_d.cpu().numpy().reshape(shape))


NOALLOC_SCRATCH_BYTES = 64 << 20


def plan_noalloc(pomdp, belief_dev, n_belief, budget, depth, prm, result_dev, stream=None):
    """vopp_plan_noalloc: enqueue a plan whose tree lives in the library's
    static device array; result_dev is a float64 device tensor of at least
    nA + 10 entries (action, root preferences, V(root), particle steps,
    beliefs, action nodes, error flags, near ties, sweep counts), written on
    the stream."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if result_dev.dtype != torch.float64 or result_dev.numel() < pomdp.nA + 10:
        raise ValueError("result_dev must be a float64 device tensor of nA + 10 entries")
    _check(lib().vopp_plan_noalloc(pomdp.handle, C.c_void_p(belief_dev.data_ptr()),
                                   int(n_belief), int(budget), int(depth), C.byref(prm),
                                   C.c_void_p(stream.cuda_stream),
                                   C.c_void_p(result_dev.data_ptr())))


def plan_anytime(pomdp, belief_dev, n_belief, max_budget, depth, time_ms, prm, ws=None,
                 stream=None):
    """vopp_plan_anytime: returns (PlanResult, iterations run)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    act = C.c_int32(-1)
    iters = C.c_int32(0)
    vals = np.zeros(pomdp.nA, np.float64)
    vroot = np.zeros(1, np.float64)
    st = vopp_stats()
    _check(lib().vopp_plan_anytime(pomdp.handle, C.c_void_p(belief_dev.data_ptr()),
                                   int(n_belief), int(max_budget), int(depth),
                                   float(time_ms), C.byref(prm),
                                   ws.handle if ws is not None else None,
                                   C.c_void_p(stream.cuda_stream), C.byref(act), _p(vals),
                                   _p(vroot), C.byref(st), C.byref(iters)))
    res = PlanResult(int(act.value), vals, float(vroot[0]), int(st.particle_steps),
                     int(st.n_beliefs), int(st.n_actions), float(st.device_ms),
                     int(st.near_ties), _sweep(st), int(st.insert_reprobes))
    return res, int(iters.value)


def reroot(pomdp, src, action, obs, next_prm, next_budget, next_depth, dst, stream=None):
    """vopp_reroot: keep the subtree of src's tree under (action, obs) in dst
    for the next plan; returns the number of kept beliefs (0: none)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    kept = C.c_int64(0)
    _check(lib().vopp_reroot(pomdp.handle, src.handle, int(action), int(obs),
                             C.byref(next_prm), int(next_budget), int(next_depth),
                             dst.handle, C.c_void_p(stream.cuda_stream), C.byref(kept)))
    return int(kept.value)


def tree_dump(ws, nA, n_beliefs, n_actions):
    out = dict(b_parent=np.zeros(n_beliefs, np.int32), b_obs=np.zeros(n_beliefs, np.int32),
               b_depth=np.zeros(n_beliefs, np.int32),
               psi=np.zeros((n_beliefs, nA), np.float32),
               b_V=np.zeros(n_beliefs, np.float32), b_N=np.zeros(n_beliefs, np.int32),
               a_parent=np.zeros(n_actions, np.int32), a_act=np.zeros(n_actions, np.int32),
               a_C=np.zeros(n_actions, np.float64), a_N=np.zeros(n_actions, np.int32))
    _check(lib().vopp_tree_dump(ws.handle, *[_p(out[k]) for k in (
        "b_parent", "b_obs", "b_depth", "psi", "b_V", "b_N", "a_parent", "a_act",
        "a_C", "a_N")]))
    return out


def level_counts(ws):
    """Beliefs created by each level step of the last plan in ws."""
    n = C.c_int32(0)
    _check(lib().vopp_level_counts(ws.handle, None, 0, C.byref(n)))
    out = np.zeros(n.value, np.int32)
    _check(lib().vopp_level_counts(ws.handle, _p(out), n.value, C.byref(n)))
    return out


def profile_enable(ws, kinds=None):
    """Bracket launches of the given kernel kinds (None: all; []: stop)."""
    if kinds is None:
        mask = -1
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << KERNEL_KINDS.index(k)
    _check(lib().vopp_profile_enable(ws.handle, mask))


def profile_reset(ws):
    _check(lib().vopp_profile_reset(ws.handle))


def profile_read(ws):
    """{kind: (total_ms, launches)} accumulated by the event profiler."""
    ms = np.zeros(len(KERNEL_KINDS), np.float64)
    n = np.zeros(len(KERNEL_KINDS), np.int64)
    _check(lib().vopp_profile_read(ws.handle, _p(ms), _p(n)))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_KINDS)}


def make_requests(items):
    """items: list of (Pomdp, belief device tensor, n_belief, budget, depth, params)."""
    arr = (vopp_request * len(items))()
    for i, (pom, bel, nb, K, depth, prm) in enumerate(items):
        arr[i] = vopp_request(pom.handle.value, bel.data_ptr(), int(nb), int(K),
                              int(depth), prm)
    return arr


def _results(arr, nAs):
    out = []
    for r, nA in zip(arr, nAs):
        out.append(PlanResult(int(r.action), np.array(r.values[:nA], np.float64),
                              float(r.v_root), int(r.particle_steps), int(r.n_beliefs),
                              int(r.n_actions), float("nan")))
    return out


class Batch:
    """vopp_batch: many requests advanced together, replayed as one hipGraph."""

    def __init__(self, items, tuning=None):
        self.items = list(items)
        self.reqs = make_requests(self.items)
        self.nAs = [it[0].nA for it in self.items]
        h = C.c_void_p()
        if tuning is not None and len(tuning) < 5:
            tuning = tuple(tuning) + (0, 1, 4)[len(tuning) - 2:]
        tu = None if tuning is None else C.byref(vopp_tuning(*tuning))
        _check(lib().vopp_batch_create(C.cast(self.reqs, C.c_void_p), len(self.items), tu,
                                       C.byref(h)))
        self.handle = h

    def __len__(self):
        return len(self.items)

    @property
    def num_launches(self):
        return int(lib().vopp_batch_num_launches(self.handle))

    @property
    def auto_mode(self):
        """The mode BATCH_AUTO runs (BATCH_GRAPH or BATCH_PERSISTENT)."""
        return int(lib().vopp_batch_auto_mode(self.handle))

    def set_request(self, i, belief_dev, n_belief, seed, step=0):
        _check(lib().vopp_batch_set_request(self.handle, int(i),
                                            C.c_void_p(belief_dev.data_ptr()),
                                            int(n_belief), int(seed) & (2 ** 64 - 1),
                                            int(step) & 0xFFFFFFFF))

    def run(self, use_graph=True, stream=None, mode=None):
        """mode: BATCH_AUTO (default: the faster mode of the last autotune,
        else the persistent launch), BATCH_PERSISTENT, BATCH_GRAPH or
        BATCH_EAGER; the older use_graph=False means BATCH_EAGER."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        if mode is None:
            mode = BATCH_AUTO if use_graph else BATCH_EAGER
        arr = (vopp_result * len(self.items))()
        ms = np.zeros(1, np.float64)
        _check(lib().vopp_batch_run(self.handle, C.c_void_p(stream.cuda_stream),
                                    int(mode), C.cast(arr, C.c_void_p), _p(ms)))
        return _results(arr, self.nAs), float(ms[0])

    def autotune(self, reps=2, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        tu = vopp_tuning()
        _check(lib().vopp_batch_autotune(self.handle, C.c_void_p(stream.cuda_stream),
                                         int(reps), C.byref(tu)))
        return (int(tu.accum_cap), int(tu.backup_cap), int(tu.blocks_per_cu),
                int(tu.forward_group), int(tu.sweep_group))

    def close(self):
        if self.handle:
            lib().vopp_batch_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def env_step(pomdp, state_dev, action, seed, step, stream=None):
    """vopp_env_step on a device state tensor (int32[1] or float32[2]), in place."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    obs = C.c_int32()
    r = C.c_float()
    term = C.c_int32()
    _check(lib().vopp_env_step(pomdp.handle, C.c_void_p(state_dev.data_ptr()), int(action),
                               int(seed) & (2 ** 64 - 1), int(step) & 0xFFFFFFFF,
                               C.c_void_p(stream.cuda_stream), C.byref(obs), C.byref(r),
                               C.byref(term)))
    return int(obs.value), float(r.value), int(term.value)


def belief_update(pomdp, particles_dev, n, action, obs, seed, step, stream=None):
    """vopp_belief_update in place on a device particle tensor; returns the
    integer weight total."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    tot = C.c_uint64()
    _check(lib().vopp_belief_update(pomdp.handle, C.c_void_p(particles_dev.data_ptr()),
                                    int(n), int(action), int(obs),
                                    int(seed) & (2 ** 64 - 1), int(step) & 0xFFFFFFFF,
                                    C.c_void_p(stream.cuda_stream), C.byref(tot)))
    return int(tot.value)


def particles_host(inst, belief):
    """Host array in vopp_plan's belief layout (tabular int32; nav x then y)."""
    if inst["kind"] == "tabular":
        return _arr(belief, np.int32)
    return np.concatenate([_arr(belief[0], np.float32), _arr(belief[1], np.float32)])


class Server:
    """vopp_server: continuous batching of many episodes' planning steps."""

    def __init__(self, hbm_budget_bytes=64 << 30, max_active=256, max_inflight=3,
                 phases_per_tick=1):
        h = C.c_void_p()
        cfg = vopp_server_config(int(hbm_budget_bytes), int(max_active), int(max_inflight),
                                 int(phases_per_tick))
        _check(lib().vopp_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self.kinds = {}

    def submit(self, pomdp, particles, budget, depth, prm, true_state, env_seed, n_steps):
        """particles: host array from particles_host(); true_state: int or (x, y)."""
        parts = np.ascontiguousarray(particles)
        n = parts.size if pomdp.kind == "tabular" else parts.size // 2
        st = (np.array([true_state], np.int32) if pomdp.kind == "tabular"
              else np.array(true_state, np.float32))
        d = vopp_episode_desc(pomdp.handle.value, _p(parts), int(n), int(budget), int(depth),
                              prm, _p(st), int(env_seed) & (2 ** 64 - 1), int(n_steps))
        eid = C.c_int32()
        _check(lib().vopp_server_submit(self.handle, C.byref(d), C.byref(eid)))
        self.kinds[eid.value] = pomdp.kind
        return int(eid.value)

    def tick(self):
        pending = C.c_int32()
        _check(lib().vopp_server_tick(self.handle, C.byref(pending)))
        return int(pending.value)

    def poll(self, max_n=4096):
        arr = (vopp_served * max_n)()
        n = lib().vopp_server_poll(self.handle, C.cast(arr, C.c_void_p), max_n)
        return [dict(episode=a.episode, step=a.step, action=a.action, status=a.status,
                     v_root=a.v_root, particle_steps=a.particle_steps,
                     arrival_s=a.arrival_s, done_s=a.done_s) for a in arr[:n]]

    def episode_state(self, eid):
        buf = np.zeros(2, np.int32)
        steps = C.c_int32()
        _check(lib().vopp_server_episode_state(self.handle, int(eid), _p(buf), C.byref(steps)))
        if self.kinds.get(eid) == "tabular":
            return int(buf[0]), int(steps.value)
        f = buf.view(np.float32)
        return (float(f[0]), float(f[1])), int(steps.value)

    def run_until_idle(self, timeout_s=120.0):
        import time
        out = []
        t0 = time.time()
        while True:
            pending = self.tick()
            out += self.poll()
            if pending == 0:
                break
            if time.time() - t0 > timeout_s:
                raise TimeoutError("server did not drain")
        return out

    def close(self):
        if self.handle:
            lib().vopp_server_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
