#!/usr/bin/env python
"""Benchmark of one VOPP planning step on one MI355X.

A "step" is one full planning step (Alg. 1: K iterations of sampling,
level-by-level forward search and bottom-up backup, then the root argmax) on
the continuous 2-D navigation POMDP: n_p = 65,536 episodes, depth 10, budget
K = 10 iterations, 8 obstacle disks, observations keyed on a 0.5 grid.  Inputs
(model tables and belief particles) are resident in HBM before timing starts.

Prints one JSON line:
  value        particle-steps/s (generative-model calls per second, whole job)
  latency_ms   p50 / p99 of the per-plan wall time (host call to result)
  roofline     achieved algorithmic GB/s of the dominant kernel (its launches'
               own start and end timestamps) against the 8 TB/s HBM peak
  cpu_baseline the serial CPU oracle timed on a bounded sample of the workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The method's bytes per unit of work (the hot-path scope table's per-unit
# figures), independent of this implementation's layout:
#   forward, per particle step: read the episode's particle (state 12 B
#     tabular, 16 B navigation), gather the preference row 4|A|, probe the
#     (belief, action) child 4, probe the belief table 16, update N and C 12,
#     write the next state and belief 8; per new action node 16; per new
#     belief 12 + 8|A| for its row, initial preferences and child links, plus
#     a 16 B table insert.
#   backup, per node visit: a belief as a child 20 (read V, N_b and its
#     parent 12, accumulate into the parent 8); an internal belief (one with
#     an action node) 12|A| + 8 (read and write its preferences, read its
#     child links, write V and N_b); an action node 20.
# The level sweeps count their own visits (vopp_stats.sweep_*); the leaf sweep
# visits every belief of the iteration's deepest depth as a child.
def method_bytes(kind, nA, particle_steps, n_beliefs, n_actions, sweep, leaf_visits):
    state = 16 if kind == "nav2d" else 12
    visits, internal, nodes = sweep
    return {
        "forward": particle_steps * (state + 4 * nA + 4 + 16 + 12 + 8) + n_actions * 16
                   + (n_beliefs - 1) * (12 + 8 * nA + 16),
        "backup_level": 20 * visits + (12 * nA + 8) * internal + 20 * nodes,
        "backup_leaf": 20 * leaf_visits,
    }


# Bytes the present layout moves for the same work (the overhead against the
# method's bytes).  The tree is one array per field indexed by belief id (ra =
# |A| rounded up to a multiple of 4).  A level sweep visit reads the position's
# list entry (4), the belief's hot fields {V, N_b, parent} (16) and its visit
# counts (4*ra), and pushes into its parent's W (16: the atomic's read and
# write); a belief with an action node also reads and writes its preference
# row (8*ra) and writes V and N_b (8); each action node reads C and W (16) and
# clears W (8).
def layout_bytes_backup_level(nA, sweep):
    ra = (nA + 3) // 4 * 4
    visits, internal, nodes = sweep
    return visits * (4 + 16 + 4 * ra + 16) + internal * (8 * ra + 8) + nodes * 24


def leaf_sweep_visits(n_p, K, depth, counts):
    """Beliefs the leaf sweeps visit over a plan (every belief of the
    iteration's deepest depth), from the beliefs created per level step."""
    D = [min(k, depth) for k in range(1, K + 1)]
    t0 = np.concatenate([[0], np.cumsum(D)[:-1]]).astype(int)
    total = 0
    for k in range(1, K + 1):
        dep = D[k - 1]
        total += sum(int(counts[t0[kk] + dep - 1]) for kk in range(k) if D[kk] >= dep)
    return total


# Measured HBM traffic of the dominant kernels per launch (bytes), from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE passes summarised in
# profiles/planning_step_hbm_traffic.md.  "copy": each counter scaled by what it
# reads for a plain device copy of known size (FETCH_SIZE x 2.0, WRITE_SIZE x
# 1.0).  "gather": FETCH_SIZE unscaled, which is what the counter reads for
# random 16-byte reads (128 B per access, one cache line), the access pattern of
# these kernels.  Valid only for the kernel sources they were taken on (hash
# below); otherwise `traffic` is reported as null.
MEASURED_TRAFFIC = {
    "sources_sha256_16": "ea77e652ac2a13d4",
    "backup_level": {"nav2d": 3.91e+07, "sparse4096": 1.294e+08},
    "forward": {"nav2d": 1.31e+08, "sparse4096": 6.829e+08},
    "gather_scale": {
        "backup_level": {"nav2d": 2.69e+07, "sparse4096": 8.177e+07},
        "forward": {"nav2d": 1.073e+08, "sparse4096": 4.898e+08},
    },
}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("vopp_kernels.hip", "vopp_device.hpp"):
        with open(os.path.join(ROOT, "paper_2510_27191_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


def cpu_baseline(inst, bel, p, budget_s=12.0, max_plans=4):
    """Time the serial oracle on whole plans of the same workload."""
    from oracle import oracle as orc
    steps = 0
    t_total = 0.0
    plans = 0
    while plans < max_plans and (t_total < budget_s or plans == 0):
        t0 = time.perf_counter()
        r = orc.plan(inst, bel, p["n_particles"], p["budget"], p["depth"],
                     eta=p["eta"], seed=7 + plans)
        t_total += time.perf_counter() - t0
        steps += r.particle_steps
        plans += 1
    return {"value": steps / t_total, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{plans} full plan(s) of the same workload "
                      f"(n_p={p['n_particles']}, K={p['budget']}, depth={p['depth']}), "
                      f"serial, {t_total:.1f} s"}


def _oracle_mix_worker(indices, barrier, queue):
    """One host core of the parallel oracle baseline: plans the given
    instances of the 256-instance mix serially (after every worker has built
    its inputs) and reports (particle steps, seconds)."""
    sys.path.insert(0, ROOT)
    from oracle import oracle as orc
    from paper_2510_27191_amd import instances as I
    mix = I.batch_mix(0)
    barrier.wait()
    t0 = time.perf_counter()
    steps = 0
    for i in indices:
        inst, bel, p = mix[i]
        r = orc.plan(inst, bel, p["n_particles"], p["budget"], p["depth"], eta=p["eta"],
                     seed=p["seed"])
        steps += r.particle_steps
    queue.put((steps, time.perf_counter() - t0))


def host_cores():
    """Host cores this process may use (the GPU machine gives one GPU 16 of them,
    whatever the machine has)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_mix_baseline(stride=16):
    """The serial oracle over a bounded sample of the 256-instance mix (the
    instances i with i % stride in {0, 1}: half tabular, half navigation),
    one worker process per host core, instances dealt round robin.  Rate =
    all particle steps / the slowest worker's planning time."""
    import multiprocessing as mp
    from paper_2510_27191_amd import instances as I
    idx = [i for i in range(256) if i % stride in (0, 1)]
    cores = min(host_cores(), len(idx))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    queue = ctx.Queue()
    # Largest instances first, so the deal balances the workers.
    mix = I.batch_mix(0)
    work = sorted(idx, key=lambda i: -mix[i][2]["n_particles"] * mix[i][2]["depth"] ** 2)
    procs = [ctx.Process(target=_oracle_mix_worker, args=(work[w::cores], barrier, queue))
             for w in range(cores)]
    for pr in procs:
        pr.start()
    got = [queue.get() for _ in procs]
    for pr in procs:
        pr.join()
    steps = sum(g[0] for g in got)
    wall = max(g[1] for g in got)
    return {"value": steps / wall, "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{len(idx)} of the 256 instances (i mod {stride} in {{0, 1}}), "
                      f"{steps} particle steps, one serial oracle process per core, "
                      f"slowest worker {wall:.1f} s, "
                      f"{sum(g[1] for g in got):.1f} s of CPU time in all"}


def bench_batch(V, I, reps=3, autotune=True, cpu=True):
    """256 mixed instances: one batched hipGraph replay vs 256 plain calls."""
    import torch
    mix = I.batch_mix(0)
    items = []
    for inst, bel, p in mix:
        pom = V.Pomdp.from_instance(inst)
        belt = V.belief_tensor(inst, bel)
        nb = belt.numel() if inst["kind"] == "tabular" else belt.numel() // 2
        items.append((pom, belt, nb, p["budget"], p["depth"],
                      V.params(p["n_particles"], eta=p["eta"], seed=p["seed"])))
    stream = torch.cuda.current_stream()
    # Plain: one vopp_plan per instance, back to back (each returns its result).
    for pom, belt, nb, K, depth, prm in items:          # warm-up, allocates
        V.plan(pom, belt, nb, K, depth, prm, stream=stream)
    torch.cuda.synchronize()
    plain_s, plain_lat = [], []
    steps = 0
    for _ in range(reps):
        t0 = time.perf_counter()
        steps = 0
        for pom, belt, nb, K, depth, prm in items:
            a = time.perf_counter()
            r = V.plan(pom, belt, nb, K, depth, prm, stream=stream)
            plain_lat.append((time.perf_counter() - a) * 1e3)
            steps += r.particle_steps
        plain_s.append(time.perf_counter() - t0)
    plain_ref = [V.plan(pom, belt, nb, K, depth, prm, stream=stream)
                 for pom, belt, nb, K, depth, prm in items]
    # Batched: the autotuner times the persistent launch over its tile sizes
    # and the per-phase graph over its block caps; each mode is then timed
    # at its own best tuning, and the faster is the batch's figure.
    batch = V.Batch(items)
    tuning = batch.autotune(reps=1) if autotune else None

    def timed(mode):
        batch.run(mode=mode)
        wall, dev, r = [], [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r, ms = batch.run(mode=mode)
            wall.append(time.perf_counter() - t0)
            dev.append(ms)
        return r, wall, dev
    res, batch_s, batch_dev = timed(V.BATCH_PERSISTENT)
    res_phase, phase_s, phase_dev = timed(V.BATCH_GRAPH)
    n_launches = batch.num_launches
    auto_mode = batch.auto_mode

    def same_all(rs):
        return all(a.action == b.action and np.array_equal(a.values, b.values)
                   and a.n_beliefs == b.n_beliefs for a, b in zip(rs, plain_ref))
    identical = same_all(res) and same_all(res_phase)
    bsteps = sum(r.particle_steps for r in res)
    out = {
        "workload": "256 mixed instances: tabular (|S| log-uniform 64-4096, |A| 3-8, "
                    "|O| 4-32, 8 successors) and 2-D navigation (4-16 obstacles), "
                    "depth 4-12, budget = depth, n_p log-uniform 2^10-2^16",
        "instances": len(items),
        "particle_steps_per_batch": bsteps,
        "plain_sequential": {"value": steps / min(plain_s), "unit": "particle-steps/s",
                             "ms_per_batch": min(plain_s) * 1e3,
                             "plan_latency_ms": {"p50": percentile(plain_lat, 50),
                                                 "p99": percentile(plain_lat, 99)}},
        "batched_persistent": {"value": bsteps / min(batch_s), "unit": "particle-steps/s",
                               "ms_per_batch": min(batch_s) * 1e3,
                               "device_ms_per_batch": min(batch_dev),
                               "launches": 1},
        "batched_per_phase_graph": {"value": bsteps / min(phase_s), "unit": "particle-steps/s",
                                    "ms_per_batch": min(phase_s) * 1e3,
                                    "device_ms_per_batch": min(phase_dev),
                                    "launches": n_launches},
        "autotuned_mode": {V.BATCH_GRAPH: "per_phase_graph",
                           V.BATCH_PERSISTENT: "persistent"}.get(auto_mode),
        "speedup": min(plain_s) / min(min(batch_s), min(phase_s)),
        "results_identical_to_plain": bool(identical),
        "tuning": {"accum_cap": tuning[0], "backup_cap": tuning[1],
                   "blocks_per_cu": tuning[2], "forward_group": tuning[3],
                   "sweep_group": tuning[4]} if tuning else None,
    }
    batch.close()
    for it in items:
        it[0].close()
    if cpu:
        out["cpu_baseline"] = oracle_mix_baseline()
    return out


def bench_anytime(V, pom, belt, n_bel, n_p, depth, eta, budgets_ms=(10.0, 30.0, 100.0),
                  k_max=128, reps=3):
    """Anytime planning (Alg. 1's wall-clock budget) on the same workload:
    iterations reached, particle steps and the overshoot past the budget."""
    prm = V.params(n_p, eta=eta, seed=1)
    ws = V.Workspace(pom, prm, k_max, depth)
    V.plan_anytime(pom, belt, n_bel, k_max, depth, budgets_ms[0], prm, ws=ws)   # warm-up
    rows = []
    for b in budgets_ms:
        ks, steps, dev = [], [], []
        for i in range(reps):
            r, k = V.plan_anytime(pom, belt, n_bel, k_max, depth, b,
                                  V.params(n_p, eta=eta, seed=2000 + i), ws=ws)
            ks.append(k)
            steps.append(r.particle_steps)
            dev.append(r.device_ms)
        rows.append({"budget_ms": b, "iterations": ks, "particle_steps": steps,
                     "device_ms": [round(x, 3) for x in dev],
                     "max_overshoot_ms": round(max(d - b for d in dev), 3),
                     "particle_steps_per_s": sum(steps) / (sum(dev) * 1e-3)})
    ws.close()
    return {"k_max": k_max, "rows": rows,
            "note": "iteration k+1 starts only if the device wall clock shows less "
                    "than the budget since set-up; device_ms includes set-up and select"}


def bench_reroot(V, inst, pom, belt, n_bel, n_p, K, depth, eta, steps=6):
    """Closed-loop real steps (plan, act in a simulated environment, update the
    belief), once starting every plan from a fresh root (Alg. 1) and once
    keeping the subtree under the executed action and perceived observation
    (vopp_reroot).  Reports the re-rooting time, the kept beliefs and the plan
    times of both."""
    import torch
    out = {}
    for mode in ("fresh", "kept"):
        prm = V.params(n_p, eta=eta, seed=1)
        wss = [V.Workspace(pom, prm, K, depth), V.Workspace(pom, prm, K, depth)]
        parts = belt.clone()
        if inst["kind"] == "tabular":
            state = parts[:1].clone()
        else:
            state = torch.stack([parts[0], parts[n_bel]]).contiguous()
        plan_ms, reroot_ms, kept, tree = [], [], [], []
        for t in range(steps):
            ws = wss[t % 2]
            p_t = V.params(n_p, eta=eta, seed=3000 + t, step=t)
            r = V.plan(pom, parts, n_bel, K, depth, p_t, ws=ws)
            plan_ms.append(r.device_ms)
            tree.append(r.n_beliefs)
            obs, _, term = V.env_step(pom, state, r.action, 77, t)
            if term:
                break
            V.belief_update(pom, parts, n_bel, r.action, obs, 78, t)
            if mode == "kept" and t + 1 < steps:
                torch.cuda.synchronize()
                a = time.perf_counter()
                kept.append(V.reroot(pom, ws, r.action, obs,
                                     V.params(n_p, eta=eta, seed=3001 + t, step=t + 1),
                                     K, depth, wss[(t + 1) % 2]))
                reroot_ms.append((time.perf_counter() - a) * 1e3)
        for w in wss:
            w.close()
        row = {"plans": len(plan_ms), "plan_device_ms": [round(x, 3) for x in plan_ms],
               "tree_beliefs": tree}
        if mode == "kept":
            row.update(reroot_ms=[round(x, 3) for x in reroot_ms], kept_beliefs=kept)
        out[mode] = row
    out["note"] = ("kept: each plan starts from the subtree under the executed action "
                   "and perceived observation; reroot_ms is the host-timed vopp_reroot "
                   "call (scratch allocation and synchronisation included)")
    return out


def serve_trace(seed, qps, seconds, steps_per_episode):
    """Poisson episode starts at rate qps / steps (each episode then issues
    its requests back to back, so the offered load is about qps requests/s)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    rate = qps / steps_per_episode
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            return out
        out.append(t)


def bench_serve(V, I, qps_list=(250, 1000, 2500), seconds=5.0, steps_per_episode=50,
                deadline_ms=50.0, plain_max_qps=1000, phases_per_tick=32):
    """Continuous-batching server vs plain one-request-at-a-time planning on
    the same arrival trace of episodes drawn from the 256-instance mix."""
    import torch
    mix = I.batch_mix(0)
    poms = [V.Pomdp.from_instance(inst) for inst, _, _ in mix]

    def episode(j):
        inst, bel, p = mix[j % len(mix)]
        n_p = p["n_particles"]
        if inst["kind"] == "tabular":
            parts = (np.arange(n_p) % inst["nS"]).astype(np.int32)
            state = int((j * 7919) % inst["nS"])
            host = parts
        else:
            x, y = I.nav_belief(p["seed"] + j, n_p)
            host = np.concatenate([x, y])
            state = (1.0, 1.0)
        return dict(pom=poms[j % len(mix)], host=host, n_p=n_p, budget=p["budget"],
                    depth=p["depth"], seed=p["seed"] + 1000003 * j, env_seed=j + 1,
                    state=state, kind=inst["kind"])

    def stats(lat, steps, wall):
        lat = np.asarray(lat)
        return {"requests": int(lat.size), "p50_ms": percentile(lat, 50),
                "p99_ms": percentile(lat, 99),
                "deadline_miss_frac": float((lat > deadline_ms).mean()) if lat.size else None,
                "particle_steps_per_s": steps / wall}

    results = []
    for qps in qps_list:
        starts = serve_trace(17, qps, seconds, steps_per_episode)
        eps = [episode(j) for j in range(len(starts))]
        # Served: continuous batching.
        srv = V.Server(hbm_budget_bytes=64 << 30, max_active=512, max_inflight=3,
                       phases_per_tick=phases_per_tick)
        lat, steps = [], 0
        t0 = time.perf_counter()
        nxt = 0
        while True:
            now = time.perf_counter() - t0
            while nxt < len(starts) and starts[nxt] <= now:
                e = eps[nxt]
                srv.submit(e["pom"], e["host"], e["budget"], e["depth"],
                           V.params(e["n_p"], seed=e["seed"]), e["state"], e["env_seed"],
                           steps_per_episode)
                nxt += 1
            pending = srv.tick()
            for r in srv.poll():
                lat.append((r["done_s"] - r["arrival_s"]) * 1e3)
                steps += r["particle_steps"]
            if pending == 0 and nxt >= len(starts):
                break
            if pending == 0:
                time.sleep(max(0.0, min(starts[nxt] - (time.perf_counter() - t0), 0.01)))
        served = stats(lat, steps, time.perf_counter() - t0)
        srv.close()
        if qps > plain_max_qps:
            # The plain path saturates below this load (its queue only grows),
            # so it is not run here.
            results.append({"offered_qps": qps, "episodes": len(starts),
                            "served_continuous_batching": served,
                            "plain_one_at_a_time": None})
            continue
        # Plain: one request at a time (plan, then environment step and belief
        # update), first come first served over the same trace.
        import heapq
        t0 = time.perf_counter()
        heap = [(starts[j], j, 0) for j in range(len(starts))]
        heapq.heapify(heap)
        dev = {}
        lat, steps = [], 0
        while heap:
            arr, j, t = heapq.heappop(heap)
            now = time.perf_counter() - t0
            if arr > now:
                time.sleep(arr - now)
            e = eps[j]
            if j not in dev:
                parts = torch.as_tensor(e["host"], device="cuda")
                st = (torch.tensor([e["state"]], dtype=torch.int32, device="cuda")
                      if e["kind"] == "tabular" else
                      torch.tensor(e["state"], dtype=torch.float32, device="cuda"))
                dev[j] = (parts, st)
            parts, st = dev[j]
            if t > 0:
                obs, _, _ = V.env_step(e["pom"], st, e["last"], e["env_seed"], t - 1)
                V.belief_update(e["pom"], parts, e["n_p"], e["last"], obs, e["seed"], t - 1)
            r = V.plan(e["pom"], parts, e["n_p"], e["budget"], e["depth"],
                       V.params(e["n_p"], seed=e["seed"], step=t))
            e["last"] = r.action
            done = time.perf_counter() - t0
            lat.append((done - arr) * 1e3)
            steps += r.particle_steps
            if t + 1 < steps_per_episode:
                heapq.heappush(heap, (done, j, t + 1))
            else:
                del dev[j]
        plain = stats(lat, steps, time.perf_counter() - t0)
        results.append({"offered_qps": qps, "episodes": len(starts),
                        "served_continuous_batching": served,
                        "plain_one_at_a_time": plain})
    for p in poms:
        p.close()
    return {"workload": f"episodes drawn from the 256-instance mix, {steps_per_episode} "
                        f"steps each, Poisson episode starts for {seconds:.0f} s, belief "
                        "particles and tree workspaces resident (each step plans a fresh "
                        "tree), 64 GiB HBM admission budget, "
                        f"{deadline_ms:.0f} ms per-step deadline",
            "phases_per_tick": phases_per_tick,
            "sweep": results}


def bench_plain(V, I, name, steps, warmup, event_profile, cpu):
    """Plain single-instance plans of one workload: throughput, latency, the
    dominant kernel against the HBM roofline and the oracle on the host."""
    import torch
    inst, bel, p = I.workload(name, seed=0)
    n_p, K, depth, eta = p["n_particles"], p["budget"], p["depth"], p["eta"]
    pom = V.Pomdp.from_instance(inst)
    prm = V.params(n_p, eta=eta, seed=1)
    ws = V.Workspace(pom, prm, K, depth)
    belt = V.belief_tensor(inst, bel)
    n_bel = belt.numel() if inst["kind"] == "tabular" else belt.numel() // 2
    stream = torch.cuda.current_stream()
    # Warm-up plans; the last one brackets every kernel kind with events to
    # find the kind that dominates device time.
    dom = None
    warm_share = None
    for i in range(warmup):
        if event_profile and i == warmup - 1:
            V.profile_reset(ws)
            V.profile_enable(ws, None)
        V.plan(pom, belt, n_bel, K, depth, V.params(n_p, eta=eta, seed=100 + i),
               ws=ws, stream=stream)
    if event_profile and warmup > 0:
        warm = V.profile_read(ws)
        dom = max((k for k in warm if k != "setup"), key=lambda k: warm[k][0])
        warm_total = sum(v[0] for v in warm.values())
        warm_share = {k: v[0] / warm_total for k, v in warm.items() if v[1]}
    # Timed region: plain plans, no event brackets.
    V.profile_enable(ws, [])
    torch.cuda.synchronize()
    lat, dev_ms, results = [], [], []
    total_steps = 0
    t0 = time.perf_counter()
    for i in range(steps):
        a = time.perf_counter()
        r = V.plan(pom, belt, n_bel, K, depth, V.params(n_p, eta=eta, seed=1000 + i),
                   ws=ws, stream=stream)
        lat.append((time.perf_counter() - a) * 1e3)
        dev_ms.append(r.device_ms)
        results.append(r)
        total_steps += r.particle_steps
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    counts = V.level_counts(ws)              # beliefs per level step, last plan
    # The dominant kind's launches timed by their own dispatch (start and end
    # events taken by hipExtLaunchKernel on the plan stream), over the same
    # plans run again, so that the timed region carries no profiling.
    prof = None
    if dom is not None:
        V.profile_reset(ws)
        V.profile_enable(ws, [dom])
        for i in range(steps):
            V.plan(pom, belt, n_bel, K, depth, V.params(n_p, eta=eta, seed=1000 + i),
                   ws=ws, stream=stream)
        torch.cuda.synchronize()
        prof = V.profile_read(ws)
        V.profile_enable(ws, [])
    out = {
        "value": total_steps / elapsed,
        "unit": "particle-steps/s",
        "ms_per_step": elapsed * 1e3 / steps,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "device_p50": percentile(dev_ms, 50)},
        "particle_steps_per_plan": total_steps / steps,
        "near_ties_per_plan": float(np.mean([r.near_ties for r in results])),
    }
    if prof is not None:
        kinds = {k: v for k, v in prof.items() if v[1] > 0}
        out["kernel_share_warmup"] = warm_share
        roof = {"kernel": dom, "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "traffic": None}
        # Method bytes summed over the timed plans (each plan's own tree).
        leaf = leaf_sweep_visits(n_p, K, depth, counts)
        per = [method_bytes(name, pom.nA, r.particle_steps, r.n_beliefs, r.n_actions,
                            r.sweep, leaf) for r in results]
        total = {k: sum(x[k] for x in per) for k in per[0]}
        if dom in total:
            ms, launches = kinds[dom]
            achieved = total[dom] / (ms * 1e-3) / 1e9
            roof.update(achieved=achieved, frac=achieved / HBM_PEAK_GBS,
                        launches_per_plan=launches // steps,
                        avg_launch_us=ms * 1e3 / launches,
                        bytes_per_launch=total[dom] / launches,
                        bytes_per_plan=total[dom] / steps,
                        byte_model="the method's bytes per unit of work (per particle "
                                   "step, new node, belief and action-node visit) "
                                   "times the units each timed plan counted",
                        timing="start and end timestamps of each launch's own dispatch "
                               "(HIP events taken by hipExtLaunchKernel on the plan stream), "
                               "over the timed plans run again")
            if dom == "backup_level":
                sw = [sum(r.sweep[i] for r in results) / launches for i in range(3)]
                roof["units_per_launch"] = {"belief_visits": sw[0],
                                            "internal_belief_visits": sw[1],
                                            "action_node_visits": sw[2]}
                lay = sum(layout_bytes_backup_level(pom.nA, r.sweep) for r in results)
                roof["layout_bytes_per_launch"] = lay / launches
            tr = MEASURED_TRAFFIC.get(dom, {}).get(name)
            if tr is not None and kernel_sources_hash() == MEASURED_TRAFFIC["sources_sha256_16"]:
                roof["traffic"] = tr
                roof["traffic_calibration"] = "plain device copy (FETCH_SIZE x 2, WRITE_SIZE x 1)"
                roof["traffic_GBs"] = tr / (ms * 1e-3 / launches) / 1e9
                roof["traffic_over_method_bytes"] = tr / (total[dom] / launches)
                tg = MEASURED_TRAFFIC["gather_scale"].get(dom, {}).get(name)
                if tg is not None:
                    roof["traffic_gather_calibration"] = tg
                    roof["traffic_gather_over_method_bytes"] = tg / (total[dom] / launches)
        else:
            roof.update(achieved=None, frac=None,
                        note=f"dominant kernel {dom} has no byte model")
        out["roofline"] = roof
    ws.close()
    pom.close()
    if cpu:
        out["cpu_baseline"] = cpu_baseline(inst, bel, p)
    out["_inputs"] = (inst, bel, p)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nav2d",
                    choices=["nav2d", "sparse4096", "tabular16", "mars625", "mars3025"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-event-profile", action="store_true",
                    help="skip the event-bracketed plans (kernel shares in the last "
                         "warm-up plan, the dominant kernel's timing after the timed "
                         "region); the roofline is then left out")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 256-instance batched vs plain comparison")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the sparse4096 line that follows the nav2d headline")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served (continuous batching) vs plain comparison")
    ap.add_argument("--no-anytime", action="store_true",
                    help="skip the wall-clock-budget (anytime) planning report")
    ap.add_argument("--no-reroot", action="store_true",
                    help="skip the closed-loop tree re-rooting report")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) to "
                         "calibrate HBM traffic counters, then exit")
    ap.add_argument("--gather-calibration", type=int, default=0, metavar="MROWS",
                    help="only gather MROWS million random 16-byte rows of a 1 GiB "
                         "table (5 times), a scattered-access calibration of the "
                         "traffic counters, then exit")
    args = ap.parse_args()

    if args.gather_calibration:
        import torch
        rows = (1 << 30) // 16
        n = args.gather_calibration * 1000000
        table = torch.ones((rows, 4), dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        idx = torch.randint(0, rows, (n,), device="cuda", generator=g)
        out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        for _ in range(5):
            torch.index_select(table, 0, idx, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"gather_calibration_rows": n, "row_bytes": 16,
                          "table_bytes": rows * 16, "gathers": 5}), flush=True)
        return

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 5}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the "
                          "planner has no multi-GPU path (independent instances "
                          "would be shared out across GPUs by HBM footprint)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(3)
    from paper_2510_27191_amd import instances as I
    from paper_2510_27191_amd import vopp as V

    WORKLOADS = {
        "nav2d": "continuous 2-D navigation POMDP, 8 obstacle disks, 0.5-grid "
                 "observation keys, n_p=65536, depth 10, budget 10 iterations",
        "sparse4096": "sparse tabular POMDP |S|=4096 |A|=8 |O|=32, 8 successors, "
                      "n_p=262144, depth 8, budget 8 iterations",
        "tabular16": "tabular POMDP |S|=16 |A|=3 |O|=4, n_p=1024, depth 4, budget 4",
        "mars625": "MARS-shaped tabular POMDP |S|=2048 |A|=625 |O|=9, 4 successors, "
                   "n_p=16384, depth 4, budget 4 iterations",
        "mars3025": "MARS-shaped tabular POMDP |S|=512 |A|=3025 |O|=9, 4 successors, "
                    "n_p=16384, depth 4, budget 4 iterations",
    }

    def config_of(name, inst, p):
        return {"workload": f"{name}: {WORKLOADS[name]}", "n_particles": p["n_particles"],
                "budget": p["budget"], "depth": p["depth"], "eta": p["eta"],
                "gamma": inst["gamma"], "schedule": "deepening",
                "parallelism": "single GPU"}

    head = bench_plain(V, I, args.workload, args.steps, args.warmup,
                       not args.no_event_profile, not args.no_cpu_baseline)
    inst, bel, p = head.pop("_inputs")
    out = {
        "metric": "particle-steps/s at fixed budget; p50/p99 plan latency, batched vs plain",
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded instance generators; no dataset)",
        "config": config_of(args.workload, inst, p),
    }
    out.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step")})
    # The large sparse tabular workload as its own line (same fields).
    if args.workload == "nav2d" and not args.no_sparse:
        sub = bench_plain(V, I, "sparse4096", args.steps, args.warmup,
                          not args.no_event_profile, not args.no_cpu_baseline)
        s_inst, _, s_p = sub.pop("_inputs")
        sub["config"] = config_of("sparse4096", s_inst, s_p)
        out["sparse4096"] = sub
    n_p, K, depth, eta = p["n_particles"], p["budget"], p["depth"], p["eta"]
    pom = V.Pomdp.from_instance(inst)
    belt = V.belief_tensor(inst, bel)
    n_bel = belt.numel() if inst["kind"] == "tabular" else belt.numel() // 2
    if not args.no_anytime:
        out["anytime"] = bench_anytime(V, pom, belt, n_bel, n_p, depth, eta)
    if not args.no_reroot:
        out["reroot"] = bench_reroot(V, inst, pom, belt, n_bel, n_p, K, depth, eta)
    pom.close()
    if not args.no_batch:
        out["batched_vs_plain"] = bench_batch(V, I, cpu=not args.no_cpu_baseline)
    if not args.no_serve:
        out["served_vs_plain"] = bench_serve(V, I, seconds=args.serve_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
