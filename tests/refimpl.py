"""Independent pure-Python constructions that pin the oracle.

None of this imports the oracle or the GPU path.  Each function is a second,
separately written route to a quantity the oracle also computes:

* ``philox``            - Philox4x32-10 from its published round function.
* ``thresholds``        - the integer CDF thresholds of a categorical row.
* ``replay_first``      - the tree built by iteration 1 (every preference row
                          still uniform), episode by episode, keyed by
                          action/observation histories.
* ``k1_values``         - Alg. 3 run once on that tree (one iteration).
* ``ref_bellman``       - the reference-based Bellman recursion of Eq. (3)-(4)
                          on exact Bayes beliefs (belief vectors, no tree).
* ``soft_vi``           - KL-regularised finite-horizon value iteration on the
                          fully observed MDP.
* ``fluid_plan``        - Alg. 1-3 with episode counts replaced by probability
                          mass flowing through every branch: the limit of the
                          method as n_p -> infinity.
"""

from __future__ import annotations

import math

import numpy as np

MASK = 0xFFFFFFFF
TWO31 = 2 ** 31


def philox(c, k):
    c0, c1, c2, c3 = (int(v) & MASK for v in c)
    k0, k1 = (int(v) & MASK for v in k)
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & MASK
            k1 = (k1 + 0xBB67AE85) & MASK
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = (((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK,
                          ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK)
    return c0, c1, c2, c3


def draw(seed, ep, tag, level, it, step):
    return philox((ep, (tag << 24) | level, it, step),
                  (seed & MASK, (seed >> 32) & MASK))


def thresholds(p):
    p = np.asarray(p, np.float32).astype(np.float64)
    cum = np.cumsum(p)                       # sequential running sum
    total = cum[-1]
    thr = np.rint(cum / total * float(TWO31))
    thr = np.clip(thr, 0, TWO31)
    thr[-1] = TWO31
    return thr.astype(np.int64)


def threshold_probs(p):
    t = thresholds(p)
    return np.diff(np.concatenate([[0], t])) / float(TWO31)


def pick(thr, x):
    u = (int(x) & MASK) >> 1
    for j, t in enumerate(thr):
        if u < t:
            return j
    return len(thr) - 1


def uniform_row_action(x0, A):
    """Action drawn from a uniform preference row by Eq. (6): the running sums
    are 1, 2, ..., |A| and t = u |A| with u = (x0 >> 8) 2^-24, so the first j
    with t < j + 1 is floor(u |A|), computed here in integers."""
    return min(((int(x0) >> 8) * A) >> 24, A - 1)


def root_probs(M):
    """Probability of each of M belief particles under idx = (x*M) >> 32."""
    edges = [-((-i * 2 ** 32) // M) for i in range(M + 1)]   # ceil(i 2^32 / M)
    return np.diff(np.asarray(edges, dtype=np.float64)) / 2.0 ** 32


# ---------------------------------------------------------------------------
# Models.
# ---------------------------------------------------------------------------

class Tabular:
    def __init__(self, inst):
        self.inst = inst
        self.nS, self.nA, self.nO = inst["nS"], inst["nA"], inst["nO"]
        rp, col, tp = inst["rowptr"], inst["col"], inst["tprob"]
        self.rows = []
        for r in range(self.nS * self.nA):
            lo, hi = int(rp[r]), int(rp[r + 1])
            self.rows.append((col[lo:hi].astype(np.int64), thresholds(tp[lo:hi]),
                              threshold_probs(tp[lo:hi])))
        Z = np.asarray(inst["zprob"], np.float32).reshape(self.nS, self.nA, self.nO)
        self.zthr = [[thresholds(Z[s, a]) for a in range(self.nA)]
                     for s in range(self.nS)]
        self.Zp = np.array([[threshold_probs(Z[s, a]) for a in range(self.nA)]
                            for s in range(self.nS)])
        self.R = np.asarray(inst["reward"], np.float32).reshape(self.nS, self.nA)
        h = inst.get("heur")
        self.H = (np.zeros(self.nS, np.float32) if h is None
                  else np.asarray(h, np.float32))
        self.gamma = inst["gamma"]
        T = np.zeros((self.nS, self.nA, self.nS))
        for s in range(self.nS):
            for a in range(self.nA):
                cols, _, pr = self.rows[s * self.nA + a]
                for c, q in zip(cols, pr):
                    T[s, a, c] += q
        self.T = T

    def step(self, s, a, w):
        cols, thr, _ = self.rows[s * self.nA + a]
        sn = int(cols[pick(thr, w[1])])
        o = pick(self.zthr[sn][a], w[2])
        return sn, o, float(self.R[s, a]), False

    def h(self, s):
        return float(self.H[s])


class Nav:
    def __init__(self, inst):
        self.p = inst
        self.g = np.asarray(inst["gauss"], np.float32)
        self.disks = np.asarray(inst["disks"], np.float32).reshape(-1, 2)
        self.gamma = inst["gamma"]
        self.nA = 4

    def _axis(self, v):
        f = np.float32
        p = self.p
        c = np.floor(f(v) * f(p["inv_bin"]))
        c = min(max(c, f(p["key_lo"])), f(p["key_lo"] + p["key_n"] - 1))
        return int(c) - p["key_lo"]

    def step(self, s, a, w):
        f = np.float32
        p = self.p
        x, y = s
        dx = [f(0), f(p["step"]), f(0), -f(p["step"])][a]
        dy = [f(p["step"]), f(0), -f(p["step"]), f(0)][a]
        zx = self.g[w[1] >> 20]
        zy = self.g[(w[1] >> 8) & 4095]
        mx = f(x) + dx
        my = f(y) + dy
        nx = min(max(f(mx + f(p["sigma_move"]) * zx), f(p["lo"])), f(p["hi"]))
        ny = min(max(f(my + f(p["sigma_move"]) * zy), f(p["lo"])), f(p["hi"]))
        sd = f(p["sigma_obs0"]) + f(p["sigma_obs_slope"]) * abs(f(nx - f(p["obs_center_x"])))
        ox = f(nx + f(sd * self.g[w[2] >> 20]))
        oy = f(ny + f(sd * self.g[(w[2] >> 8) & 4095]))
        key = self._axis(ox) * p["key_n"] + self._axis(oy)
        gx = f(nx - f(p["goal_x"]))
        gy = f(ny - f(p["goal_y"]))
        goal = bool(f(gx * gx) + f(gy * gy) <= f(p["goal_r2"]))
        hit = False
        for cx, cy in self.disks:
            ex = f(nx - cx)
            ey = f(ny - cy)
            if f(ex * ex) + f(ey * ey) <= f(p["disk_r2"]):
                hit = True
        r = f(p["r_step"])
        if goal:
            r = f(r + f(p["r_goal"]))
        if hit:
            r = f(r + f(p["r_hit"]))
        return (nx, ny), key, float(r), goal

    def h(self, s):
        if self.p["heuristic"] == 0:
            return 0.0
        f = np.float32
        return float(-(abs(f(s[0] - f(self.p["goal_x"]))) +
                       abs(f(s[1] - f(self.p["goal_y"])))))


def model_of(inst):
    return Tabular(inst) if inst["kind"] == "tabular" else Nav(inst)


# ---------------------------------------------------------------------------
# Iteration-1 replay: every preference row is uniform, so each draw is fixed
# by its random word alone.  Histories key the nodes; new nodes take the next
# row in ascending episode order at each level.
# ---------------------------------------------------------------------------

def replay_first(inst, belief, n_p, D, seed, step=0, k=1):
    mdl = model_of(inst)
    A = mdl.nA
    if inst["kind"] == "tabular":
        bel = np.asarray(belief)
        M = bel.size
        get = lambda i: int(bel[i])
    else:
        bx, by = belief
        M = len(bx)
        get = lambda i: (np.float32(bx[i]), np.float32(by[i]))
    beliefs = {(): 0}
    b_rows = [dict(parent=-1, obs=-1, depth=0)]
    acts = {}
    a_rows = []
    eps = []
    for ep in range(n_p):
        w = draw(seed, ep, 1, 0, k, step)
        idx = (w[0] * M) >> 32
        eps.append(dict(ep=ep, s=get(idx), hist=(), alive=True))
    steps = 0
    for d in range(D):
        for e in eps:
            if not e["alive"]:
                continue
            w = draw(seed, e["ep"], 2, d, k, step)
            a = uniform_row_action(w[0], A)
            sn, o, r, term = mdl.step(e["s"], a, w)
            steps += 1
            key = (e["hist"], a)
            if key not in acts:
                acts[key] = len(a_rows)
                a_rows.append(dict(parent=beliefs[e["hist"]], act=a, C=0.0, N=0,
                                   depth=d))
            an = acts[key]
            a_rows[an]["C"] += r
            a_rows[an]["N"] += 1
            if term:
                e["alive"] = False
                continue
            hist = e["hist"] + (a, o)
            if hist not in beliefs:
                beliefs[hist] = len(b_rows)
                b_rows.append(dict(parent=an, obs=o, depth=d + 1))
            e["hist"] = hist
            e["s"] = sn
    leaves = {}
    for e in eps:
        if e["alive"]:
            b = beliefs[e["hist"]]
            c, s = leaves.get(b, (0, 0.0))
            leaves[b] = (c + 1, s + mdl.h(e["s"]))
    return dict(b_rows=b_rows, a_rows=a_rows, leaves=leaves, steps=steps, A=A,
                gamma=mdl.gamma)


def lse(x, eta):
    x = np.asarray(x, np.float64)
    m = x.max()
    return m + math.log(np.exp(eta * (x - m)).sum()) / eta


def k1_values(rep, eta):
    """One backup (Alg. 3) over the iteration-1 tree: node values, Psi rows."""
    A, gamma = rep["A"], rep["gamma"]
    nb, na = len(rep["b_rows"]), len(rep["a_rows"])
    psi0 = -math.log(A) / eta
    psi = np.full((nb, A), psi0)
    V = np.zeros(nb)
    Nb = np.zeros(nb, np.int64)
    for b, (c, s) in rep["leaves"].items():
        Nb[b] = c
        V[b] = s / c
    depth_b = np.array([r["depth"] for r in rep["b_rows"]])
    children = {}
    for b, r in enumerate(rep["b_rows"]):
        if r["parent"] >= 0:
            children.setdefault(r["parent"], []).append(b)
    by_belief = {}
    for an, r in enumerate(rep["a_rows"]):
        by_belief.setdefault(r["parent"], []).append(an)
    D = depth_b.max()
    for d in range(D, 0, -1):
        for b in np.nonzero(depth_b == d - 1)[0]:
            ans = by_belief.get(int(b), [])
            if not ans:
                continue
            vc = lse(psi[b], eta)
            for an in ans:
                r = rep["a_rows"][an]
                w = sum(V[c] * Nb[c] for c in children.get(an, []))
                q = r["C"] / r["N"] + gamma * (w / r["N"])
                psi[b, r["act"]] = psi[b, r["act"]] - vc + q
            Nb[b] = sum(rep["a_rows"][an]["N"] for an in ans)
            V[b] = lse(psi[b], eta)
    return psi, V, Nb


# ---------------------------------------------------------------------------
# Exact reference-based Bellman recursion (Eq. 3-4) on Bayes beliefs.
# ---------------------------------------------------------------------------

def ref_bellman(inst, b0, depth, eta, pi0=None):
    """The reference-based Bellman recursion of Eq. (3)-(4) on exact Bayes
    beliefs: V(b) = L_eta[(1/eta) log pi0 + R(b, .) + gamma E_o V(tau(b, ., o))]."""
    mdl = Tabular(inst)
    A = mdl.nA
    if pi0 is None:
        logpi0 = -math.log(A)
    else:
        pi = np.asarray(pi0, np.float64)
        logpi0 = np.log(pi / pi.sum())

    def V(b, d):
        if d == depth:
            return float(b @ mdl.H.astype(np.float64))
        qs = []
        for a in range(A):
            r = float(b @ mdl.R[:, a].astype(np.float64))
            pred = b @ mdl.T[:, a, :]
            joint = pred[:, None] * mdl.Zp[:, a, :]
            po = joint.sum(0)
            fut = 0.0
            for o in range(mdl.nO):
                if po[o] > 0:
                    fut += po[o] * V(joint[:, o] / po[o], d + 1)
            qs.append(r + mdl.gamma * fut)
        qs = np.array(qs)
        return lse(logpi0 / eta + qs, eta)

    return V(np.asarray(b0, np.float64), 0)


def soft_vi(inst, b0, depth, eta):
    """Fully observed case: KL-regularised value iteration, horizon ``depth``."""
    mdl = Tabular(inst)
    A, nS = mdl.nA, mdl.nS
    R = mdl.R.astype(np.float64)
    Vt = mdl.H.astype(np.float64).copy()
    for _ in range(depth - 1):
        Q = R + mdl.gamma * np.einsum("sat,t->sa", mdl.T, Vt)
        Vt = np.array([np.log(np.mean(np.exp(eta * Q[s]))) / eta for s in range(nS)])
    b0 = np.asarray(b0, np.float64)
    q0 = b0 @ R + mdl.gamma * np.einsum("s,sat,t->a", b0, mdl.T, Vt)
    return float(np.log(np.mean(np.exp(eta * q0))) / eta)


# ---------------------------------------------------------------------------
# Expected-count (fluid) Alg. 1-3 on a tabular POMDP.
# ---------------------------------------------------------------------------

def fluid_plan(inst, b0, K, depth, eta, schedule=0):
    mdl = Tabular(inst)
    A, gamma = mdl.nA, mdl.gamma
    R = mdl.R.astype(np.float64)
    H = mdl.H.astype(np.float64)
    psi0 = -math.log(A) / eta
    bel = {(): dict(psi=np.full(A, psi0), V=0.0, Nb=0.0, depth=0)}
    act = {}
    for k in range(1, K + 1):
        D = depth if schedule == 1 else min(k, depth)
        frontier = {(): np.asarray(b0, np.float64)}
        for d in range(D):
            nxt = {}
            for hist, m in frontier.items():
                node = bel[hist]
                z = eta * (node["psi"] - node["psi"].max())
                pi = np.exp(z) / np.exp(z).sum()
                for a in range(A):
                    ma = m * pi[a]
                    tot = ma.sum()
                    if tot <= 0:
                        continue
                    an = act.setdefault((hist, a), dict(C=0.0, N=0.0, depth=d))
                    an["C"] += float(ma @ R[:, a])
                    an["N"] += tot
                    joint = (ma @ mdl.T[:, a, :])[:, None] * mdl.Zp[:, a, :]
                    for o in range(mdl.nO):
                        col = joint[:, o]
                        if col.sum() <= 0:
                            continue
                        ch = hist + (a, o)
                        if ch not in bel:
                            bel[ch] = dict(psi=np.full(A, psi0), V=0.0, Nb=0.0,
                                           depth=d + 1)
                        nxt[ch] = nxt.get(ch, 0.0) + col
            frontier = nxt
        for hist, m in frontier.items():
            bel[hist]["Nb"] = m.sum()
            bel[hist]["V"] = float(m @ H) / m.sum()
        for d in range(D, 0, -1):
            W = {}
            for hist, node in bel.items():
                if node["depth"] == d:
                    key = (hist[:-2], hist[-2])
                    W[key] = W.get(key, 0.0) + node["V"] * node["Nb"]
            for hist, node in bel.items():
                if node["depth"] != d - 1:
                    continue
                mine = [(a, act[(hist, a)]) for a in range(A) if (hist, a) in act]
                if not mine:
                    continue
                vc = lse(node["psi"], eta)
                for a, an in mine:
                    q = an["C"] / an["N"] + gamma * (W.get((hist, a), 0.0) / an["N"])
                    node["psi"][a] = node["psi"][a] - vc + q
                node["Nb"] = sum(an["N"] for _, an in mine)
                node["V"] = lse(node["psi"], eta)
    root = bel[()]
    return root["psi"].copy(), root["V"]


# ---------------------------------------------------------------------------
# Between real steps: true environment and SIR belief update.
# ---------------------------------------------------------------------------

def env_step(inst, state, a, seed, step):
    mdl = model_of(inst)
    w = philox((0, 4 << 24, 0, step), (seed & MASK, (seed >> 32) & MASK))
    return mdl.step(state, a, w)


def nav_cell_count(mdl, v, sd, k):
    f = np.float32
    g = mdl.g
    return sum(1 for j in range(4096) if mdl._axis(f(f(v) + f(f(sd) * g[j]))) == k)


def pf_update(inst, particles, a, o, seed, step):
    """Propagate, weight by the exact integer likelihood, resample
    multinomially with 64-bit uniforms."""
    mdl = model_of(inst)
    key = (seed & MASK, (seed >> 32) & MASK)
    n = len(particles)
    moved, cum = [], []
    total = 0
    for i in range(n):
        w = philox((i, 5 << 24, 0, step), key)
        if inst["kind"] == "tabular":
            s = int(particles[i])
            cols, thr, _ = mdl.rows[s * mdl.nA + a]
            sn = int(cols[pick(thr, w[1])])
            zt = mdl.zthr[sn][a]
            wt = int(zt[o]) - (int(zt[o - 1]) if o > 0 else 0)
            moved.append(sn)
        else:
            (nx, ny), _, _, _ = mdl.step(particles[i], a, (0, w[1], 0, 0))
            f = np.float32
            p = mdl.p
            sd = f(f(p["sigma_obs0"]) + f(f(p["sigma_obs_slope"]) *
                                          abs(f(nx - f(p["obs_center_x"])))))
            kn = p["key_n"]
            wt = nav_cell_count(mdl, nx, sd, o // kn) * nav_cell_count(mdl, ny, sd, o % kn)
            moved.append((nx, ny))
        total += wt
        cum.append(total)
    if total == 0:
        return moved, 0
    out = []
    for j in range(n):
        y = philox((j, 6 << 24, 0, step), key)
        u = (y[0] << 32) | y[1]
        target = (u * total) >> 64
        i = next(k for k, c in enumerate(cum) if c > target)
        out.append(moved[i])
    return out, total
