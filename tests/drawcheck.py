"""Draw-by-draw parity of the HIP planner with the oracle (test infrastructure).

The action draw of Eq. (6) is decided by floating point: the kernels keep
non-root preference rows in single precision, the oracle in double.  A draw
whose position t = u * P_last lies close to a boundary P_j of the running sums
can therefore go either way.  The protocol:

1. The oracle plans first and exports every draw (action, observation key)
   by (level step, episode), flagging near ties with the screen
       |t - P_j| <= (TAU + TAU_PSI * eta * max_j |Psi_j|) * P_last.
   The kernels take single-precision weights exp(eta (psi_j - max)) and sum
   them in double precision (rows of more than 64 actions: quads of four
   weights summed in double and rounded once to single precision, then
   scanned in double).  TAU covers the single-precision exponential (about
   one unit of 2^-24 of each weight) and the quad rounding (one unit of 2^-24
   of each quad sum): every running sum and t move by at most a few units of
   2^-24 of P_last.  TAU_PSI covers the single-precision preference rows
   themselves: if a row computed in single precision over K backups differs
   from the double one by at most E units of 2^-24 of its largest entry
   |Psi|max, every weight moves by at most 2 eta E 2^-24 |Psi|max (relative;
   the entry and the row maximum each move), every running sum and t by that
   much of P_last, and the decision by twice that: TAU_PSI = 4 E 2^-24.  The
   GPU tests measure E on every plan (psi_row_ulps): at most 8.2 on the
   benchmark shapes, so E = 16 (TAU_PSI = 2^-18) leaves a factor of two.
2. The GPU plans through vopp_plan_trace with the oracle's decision forced at
   exactly the flagged draws (the oracle never reads anything from the GPU),
   and exports its own decision at every draw.
3. Every unflagged GPU decision must equal the oracle's, the same episodes
   must be alive at every level step, and every observation key must match.
   The flagged draws where the GPU's own decision differs are counted (the
   follow count).
4. The two trees must then match: structure bit for bit, values within
   1e-4 * max(|oracle|, 1).
"""

import numpy as np

TAU = 2.0 ** -21
TAU_PSI = 2.0 ** -18
PSI_ULPS_MAX = 16.0          # the E that TAU_PSI = 4 E 2^-24 assumes
REL = 1e-4


def screen(inst):
    """Near-tie screen (tau, tau_psi, tau_abs) of the oracle for this model."""
    return dict(tau=TAU, tau_psi=TAU_PSI, tau_abs=0.0)


def oracle_plan(orc, inst, belief, n_p, K, depth, **kw):
    """The oracle's plan with its per-draw export under the screen."""
    return orc.plan(inst, belief, n_p, K, depth, draws=True, **screen(inst), **kw)


def force_array(o):
    """int16 [level steps * n_p]: the oracle's action at flagged draws, else -1."""
    dr = o.draws
    near = (dr["flags"] & 4) != 0
    return np.where(near, dr["act"], -1).astype(np.int16)


def check_draws(o, act, obs):
    """Compare the GPU's own decisions with the oracle's.  Returns
    (follow count, flagged draws, draws)."""
    dr = o.draws
    oa = dr["act"].reshape(act.shape)
    oo = dr["obs"].reshape(act.shape)
    fl = dr["flags"].reshape(act.shape)
    drawn = (fl & 1) != 0
    near = (fl & 4) != 0
    assert np.array_equal(act >= 0, drawn), "different episodes alive"
    free = drawn & ~near
    bad = np.nonzero(free & (act != oa))
    assert bad[0].size == 0, (
        "unflagged draws differ at (level step, episode) "
        f"{list(zip(bad[0][:5].tolist(), bad[1][:5].tolist()))}, {bad[0].size} in all")
    assert np.array_equal(obs[drawn], oo[drawn]), "observation keys differ"
    follow = int((near & (act != oa)).sum())
    return follow, int(near.sum()), int(drawn.sum())


def close(a, b, rel=REL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    tol = rel * np.maximum(np.abs(b), 1.0)
    bad = np.abs(a - b) > tol
    return (not bad.any()), (np.max(np.abs(a - b) / tol) if a.size else 0.0)


def assert_tree_parity(res, tree, o, A):
    """Structure bit for bit, values within REL (rows in canonical order)."""
    from tests.treecanon import canonical_tree
    assert res.n_beliefs == len(o.b_parent)
    assert res.n_actions == len(o.a_parent)
    assert res.particle_steps == o.particle_steps
    oc = canonical_tree(o)
    for k in ("b_parent", "b_obs", "b_depth", "a_parent", "a_act"):
        assert np.array_equal(tree[k], oc[k]), k
    assert np.array_equal(tree["a_N"], oc["a_N"])
    assert np.array_equal(tree["b_N"], oc["b_N"])
    ok, worst = close(tree["a_C"], oc["a_C"])
    assert ok, ("a_C", worst)
    ok, worst = close(tree["psi"][1:], oc["psi"][1:])
    assert ok, ("psi", worst)
    ok, worst = close(tree["b_V"][1:], oc["b_V"][1:])
    assert ok, ("b_V", worst)
    ok, worst = close(res.values, o.psi_root)
    assert ok, ("root psi", worst)
    ok, worst = close([res.v_root], [o.v_root])
    assert ok, ("v_root", worst)
    srt = np.sort(o.psi_root)[::-1]
    if A > 1 and srt[0] - srt[1] > REL * max(abs(srt[0]), 1.0):
        assert res.action == o.action
    else:
        assert res.action in np.nonzero(o.psi_root >= srt[0] - REL * max(abs(srt[0]), 1.0))[0]
    return oc


def gpu_forced_plan(V, pom, ws, inst, belief_dev, n_belief, n_p, K, depth, o, seed=1,
                    schedule=0, eta=1.0, step=0):
    """vopp_plan_trace with the oracle's flagged draws forced; returns
    (result, tree, own actions, observation keys)."""
    prm = V.params(n_p, eta=eta, seed=seed, schedule=schedule, step=step)
    res, act, obs = V.plan_trace(pom, belief_dev, n_belief, K, depth, prm, ws=ws,
                                 force=force_array(o))
    tree = V.tree_dump(ws, pom.nA, res.n_beliefs, res.n_actions)
    return res, tree, act, obs


def forced_parity(V, orc, inst, belief, n_p, K, depth, seed=1, schedule=0, eta=1.0,
                  step=0, pi0=None, max_flag_frac=0.02):
    """The whole protocol on a fresh model and workspace.  Returns a dict of
    draw statistics (follow, flagged, draws) and the two results."""
    o = oracle_plan(orc, inst, belief, n_p, K, depth, eta=eta, seed=seed,
                    schedule=schedule, step=step, pi0=pi0)
    pom = V.Pomdp.from_instance(inst)
    try:
        if pi0 is not None:
            pom.set_reference_policy(pi0)
        prm = V.params(n_p, eta=eta, seed=seed, schedule=schedule, step=step)
        ws = V.Workspace(pom, prm, K, depth)
        try:
            bel = V.belief_tensor(inst, belief)
            nb = bel.numel() if inst["kind"] == "tabular" else bel.numel() // 2
            res, tree, act, obs = gpu_forced_plan(V, pom, ws, inst, bel, nb, n_p, K, depth, o,
                                                  seed=seed, schedule=schedule, eta=eta,
                                                  step=step)
        finally:
            ws.close()
    finally:
        pom.close()
    follow, flagged, draws = check_draws(o, act, obs)
    oc = assert_tree_parity(res, tree, o, int(inst["nA"]))
    ulps = psi_row_ulps(tree, oc)
    print(f"[drawcheck] draws {draws} flagged {flagged} followed {follow} "
          f"max row error {ulps:.1f} units of 2^-24 of the row's largest entry", flush=True)
    # The screen's premise (TAU_PSI) and its purpose: it excuses rounding, it
    # does not skip the comparison.
    assert ulps <= PSI_ULPS_MAX, ulps
    assert flagged <= max_flag_frac * draws + 5, (flagged, draws)
    return dict(follow=follow, flagged=flagged, draws=draws, res=res, tree=tree, o=o,
                psi_ulps=ulps)


def psi_row_ulps(tree, oc):
    """Largest |Psi_gpu - Psi_oracle| of a non-root row, in units of 2^-24 of
    that row's largest |Psi| (the quantity TAU_PSI bounds); oc: the oracle's
    tree in canonical order."""
    g = np.asarray(tree["psi"][1:], np.float64)
    r = np.asarray(oc["psi"][1:], np.float64)
    if g.size == 0:
        return 0.0
    scale = np.maximum(np.abs(r).max(axis=1), 1e-30) * 2.0 ** -24
    return float((np.abs(g - r).max(axis=1) / scale).max())
