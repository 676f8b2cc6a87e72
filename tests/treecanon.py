"""Canonical row order of a VOPP search tree (test infrastructure).

The tensors of Sec. III-C are sets of rows: which row number a belief or an
action node gets depends on the order in which episodes reached it, not on
the tree.  The oracle numbers rows in first-visitor order; the HIP path
numbers them by table slot and dumps them in the canonical order defined
here, which depends only on the tree:

  beliefs       by depth, then by (row of the parent belief, action,
                observation key); the root is row 0;
  action nodes  by (row of the parent belief, action).

canonical_tree() reorders any tree given in another row order (for example
the oracle's) into that order, renumbering every row reference.
"""

import numpy as np

BELIEF_KEYS = ("b_parent", "b_obs", "b_depth", "psi", "b_V", "b_N")
ACTION_KEYS = ("a_parent", "a_act", "a_C", "a_N")


def _get(t, k):
    return np.asarray(t[k] if isinstance(t, dict) else getattr(t, k))


def canonical_tree(t):
    b_parent = _get(t, "b_parent").astype(np.int64)
    b_obs = _get(t, "b_obs").astype(np.int64)
    b_depth = _get(t, "b_depth").astype(np.int64)
    a_parent = _get(t, "a_parent").astype(np.int64)
    a_act = _get(t, "a_act").astype(np.int64)
    nb, na = b_parent.size, a_parent.size
    pos = np.full(nb, -1, np.int64)
    pos[0] = 0
    order = [np.array([0], np.int64)]
    filled = 1
    for d in range(1, int(b_depth.max(initial=0)) + 1):
        idx = np.nonzero(b_depth == d)[0]
        pa = b_parent[idx]                         # parent action rows
        srt = np.lexsort((b_obs[idx], a_act[pa], pos[a_parent[pa]]))
        idx = idx[srt]
        pos[idx] = filled + np.arange(idx.size)
        filled += idx.size
        order.append(idx)
    order = np.concatenate(order)
    assert filled == nb and np.all(pos >= 0), "tree rows are not all reachable"
    aord = np.lexsort((a_act, pos[a_parent]))
    apos = np.empty(na, np.int64)
    apos[aord] = np.arange(na)
    out = {}
    for k in BELIEF_KEYS:
        out[k] = _get(t, k)[order].copy()
    for k in ACTION_KEYS:
        out[k] = _get(t, k)[aord].copy()
    bp = b_parent[order]
    out["b_parent"] = np.where(bp < 0, -1, apos[np.maximum(bp, 0)]).astype(_get(t, "b_parent").dtype)
    out["a_parent"] = pos[a_parent[aord]].astype(_get(t, "a_parent").dtype)
    return out
