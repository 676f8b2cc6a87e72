"""The canonical row order used to compare trees depends only on the tree."""

import numpy as np

from paper_2510_27191_amd import instances as I
from tests.treecanon import ACTION_KEYS, BELIEF_KEYS, canonical_tree


def _tree(orc, seed=3):
    inst = I.tabular_dense(5, 9, 3, 4, with_heuristic=True)
    o = orc.plan(inst, I.tabular_belief(inst), 400, 4, 3, seed=seed)
    return {k: np.asarray(getattr(o, k)) for k in BELIEF_KEYS + ACTION_KEYS}


def _relabel(t, rng):
    """The same tree with its non-root belief rows and its action rows shuffled."""
    nb, na = t["b_parent"].size, t["a_parent"].size
    bperm = np.concatenate([[0], 1 + rng.permutation(nb - 1)])   # new row i <- old bperm[i]
    aperm = rng.permutation(na)
    bnew = np.empty(nb, np.int64)
    bnew[bperm] = np.arange(nb)
    anew = np.empty(na, np.int64)
    anew[aperm] = np.arange(na)
    out = {k: t[k][bperm].copy() for k in BELIEF_KEYS}
    out.update({k: t[k][aperm].copy() for k in ACTION_KEYS})
    bp = out["b_parent"]
    out["b_parent"] = np.where(bp < 0, -1, anew[np.maximum(bp, 0)])
    out["a_parent"] = bnew[out["a_parent"]]
    return out


def test_canonical_order_is_label_free(orc):
    t = _tree(orc)
    c = canonical_tree(t)
    rng = np.random.default_rng(0)
    for _ in range(3):
        c2 = canonical_tree(_relabel(t, rng))
        for k in c:
            assert np.array_equal(c[k], c2[k]), k
    # Idempotent.
    c3 = canonical_tree(c)
    for k in c:
        assert np.array_equal(c[k], c3[k]), k


def test_canonical_order_properties(orc):
    c = canonical_tree(_tree(orc, seed=5))
    d = c["b_depth"]
    assert d[0] == 0 and c["b_parent"][0] == -1
    assert np.all(np.diff(d) >= 0)
    pa = c["b_parent"][1:]
    key = np.stack([c["a_parent"][pa], c["a_act"][pa], c["b_obs"][1:]], 1)
    for dd in np.unique(d[1:]):
        k = key[d[1:] == dd]
        # strictly increasing (parent row, action, observation) within a depth
        assert all(tuple(k[i]) < tuple(k[i + 1]) for i in range(len(k) - 1))
    ka = np.stack([c["a_parent"], c["a_act"]], 1)
    assert all(tuple(ka[i]) < tuple(ka[i + 1]) for i in range(len(ka) - 1))
    # Parents come before children.
    assert np.all(c["a_parent"][pa] < np.arange(1, d.size))
