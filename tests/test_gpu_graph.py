"""Plans on a non-default stream replay the launch sequence captured for
their shape (one graph per workspace and shape).  Every replay must equal the
same plan launched kernel by kernel on the default stream, bit for bit, with
eager work and synchronisations between the replays; a new shape or a change
of the profiling brackets captures again.
"""

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27191_amd import vopp
    vopp.lib()
    return vopp


def same(V, ra, wa, rb, wb, A):
    assert ra.action == rb.action and ra.v_root == rb.v_root
    assert np.array_equal(ra.values, rb.values)
    assert (ra.particle_steps, ra.n_beliefs, ra.n_actions) == \
        (rb.particle_steps, rb.n_beliefs, rb.n_actions)
    ta = V.tree_dump(wa, A, ra.n_beliefs, ra.n_actions)
    tb = V.tree_dump(wb, A, rb.n_beliefs, rb.n_actions)
    for k in ta:
        assert np.array_equal(ta[k], tb[k]), k


@pytest.mark.parametrize("name", ["nav", "tabular", "wide"])
def test_replays_equal_eager_plans(V, name):
    import torch
    if name == "nav":
        inst, bel, A = I.nav2d(2, 8, heuristic=1), I.nav_belief(3, 3000), 4
    elif name == "tabular":
        inst = I.tabular_sparse(3, 300, 6, 9, 5, with_heuristic=True)
        bel, A = I.tabular_belief(inst), 6
    else:
        inst = I.mars_like(1, 128, 625, reward_scale=0.05)
        bel, A = I.tabular_belief(inst), 625
    pom = V.Pomdp.from_instance(inst)
    b = V.belief_tensor(inst, bel)
    nb = b.numel() if inst["kind"] == "tabular" else b.numel() // 2
    side = torch.cuda.Stream()
    prm0 = V.params(2000, seed=1)
    wg, we = V.Workspace(pom, prm0, 6, 5), V.Workspace(pom, prm0, 6, 5)
    try:
        torch.cuda.synchronize()
        shapes = [(2000, 4, 4), (2000, 4, 4), (2000, 4, 4), (1500, 6, 5), (1500, 6, 5),
                  (2000, 4, 4)]
        for i, (n_p, K, depth) in enumerate(shapes):
            prm = V.params(n_p, seed=10 + i)
            rg = V.plan(pom, b, nb, K, depth, prm, ws=wg, stream=side)
            x = torch.randn(1000, device="cuda").sum()     # eager work in between
            torch.cuda.synchronize()
            re = V.plan(pom, b, nb, K, depth, prm, ws=we)
            same(V, rg, wg, re, we, A)
            assert torch.isfinite(x)
    finally:
        wg.close()
        we.close()
        pom.close()


def test_profiled_replays(V):
    import torch
    inst = I.tabular_sparse(4, 200, 5, 7, 4)
    bel = I.tabular_belief(inst)
    pom = V.Pomdp.from_instance(inst)
    b = V.belief_tensor(inst, bel)
    side = torch.cuda.Stream()
    prm = V.params(3000, seed=2)
    wg, we = V.Workspace(pom, prm, 5, 5), V.Workspace(pom, prm, 5, 5)
    try:
        V.profile_enable(wg, ["backup_level", "forward"])
        V.profile_reset(wg)
        for i in range(3):
            p = V.params(3000, seed=20 + i)
            rg = V.plan(pom, b, b.numel(), 5, 5, p, ws=wg, stream=side)
            re = V.plan(pom, b, b.numel(), 5, 5, p, ws=we)
            same(V, rg, wg, re, we, 5)
        prof = V.profile_read(wg)
        # 5 iterations (D = 1..5): 5 forward launches and 0+1+2+3+4 level sweeps per plan.
        assert prof["forward"][1] == 15 and prof["backup_level"][1] == 30
        assert prof["forward"][0] > 0 and prof["backup_level"][0] > 0
        assert prof["accumulate"][1] == 0
        V.profile_enable(wg, [])
        p = V.params(3000, seed=40)
        rg = V.plan(pom, b, b.numel(), 5, 5, p, ws=wg, stream=side)
        re = V.plan(pom, b, b.numel(), 5, 5, p, ws=we)
        same(V, rg, wg, re, we, 5)
    finally:
        wg.close()
        we.close()
        pom.close()
