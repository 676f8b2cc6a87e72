"""The allocation-free entry point (vopp_plan_noalloc) against vopp_plan: two
calls in a row on the library's static scratch array, the second with a
smaller input, each equal to the workspace plan bit for bit."""

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


def plain(V, pom, bel, nb, K, depth, prm):
    ws = V.Workspace(pom, prm, K, depth)
    try:
        return V.plan(pom, bel, nb, K, depth, prm, ws=ws)
    finally:
        ws.close()


def noalloc(V, pom, bel, nb, K, depth, prm):
    import torch
    out = torch.full((pom.nA + 10,), -7.0, dtype=torch.float64, device="cuda")
    V.plan_noalloc(pom, bel, nb, K, depth, prm, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def same(r, o, A):
    assert int(o[0]) == r.action
    assert np.array_equal(o[1:1 + A], r.values)
    assert o[A + 1] == r.v_root
    assert (int(o[A + 2]), int(o[A + 3]), int(o[A + 4])) == \
        (r.particle_steps, r.n_beliefs, r.n_actions)
    assert int(o[A + 5]) == 0
    assert int(o[A + 6]) == r.near_ties
    assert tuple(int(x) for x in o[A + 7:A + 10]) == r.sweep


@pytest.mark.parametrize("kind", ["nav", "tabular"])
def test_noalloc_equals_plan_twice(V, kind):
    if kind == "nav":
        inst = I.nav2d(2, 8, heuristic=1)
        big, small = I.nav_belief(3, 3000), I.nav_belief(4, 700)
        sizes = [(6000, 5, 6, 3000, big), (2500, 3, 4, 700, small)]
    else:
        inst = I.tabular_sparse(1, 512, 8, 32, 8, with_heuristic=True)
        bel = I.tabular_belief(inst)
        sizes = [(8000, 5, 5, bel.size, bel), (1500, 2, 3, bel.size, bel)]
    pom = V.Pomdp.from_instance(inst)
    try:
        for i, (n_p, K, depth, nb, b) in enumerate(sizes):
            prm = V.params(n_p, seed=11 + i, schedule=i % 2)
            belt = V.belief_tensor(inst, b)
            assert V.footprint(pom, prm, K, depth) <= V.NOALLOC_SCRATCH_BYTES
            o = noalloc(V, pom, belt, nb, K, depth, prm)
            r = plain(V, pom, belt, nb, K, depth, prm)
            same(r, o, pom.nA)
    finally:
        pom.close()


def test_noalloc_rejects_plans_beyond_the_scratch(V):
    import torch
    inst, bel, p = I.workload("nav2d", seed=0)
    pom = V.Pomdp.from_instance(inst)
    try:
        prm = V.params(p["n_particles"], seed=1)
        assert V.footprint(pom, prm, 10, 10) > V.NOALLOC_SCRATCH_BYTES
        out = torch.zeros(pom.nA + 10, dtype=torch.float64, device="cuda")
        belt = V.belief_tensor(inst, bel)
        with pytest.raises(V.VoppError) as e:
            V.plan_noalloc(pom, belt, belt.numel() // 2, 10, 10, prm, out)
        assert e.value.status == V.VOPP_E_INVALID
        assert "allocation-free" in str(e.value)
    finally:
        pom.close()
