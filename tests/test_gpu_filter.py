"""GPU true-environment step and SIR belief update against the oracle: the
particles, observations and weight totals must match bit for bit."""

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests.test_oracle_filter import deterministic_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27191_amd import vopp
    vopp.lib()
    return vopp


@pytest.mark.parametrize("n", [1, 7, 256, 1000, 65536])
def test_tabular_belief_update(V, orc, n):
    import torch
    inst = I.tabular_sparse(2, 300, 6, 9, 5)
    rng = np.random.default_rng(n)
    parts = rng.integers(0, 300, size=n).astype(np.int32)
    pom = V.Pomdp.from_instance(inst)
    for step, (a, o) in enumerate([(1, 3), (4, 0), (5, 8)]):
        dev = torch.as_tensor(parts, device="cuda")
        tot = V.belief_update(pom, dev, n, a, o, seed=99, step=step)
        ref, rtot = orc.belief_update(inst, parts, a, o, seed=99, step=step)
        assert tot == rtot
        assert np.array_equal(dev.cpu().numpy(), ref)
        parts = ref
    pom.close()


@pytest.mark.parametrize("n", [3, 500, 4097])
def test_nav_belief_update(V, orc, n):
    import torch
    inst = I.nav2d(5, 8)
    bx, by = I.nav_belief(6, n, 2.0, 4.0)
    pom = V.Pomdp.from_instance(inst)
    st = (3.0, 3.0)
    for step in range(3):
        a = step % 4
        st, obs, _, _ = orc.env_step(inst, st, a, seed=4, step=step)
        dev = torch.as_tensor(np.concatenate([bx, by]), device="cuda")
        tot = V.belief_update(pom, dev, n, a, obs, seed=12, step=step)
        (rx, ry), rtot = orc.belief_update(inst, (bx, by), a, obs, seed=12, step=step)
        assert tot == rtot
        out = dev.cpu().numpy()
        assert np.array_equal(out[:n], rx) and np.array_equal(out[n:], ry)
        bx, by = rx, ry
    pom.close()


def test_zero_weight_keeps_moved_particles(V, orc):
    import torch
    inst = deterministic_instance()
    pom = V.Pomdp.from_instance(inst)
    parts = np.zeros(10, np.int32)
    dev = torch.as_tensor(parts, device="cuda")
    tot = V.belief_update(pom, dev, 10, 0, 3, seed=5, step=2)
    ref, rtot = orc.belief_update(inst, parts, 0, 3, seed=5, step=2)
    assert tot == rtot == 0 and np.array_equal(dev.cpu().numpy(), ref)
    pom.close()


def test_env_steps(V, orc):
    import torch
    inst = I.tabular_dense(2, 10, 3, 4)
    pom = V.Pomdp.from_instance(inst)
    s = 4
    dev = torch.tensor([s], dtype=torch.int32, device="cuda")
    for t in range(6):
        obs, r, term = V.env_step(pom, dev, t % 3, seed=77, step=t)
        s, o2, r2, term2 = orc.env_step(inst, s, t % 3, seed=77, step=t)
        assert (int(dev.item()), obs, r, term) == (s, o2, r2, term2)
    pom.close()
    nav = I.nav2d(3, 8)
    pom = V.Pomdp.from_instance(nav)
    st = (8.2, 8.4)
    dev = torch.tensor(st, dtype=torch.float32, device="cuda")
    for t in range(6):
        obs, r, term = V.env_step(pom, dev, t % 4, seed=5, step=t)
        st, o2, r2, term2 = orc.env_step(nav, st, t % 4, seed=5, step=t)
        got = dev.cpu().numpy()
        assert (float(got[0]), float(got[1])) == st and (obs, r, term) == (o2, r2, term2)
    pom.close()


def test_filter_arguments_validated(V):
    import torch
    inst = I.tabular_dense(0, 5, 2, 3)
    pom = V.Pomdp.from_instance(inst)
    dev = torch.zeros(4, dtype=torch.int32, device="cuda")
    for a, o in ((2, 0), (0, 3), (-1, 0)):
        with pytest.raises(V.VoppError):
            V.belief_update(pom, dev, 4, a, o, seed=1, step=0)
    with pytest.raises(V.VoppError):
        V.env_step(pom, torch.tensor([9], dtype=torch.int32, device="cuda"), 0, 1, 0)
    pom.close()
