"""Pins of the oracle's reference policy pi0 (Eq. 4, first term): the initial
preference row is (1/eta) ln pi0, the same at every belief."""

import math

import numpy as np
import pytest

from paper_2510_27191_amd import instances as I
from tests import refimpl as R


def _root_counts(res, A):
    m = res.a_parent == 0
    n = np.zeros(A, np.int64)
    n[res.a_act[m]] = res.a_N[m]
    return n


def test_first_iteration_root_draws_follow_pi0(orc):
    # softmax(eta * ln(pi0) / eta) = pi0: root action counts are multinomial.
    inst = I.tabular_dense(4, 8, 5, 3)
    pi0 = np.array([0.05, 0.1, 0.15, 0.3, 0.4])
    n = 40000
    res = orc.plan(inst, I.tabular_belief(inst), n, 1, 1, eta=0.7, seed=3, pi0=pi0 * 3.0)
    cnt = _root_counts(res, 5)
    chi2 = (((cnt - n * pi0) ** 2) / (n * pi0)).sum()
    assert cnt.sum() == n and chi2 < 23.0     # p ~ 1e-4 for 4 degrees of freedom


def test_uniform_pi0_is_the_default(orc):
    inst = I.tabular_dense(2, 9, 3, 4, with_heuristic=True)
    bel = I.tabular_belief(inst)
    a = orc.plan(inst, bel, 700, 3, 3, seed=5)
    b = orc.plan(inst, bel, 700, 3, 3, seed=5, pi0=np.full(3, 2.5))
    for k in ("b_parent", "b_obs", "a_parent", "a_act", "a_N", "b_N"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    np.testing.assert_allclose(b.psi, a.psi, rtol=0, atol=1e-12)
    assert abs(a.v_root - b.v_root) < 1e-12


def test_depth1_value_is_the_prior_weighted_log_sum_exp(orc):
    # K = 1, depth 1: Psi(root, a) = Psi0(a) + Q_a for sampled actions, and
    # V = L_eta Psi = (1/eta) ln sum_a pi0(a) exp(eta Q_a) (Q = 0 if unsampled).
    inst = I.tabular_dense(6, 16, 4, 4, with_heuristic=True)
    pi0 = np.array([0.4, 0.3, 0.2, 0.1])
    eta = 0.8
    res = orc.plan(inst, I.tabular_belief(inst), 3000, 1, 1, eta=eta, seed=12, pi0=pi0)
    psi0 = np.log(pi0 / pi0.sum()) / eta
    Q = res.psi_root - psi0
    want = math.log(np.sum(pi0 / pi0.sum() * np.exp(eta * Q))) / eta
    assert abs(res.v_root - want) < 1e-12
    # The visit-weighted mean of Q is the mean one-step return of the episodes.
    cnt = _root_counts(res, 4)
    assert cnt.sum() == 3000 and np.all(cnt > 0)


@pytest.mark.slow
def test_k1_with_pi0_converges_to_reference_bellman(orc):
    inst = I.tabular_dense(1, 3, 2, 2, gamma=0.9, with_heuristic=True)
    bel = I.tabular_belief(inst)
    b0 = R.root_probs(bel.size)
    eta, depth = 1.5, 2
    pi0 = np.array([0.8, 0.2])
    exact = R.ref_bellman(inst, b0, depth, eta, pi0=pi0)
    assert abs(exact - R.ref_bellman(inst, b0, depth, eta)) > 1e-3   # the prior matters
    vs = np.array([orc.plan(inst, bel, 2 ** 15, 1, depth, eta=eta, seed=sd, schedule=1,
                            pi0=pi0).v_root for sd in range(1, 13)])
    se = vs.std(ddof=1) / math.sqrt(vs.size)
    assert abs(vs.mean() - exact) <= 4.5 * se + 2e-3, (vs.mean(), exact, se)
