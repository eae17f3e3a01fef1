"""Pins of the oracle's unrolled-network gradients (FP64, CPU).

The layer Jacobian-vector products and the network gradient are checked
against central finite differences of the forward map itself (one iteration
of Algorithm 1, and the BCE loss of eqs. Loss_alpha / Loss_gamma after K
iterations), on N = 20, L = 8 instances."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2503_15259_amd import instances as I

VARIANTS = [O.ML_K, O.MAP_K, O.ML_UD, O.MAP_UR, O.MAP_K2]


def tiny(variant, seed=0):
    if variant == O.MAP_K2:
        inst = I.make_group_instance(3, 100 + seed, 20, 8, 64, 0.3, 4, 1.5)
    else:
        inst = I.make_instance(3, 100 + seed, 20, 8, 64, 0.3)
    return inst, O.problem_from_instance(inst, variant, eps=0.01)


def interior_point(prob, inst, rng):
    """An iterate away from the clip bounds and the prior's branch points."""
    if prob.variant in O.KNOWN_PATHLOSS:
        return rng.uniform(0.1, 0.9, prob.N)
    x = inst.g * rng.uniform(0.2, 1.5, prob.N)
    if prob.variant == O.MAP_UR:
        pr = prob.prior
        pts = np.array([pr.eps, pr.g_l - pr.eps, pr.g_l])
        for n in range(prob.N):
            while np.min(np.abs(x[n] - pts)) < 1e-2 * pr.g_l:
                x[n] *= 1.1
        x = np.minimum(x, 0.9 * pr.g_u)
    return x


def test_prior_second_derivative_matches_finite_differences():
    prob = O.problem_from_instance(I.make_instance(3, 1, 20, 8, 64, 0.3), O.MAP_UR, eps=0.5)
    pr = prob.prior
    for x in (0.1, 0.3, pr.g_l - 0.3, pr.g_l - 0.1, 1.5 * pr.g_l, 40.0 * pr.g_l):
        h = 1e-6 * max(1.0, x)
        fd = (pr.log_ratio(x + h) - pr.log_ratio(x - h)) / (2 * h)
        assert pr.dlog_ratio(x) == pytest.approx(fd, rel=1e-5, abs=1e-9), x
    # power-law density branch: p'/p = -(2/beta + 1)/x, so its derivative is (2/beta + 1)/x^2
    x = 3.0 * pr.g_l
    assert pr.dlog_ratio(x) == pytest.approx((2.0 / pr.beta + 1.0) / x ** 2, rel=1e-10)
    assert pr.dlog_ratio(0.5 * pr.g_l) == 0.0   # the gap


@pytest.mark.parametrize("variant", VARIANTS)
def test_layer_vjp_matches_finite_differences(variant):
    rng = np.random.default_rng(7 + variant)
    inst, prob = tiny(variant, variant)
    x = interior_point(prob, inst, rng)
    rho = 0.37
    v = rng.standard_normal(prob.N)
    dx, drho = O.layer_vjp(prob, x, rho, v)

    def layer(xx, rr):
        return O.psca_iteration(prob, xx, rr).x_next

    fd = np.empty(prob.N)
    for m in range(prob.N):
        h = 1e-6 * max(1.0, abs(x[m]))
        e = np.zeros(prob.N)
        e[m] = h
        fd[m] = v @ (layer(x + e, rho) - layer(x - e, rho)) / (2 * h)
    np.testing.assert_allclose(dx, fd, rtol=2e-5, atol=1e-7 * np.max(np.abs(fd)))
    h = 1e-6
    fdr = v @ (layer(x, rho + h) - layer(x, rho - h)) / (2 * h)
    assert drho == pytest.approx(fdr, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("variant", [O.ML_K, O.ML_UD, O.MAP_UR])
def test_network_gradient_matches_finite_differences(variant):
    inst, prob = tiny(variant, 10 + variant)
    rhos = O.step_sizes(5)
    loss, g = O.net_loss_and_grad(prob, rhos, inst.alpha, inst.g)
    for k in range(5):
        h = 1e-6
        rp, rm = rhos.copy(), rhos.copy()
        rp[k] += h
        rm[k] -= h
        lp, _ = O.bce_loss(prob, O.net_forward(prob, rp)[-1], inst.alpha, inst.g)
        lm, _ = O.bce_loss(prob, O.net_forward(prob, rm)[-1], inst.alpha, inst.g)
        assert g[k] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9), k


def test_bce_loss_closed_form():
    """Two devices, alpha = (1, 0), outputs (0.8, 0.3): loss = -(ln 0.8 + ln 0.7)/2."""
    prob = O.Problem(Sigma_hat=np.eye(1), S=np.ones((1, 2)), sigma2=1.0, M=1, variant=O.ML_K,
                     g=np.ones(2))
    loss, d = O.bce_loss(prob, np.array([0.8, 0.3]), np.array([1.0, 0.0]), np.ones(2))
    assert loss == pytest.approx(-(np.log(0.8) + np.log(0.7)) / 2)
    np.testing.assert_allclose(d, [-1.0 / 0.8 / 2, 1.0 / 0.7 / 2])
