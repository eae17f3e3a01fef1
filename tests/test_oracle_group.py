"""Pins of the oracle's second-order activity prior (MAP-K2) and of the
group-activity generator that draws data from that model (CPU, FP64).

MAP-K2 is PSCA-MAP-K with the activity model of eq. second: first-order
coefficients c_n and pairwise c_{n,n'}; its gradient is eq. ft_gradient
(case G) restricted to sets of at most two devices."""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix

import oracle as O
from oracle import psca_oracle as PO
from paper_2503_15259_amd import instances as I


def tiny_group(seed=0, N=30, L=8, M=64, K=3, b=1.5, p=0.2):
    inst = I.make_group_instance(9, seed, N, L, M, p, K, b)
    return inst, O.problem_from_instance(inst, O.MAP_K2)


def fd_grad(prob, x, n, h):
    xp = x.copy(); xp[n] += h
    xm = x.copy(); xm[n] -= h
    return (O.objective(prob, xp) - O.objective(prob, xm)) / (2 * h)


def test_pairwise_prior_matrix_is_symmetric_group_block():
    inst, prob = tiny_group(N=31, K=4)   # a short last group
    C = prob.C2.toarray()
    assert np.array_equal(C, C.T)
    assert np.all(np.diag(C) == 0)
    same = inst.group[:, None] == inst.group[None, :]
    np.testing.assert_array_equal(C != 0, same & ~np.eye(inst.N, dtype=bool))
    assert np.all(C[C != 0] == inst.c_pair)
    np.testing.assert_array_equal(prob.c1, np.full(inst.N, inst.c_single))


def test_objective_prior_term_is_the_exponent_of_the_second_order_model():
    """f_MAP-K2 - f_ML-K = -(1/M) (sum_n c_n a_n + sum_{n<n'} c_{n,n'} a_n a_n'),
    summed pair by pair over the group structure, at binary and relaxed points."""
    inst, prob = tiny_group(seed=3)
    ml = O.Problem(prob.Sigma_hat, prob.S, prob.sigma2, prob.M, O.ML_K, g=prob.g)
    rng = np.random.default_rng(5)
    for x in (rng.uniform(0, 1, inst.N), (rng.random(inst.N) < 0.4).astype(float)):
        expo = inst.c_single * x.sum()
        for n1 in range(inst.N):
            for n2 in range(n1 + 1, inst.N):
                if inst.group[n1] == inst.group[n2]:
                    expo += inst.c_pair * x[n1] * x[n2]
        d = O.objective(prob, x) - O.objective(ml, x)
        assert d == pytest.approx(-expo / prob.M, rel=1e-12, abs=1e-12)


def test_gradient_matches_finite_differences():
    inst, prob = tiny_group(seed=1)
    x = np.random.default_rng(2).uniform(0.1, 0.9, prob.N)
    rec = O.psca_iteration(prob, x, 0.5)
    grad, curv = PO.gradient_and_curvature(prob, x, rec.q, rec.r)
    np.testing.assert_allclose(curv, (prob.g * rec.q) ** 2)
    for n in range(prob.N):
        h = 1e-6
        fd = fd_grad(prob, x, n, h)
        assert abs(fd - grad[n]) <= 1e-5 * max(1.0, abs(grad[n])), (n, fd, grad[n])


def test_without_pairs_equals_independent_map_k():
    """With every c_{n,n'} = 0 and c_n = log(p/(1-p)), eq. second is the
    independent model and MAP-K2 is MAP-K, iterate for iterate."""
    inst = I.make_instance(0, 3, 100, 20, 32, 0.1)
    mapk = O.problem_from_instance(inst, O.MAP_K)
    k2 = O.Problem(mapk.Sigma_hat, mapk.S, mapk.sigma2, mapk.M, O.MAP_K2, g=mapk.g,
                   c1=np.log(mapk.p / (1 - mapk.p)), C2=csr_matrix((inst.N, inst.N)))
    np.testing.assert_allclose(O.psca(k2, 40), O.psca(mapk, 40), rtol=0, atol=1e-13)


def test_pair_term_of_the_gradient():
    """At x = 1/2 everywhere the prior part of each gradient is
    -(c_n + c_pair (K - 1) / 2) / M: eq. ft_gradient's pair term counts
    each group mate once."""
    inst, prob = tiny_group(seed=4, K=3)
    x = np.full(prob.N, 0.5)
    members = np.flatnonzero(inst.group == inst.group[0])
    rec0 = O.psca_iteration(prob, x, 0.5)
    g0, _ = PO.gradient_and_curvature(prob, x, rec0.q, rec0.r)
    ml = O.Problem(prob.Sigma_hat, prob.S, prob.sigma2, prob.M, O.ML_K, g=prob.g)
    g0ml, _ = PO.gradient_and_curvature(ml, x, rec0.q, rec0.r)
    for n in members:
        mates = len(members) - 1
        assert g0[n] - g0ml[n] == pytest.approx(-(inst.c_single + inst.c_pair * 0.5 * mates) / prob.M, rel=1e-12)


def test_descent_inequality_every_iteration():
    inst = I.make_group_instance(9, 7, 100, 20, 32, 0.1, 4, 2.0)
    prob = O.problem_from_instance(inst, O.MAP_K2)
    _, hist = O.psca(prob, 30, record=True)
    for rec in hist:
        grad, curv = PO.gradient_and_curvature(prob, rec.x, rec.q, rec.r)
        d = rec.x_tilde - rec.x
        assert float(grad @ d) <= -float(np.sum(curv * d * d)) + 1e-12


def test_permutation_equivariance():
    inst, prob = tiny_group(seed=6)
    perm = np.random.default_rng(1).permutation(prob.N)
    C = prob.C2.toarray()[np.ix_(perm, perm)]
    pp = O.Problem(prob.Sigma_hat, prob.S[:, perm], prob.sigma2, prob.M, O.MAP_K2, g=prob.g[perm],
                   c1=prob.c1[perm], C2=csr_matrix(C))
    np.testing.assert_allclose(O.psca(pp, 25), O.psca(prob, 25)[perm], rtol=1e-10, atol=1e-13)


def test_brute_force_support_on_tiny_instances():
    """Thresholded MAP-K2 support against the minimiser of f_MAP-K2 over
    {0,1}^N (2^10 evaluations) on most seeds: the relaxed iteration
    reaches the binary optimum when M is large."""
    hits = 0
    seeds = range(20)
    for s in seeds:
        inst = I.make_group_instance(9, 100 + s, 10, 6, 256, 0.2, 5, 2.0)
        prob = O.problem_from_instance(inst, O.MAP_K2)
        x = O.psca(prob, 300)
        best, arg = math.inf, None
        for bits in itertools.product((0.0, 1.0), repeat=10):
            f = O.objective(prob, np.array(bits))
            if f < best:
                best, arg = f, np.array(bits)
        hits += int(np.array_equal((x >= 0.5).astype(float), arg))
    assert hits >= 0.9 * len(seeds), hits


def test_group_generator_draws_the_second_order_law():
    """Per-group activity counts over many groups against the exact law
    p(k active of K) = C(K, k) exp(a k + b k(k-1)/2) / Z (eq. second with
    block coefficients), and the marginal p."""
    K, b, p = 4, 1.5, 0.15
    inst = I.make_group_instance(9, 999, 40000, 1, 1, p, K, b)
    a = inst.c_single
    logw = np.array([math.log(math.comb(K, k)) + a * k + b * k * (k - 1) / 2 for k in range(K + 1)])
    law = np.exp(logw - logw.max()); law /= law.sum()
    counts = np.bincount(np.bincount(inst.group, weights=inst.alpha).astype(int), minlength=K + 1)
    n_groups = counts.sum()
    expect = law * n_groups
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 25.0, (counts, expect)          # 4 dof: P(chi2 > 25) < 1e-4
    marg = float(law @ np.arange(K + 1)) / K
    assert marg == pytest.approx(p, abs=1e-9)
    assert abs(inst.alpha.mean() - p) < 5 * math.sqrt(p * (1 - p) / inst.N) * 2
