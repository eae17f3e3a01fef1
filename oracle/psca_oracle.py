"""FP64 CPU oracle for PSCA device activity detection (Tan & Cui, arXiv 2503.15259).

TEST INFRASTRUCTURE ONLY.  This module is a plain, slow, obviously-correct
restatement of the paper's per-iteration method in float64 / complex128
NumPy.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it.  The HIP library never calls it, and it shares no code,
constant table or helper with the HIP path.

What it computes (paper Sec. III and IV, Algorithm 1 "PSCA Algorithms"):
  x^(0) = 0; for k = 0, 1, ...:
    Sigma_k  = S diag(w) S^H + sigma^2 I,  w = g*alpha (known g) or gamma
    Sigma_k^-1 by Frobenius inversion (Sec. III-A, eqs. Frobenius_inversion_1/2)
    q_n = s_n^H Sigma^-1 s_n,  r_n = s_n^H Sigma^-1 SigmaHat Sigma^-1 s_n
    gradient of the variant's objective, curvature (g_n q_n)^2 or q_n^2
    x~_n = clip(x_n - grad_n / curv_n, lo, hi)      (Lemmas 1-4)
    x_n <- (1 - rho_k) x_n + rho_k x~_n              (eqs. Update_*)
    rho_{k+1} = rho_k (1 - 0.5 rho_k), rho_0 = 0.5   (Sec. V)

Readings where the paper is silent, ambiguous or garbled:
  R1  MAP-K independent-prior gradient carries the 1/M factor of its
      objective f_I (eq. ft); the printed gradient (eq. ft_gradient) drops it.
  R2  The derivative of H2 (eq. pepsd, third case) uses coefficient 2, the
      exact derivative of eq. H2; the printed 12 breaks Theorem 1(ii)'s
      junction slope at g_l.
  R3  Where p^eps = 0 (the gap [eps, g_l - eps], including its closed left
      end of the H2 piece), the prior term p^eps'/p^eps is taken as 0.
  R4  Pathloss map phi(d) = c0 d^-beta (power law); one common annulus
      [d_l, d_u] for all n.  The distance law is area-uniform (eq. dispdf,
      law 0) by default; law 1 is uniform in d, the law the synthetic
      instances are drawn from.  The pathloss density is eq. pg's change of
      variables p_G(x) = p_D(psi(x)) |psi'(x)| for either law.
  R5  Step sizes: rho_0 = 0.5, rho_{k+1} = rho_k (1 - 0.5 rho_k); the update
      at iteration k uses rho_k.  Fixed iteration count (no stopping rule).
  R6  Clip bounds are inclusive; K variants [0, 1], ML-UD [0, inf),
      MAP-UR [0, g_u].
  R8  MAP-K2 is PSCA-MAP-K under the second-order approximation of the
      general activity model (eq. second): f_t of eq. ft with t = G keeps
      the coefficients c_{n} and c_{n,n'} only, so its gradient (eq.
      ft_gradient, case G) is -(1/M)(c_n + sum_{n'} c_{n,n'} alpha_n').
      The pairwise coefficients form a symmetric matrix C with zero
      diagonal, and f_t = -(1/M)(c^T alpha + alpha^T C alpha / 2).
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

ML_K, MAP_K, ML_UD, MAP_UR, MAP_K2 = 0, 1, 2, 3, 4
VARIANT_NAMES = {ML_K: "ML-K", MAP_K: "MAP-K", ML_UD: "ML-UD", MAP_UR: "MAP-UR", MAP_K2: "MAP-K2"}
KNOWN_PATHLOSS = (ML_K, MAP_K, MAP_K2)


# ---------------------------------------------------------------------------
# Covariances (Sec. III-A eq. cov_a, Sec. IV-A eq. cov_b, and the empirical
# covariance defined with eq. likelihood_Y)
# ---------------------------------------------------------------------------

def sample_covariance(Y: np.ndarray) -> np.ndarray:
    """SigmaHat_Y = Y Y^H / M (the sufficient statistic; computed once)."""
    Y = np.asarray(Y, dtype=np.complex128)
    return Y @ Y.conj().T / Y.shape[1]


def model_covariance(S: np.ndarray, w: np.ndarray, sigma2: float) -> np.ndarray:
    """Sigma = S Diag(w) S^H + sigma^2 I  (w = g*alpha or gamma)."""
    L = S.shape[0]
    # S Diag(w): column n of S scaled by w_n (the same products as the dense
    # diagonal matrix, without forming an N x N array)
    return (S * np.asarray(w, dtype=np.float64)[None, :]) @ S.conj().T + sigma2 * np.eye(L)


def frobenius_inverse(Sigma: np.ndarray) -> np.ndarray:
    """Inverse of a complex positive-definite matrix from real inverses
    (Sec. III-A, eqs. Frobenius_inversion_1 and _2):
        Re(Sigma^-1) = (A + B A^-1 B)^-1
        Im(Sigma^-1) = -A^-1 B (A + B A^-1 B)^-1,   A = Re Sigma, B = Im Sigma.
    """
    A = Sigma.real
    B = Sigma.imag
    A_inv = np.linalg.inv(A)
    re = np.linalg.inv(A + B @ A_inv @ B)
    im = -A_inv @ B @ re
    return re + 1j * im


def quadratic_forms(S: np.ndarray, Sigma_inv: np.ndarray, Sigma_hat: np.ndarray):
    """q_n = s_n^H Sigma^-1 s_n and r_n = s_n^H Sigma^-1 SigmaHat Sigma^-1 s_n,
    the two terms of the ML gradients (eqs. gradient_ML, gradient_ML_U).
    Both are real for Hermitian Sigma, SigmaHat; the imaginary round-off is
    dropped."""
    N = S.shape[1]
    q = np.empty(N)
    r = np.empty(N)
    T = Sigma_inv @ Sigma_hat @ Sigma_inv
    for n in range(N):
        s = S[:, n]
        q[n] = np.real(s.conj() @ Sigma_inv @ s)
        r[n] = np.real(s.conj() @ T @ s)
    return q, r


# ---------------------------------------------------------------------------
# MAP-UR prior (Sec. II: eqs. dispdf, gn, pg, pgamma, H2, peps; Sec. IV-B:
# eq. pepsd; Theorem 1)
# ---------------------------------------------------------------------------

AREA_UNIFORM, UNIFORM_IN_D = 0, 1   # distance laws (reading R4)


@dataclass
class PowerLawPrior:
    """Effective-pathloss prior for one device with phi(d) = c0 d^-beta,
    distance on [d_l, d_u] with law `law` (AREA_UNIFORM: p_D(d) = 2d/D as
    eq. dispdf; UNIFORM_IN_D: p_D(d) = 1/(d_u - d_l)), activity probability p
    and Hermite smoothing width eps."""
    p: float
    d_l: float
    d_u: float
    c0: float
    beta: float
    eps: float
    law: int = AREA_UNIFORM

    # psi = phi^-1 and its derivatives
    def psi(self, x):
        return (self.c0 / x) ** (1.0 / self.beta)

    def dpsi(self, x):
        return -self.psi(x) / (self.beta * x)

    def ddpsi(self, x):
        return self.psi(x) * (1.0 / self.beta) * (1.0 / self.beta + 1.0) / (x * x)

    @property
    def g_l(self):
        return self.c0 * self.d_u ** (-self.beta)

    @property
    def g_u(self):
        return self.c0 * self.d_l ** (-self.beta)

    @property
    def D(self):
        return self.d_u ** 2 - self.d_l ** 2

    def dddpsi(self, x):
        b = 1.0 / self.beta
        return -b * (b + 1.0) * (b + 2.0) * self.psi(x) / x ** 3

    def p_G(self, x):
        """Pathloss density on [g_l, g_u] (eq. pg): p_D(psi(x)) |psi'(x)|,
        psi decreasing."""
        if self.law == UNIFORM_IN_D:
            return -self.dpsi(x) / (self.d_u - self.d_l)
        return -2.0 * self.psi(x) * self.dpsi(x) / self.D

    def p_upsilon_cont(self, x):
        """Continuous part of eq. pgamma on [g_l, g_u]: p * p_G."""
        return self.p * self.p_G(x)

    def dp_upsilon_cont(self, x):
        """Derivative of the continuous part (fourth case of eq. pepsd)."""
        if self.law == UNIFORM_IN_D:
            return -self.p * self.ddpsi(x) / (self.d_u - self.d_l)
        return -2.0 * self.p / self.D * (self.dpsi(x) ** 2 + self.psi(x) * self.ddpsi(x))

    def ddp_upsilon_cont(self, x):
        """Second derivative of the continuous part (needs the third
        derivative of psi for the power law)."""
        if self.law == UNIFORM_IN_D:
            return -self.p * self.dddpsi(x) / (self.d_u - self.d_l)
        return -2.0 * self.p / self.D * (3.0 * self.dpsi(x) * self.ddpsi(x) + self.psi(x) * self.dddpsi(x))

    def H1(self, x):
        e = self.eps
        return (1.0 - self.p) * (1.0 + 2.0 * x / e) * ((x - e) / e) ** 2

    def dH1(self, x):
        e = self.eps
        return 6.0 * (1.0 - self.p) / e ** 3 * x * (x - e)

    def ddH1(self, x):
        e = self.eps
        return 6.0 * (1.0 - self.p) / e ** 3 * (2.0 * x - e)

    def _AB(self):
        """The coefficients of eq. H2, written out at g_l = phi(d_u) (so
        psi(g_l) = d_u).  Area-uniform law: as eq. H2 defines them.  Uniform
        in d: the same construction with p_D = 1/(d_u - d_l).  Theorem 1
        makes them p_Upsilon(g_l) and p_Upsilon'(g_l); the junction pins
        check that against the density functions above."""
        gl = self.g_l
        if self.law == UNIFORM_IN_D:
            w = self.d_u - self.d_l
            return -self.p / w * self.dpsi(gl), -self.p / w * self.ddpsi(gl)
        A = -2.0 * self.p * self.d_u / self.D * self.dpsi(gl)
        B = -2.0 * self.p / self.D * (self.dpsi(gl) ** 2 + self.ddpsi(gl) * self.d_u)
        return A, B

    def H2(self, x):
        """Eq. H2, u = gamma - g_l."""
        A, B = self._AB()
        e = self.eps
        u = x - self.g_l
        return A * (1.0 - 2.0 * u / e) * ((u + e) / e) ** 2 + B * u * ((u + e) / e) ** 2

    def dH2(self, x):
        """Exact derivative of eq. H2 (reading R2: coefficient 2, not 12)."""
        A, B = self._AB()
        e = self.eps
        u = x - self.g_l
        return -6.0 * A / e ** 3 * u * (u + e) + B / e ** 2 * (u + e) * (3.0 * u + e)

    def ddH2(self, x):
        A, B = self._AB()
        e = self.eps
        u = x - self.g_l
        return -6.0 * A / e ** 3 * (2.0 * u + e) + B / e ** 2 * (6.0 * u + 4.0 * e)

    def branch(self, x) -> int:
        """Which piece of eq. peps holds x: 0 H1, 1 gap, 2 H2, 3 density."""
        if x < self.eps:
            return 0
        if x < self.g_l - self.eps:
            return 1
        if x < self.g_l:
            return 2
        return 3

    def p_eps(self, x):
        """Smoothed prior density p^eps (eq. peps)."""
        b = self.branch(x)
        if b == 0:
            return self.H1(x)
        if b == 1:
            return 0.0
        if b == 2:
            return self.H2(x)
        return self.p_upsilon_cont(x)

    def dp_eps(self, x):
        """Its derivative (eq. pepsd with reading R2)."""
        b = self.branch(x)
        if b == 0:
            return self.dH1(x)
        if b == 1:
            return 0.0
        if b == 2:
            return self.dH2(x)
        return self.dp_upsilon_cont(x)

    def ddp_eps(self, x):
        b = self.branch(x)
        if b == 0:
            return self.ddH1(x)
        if b == 1:
            return 0.0
        if b == 2:
            return self.ddH2(x)
        return self.ddp_upsilon_cont(x)

    def dlog_ratio(self, x):
        """Derivative of p^eps'/p^eps: (p'' p - p'^2) / p^2; 0 in the gap."""
        pe = self.p_eps(x)
        if pe == 0.0:
            return 0.0
        d1 = self.dp_eps(x)
        return (self.ddp_eps(x) * pe - d1 * d1) / (pe * pe)

    def log_ratio(self, x):
        """p^eps'(x) / p^eps(x), the prior term of eq. gradient_MAP_U;
        0 where p^eps = 0 (reading R3)."""
        pe = self.p_eps(x)
        if pe == 0.0:
            return 0.0
        return self.dp_eps(x) / pe


def make_prior(p, d_l, d_u, c0, beta, eps, law: int = AREA_UNIFORM) -> PowerLawPrior:
    return PowerLawPrior(p=float(p), d_l=float(d_l), d_u=float(d_u), c0=float(c0),
                         beta=float(beta), eps=float(eps), law=int(law))


# ---------------------------------------------------------------------------
# Objectives (eqs. likelihood_Y, likelihood_Y_MAP with f_I of eq. ft,
# likelihood_Y_U, likelihood_Y_MAP_U with eq. feps)
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """Inputs of one detection: SigmaHat, S, sigma^2, M and the variant data."""
    Sigma_hat: np.ndarray
    S: np.ndarray
    sigma2: float
    M: int
    variant: int
    g: np.ndarray | None = None        # known pathloss (ML-K, MAP-K)
    p: np.ndarray | None = None        # activity probabilities (MAP-K)
    prior: PowerLawPrior | None = None  # MAP-UR prior (common to all devices)
    c1: np.ndarray | None = None       # MAP-K2: first-order coefficients c_{n}
    C2: object | None = None           # MAP-K2: pairwise c_{n,n'} (scipy CSR, symmetric, zero diagonal)

    @property
    def N(self):
        return self.S.shape[1]

    def weights(self, x):
        """w in Sigma = S Diag(w) S^H + sigma^2 I."""
        if self.variant in KNOWN_PATHLOSS:
            return self.g * x
        return np.asarray(x, dtype=np.float64)

    def bounds(self):
        if self.variant in KNOWN_PATHLOSS:
            return 0.0, 1.0
        if self.variant == ML_UD:
            return 0.0, math.inf
        return 0.0, self.prior.g_u


def ml_objective(Sigma: np.ndarray, Sigma_hat: np.ndarray) -> float:
    """log|Sigma| + tr(Sigma^-1 SigmaHat), via slogdet and a linear solve."""
    sign, logdet = np.linalg.slogdet(Sigma)
    assert sign.real > 0
    return float(logdet.real + np.real(np.trace(np.linalg.solve(Sigma, Sigma_hat))))


def objective(prob: Problem, x: np.ndarray) -> float:
    """The variant's objective f(x); +inf for MAP-UR where p^eps(x_n) = 0."""
    Sigma = model_covariance(prob.S, prob.weights(x), prob.sigma2)
    f = ml_objective(Sigma, prob.Sigma_hat)
    if prob.variant == MAP_K:
        f += -np.sum(np.log(prob.p / (1.0 - prob.p)) * x) / prob.M
    elif prob.variant == MAP_K2:   # reading R8
        f += -(np.dot(prob.c1, x) + 0.5 * np.dot(x, prob.C2 @ x)) / prob.M
    elif prob.variant == MAP_UR:
        for xn in x:
            pe = prob.prior.p_eps(float(xn))
            if pe <= 0.0:
                return math.inf
            f += -math.log(pe) / prob.M
    return f


# ---------------------------------------------------------------------------
# One PSCA iteration (Algorithm 1, steps 5-8)
# ---------------------------------------------------------------------------

def gradient_and_curvature(prob: Problem, x: np.ndarray, q: np.ndarray, r: np.ndarray):
    """Partial derivatives of the objective and the surrogate's quadratic
    coefficient 2c (eqs. gradient_ML, gradient_MAP + ft_gradient,
    gradient_ML_U, gradient_MAP_U; Surrogate_*_separate)."""
    v = prob.variant
    if v == ML_K:
        grad = prob.g * (q - r)
        curv = (prob.g * q) ** 2
    elif v == MAP_K:
        grad = prob.g * (q - r) - np.log(prob.p / (1.0 - prob.p)) / prob.M   # reading R1
        curv = (prob.g * q) ** 2
    elif v == MAP_K2:
        grad = prob.g * (q - r) - (prob.c1 + prob.C2 @ x) / prob.M   # eq. ft_gradient, case G; R8
        curv = (prob.g * q) ** 2
    elif v == ML_UD:
        grad = q - r
        curv = q ** 2
    elif v == MAP_UR:
        lr = np.array([prob.prior.log_ratio(float(xn)) for xn in x])
        grad = q - r - lr / prob.M
        curv = q ** 2
    else:
        raise ValueError(f"unknown variant {v}")
    return grad, curv


def coordinate_step(x: np.ndarray, grad: np.ndarray, curv: np.ndarray, lo: float, hi: float):
    """Minimiser of grad (t - x) + curv/2 (t - x)^2 over [lo, hi]
    (Lemmas 1-4 via Lemmas 5-6 of Appendix C)."""
    return np.minimum(np.maximum(x - grad / curv, lo), hi)


@dataclass
class IterationRecord:
    x: np.ndarray        # x^(k)
    q: np.ndarray
    r: np.ndarray
    x_tilde: np.ndarray
    rho: float
    x_next: np.ndarray   # x^(k+1)


def psca_iteration(prob: Problem, x: np.ndarray, rho: float) -> IterationRecord:
    """Steps 5-8 of Algorithm 1 for one iteration."""
    Sigma = model_covariance(prob.S, prob.weights(x), prob.sigma2)
    Sigma_inv = frobenius_inverse(Sigma)
    q, r = quadratic_forms(prob.S, Sigma_inv, prob.Sigma_hat)
    grad, curv = gradient_and_curvature(prob, x, q, r)
    lo, hi = prob.bounds()
    x_tilde = coordinate_step(x, grad, curv, lo, hi)
    x_next = (1.0 - rho) * x + rho * x_tilde
    return IterationRecord(x=x.copy(), q=q, r=r, x_tilde=x_tilde, rho=rho, x_next=x_next)


def step_sizes(iters: int, rho0: float = 0.5, decay: float = 0.5) -> np.ndarray:
    """rho_0 = rho0, rho_{k+1} = rho_k (1 - decay rho_k) (Sec. V)."""
    out = np.empty(iters)
    rho = rho0
    for k in range(iters):
        out[k] = rho
        rho = rho * (1.0 - decay * rho)
    return out


def psca(prob: Problem, iters: int, rho=None, record: bool = False):
    """Algorithm 1 from x^(0) = 0 for a fixed number of iterations.

    rho: None for the paper's schedule, else an explicit per-iteration list
    (used by the unrolled network, whose step sizes are learned).
    Returns x^(iters) and, if record, the list of IterationRecord."""
    rhos = step_sizes(iters) if rho is None else np.asarray(rho, dtype=np.float64)
    x = np.zeros(prob.N)
    hist = []
    for k in range(iters):
        rec = psca_iteration(prob, x, float(rhos[k]))
        if record:
            hist.append(rec)
        x = rec.x_next
    return (x, hist) if record else x


def bcd(prob: Problem, sweeps: int) -> np.ndarray:
    """Block coordinate descent from x = 0 (the sequential counterpart of
    PSCA: the BCD-ML-K listing of Sec. III-A, Algorithm 2, which Sec. IV-A
    carries over to gamma as BCD-ML-UD).  Each sweep visits n = 0..N-1 in
    order; device n takes the clipped coordinate step of eq. Solution_ML
    (Solution_ML_U) computed from the current inverse, x_n <- clip(x_n -
    grad_n / curv_n), and the inverse follows the change by the
    Sherman-Morrison (Woodbury) rank-one update.  ML-K and ML-UD only: there
    the step is the exact coordinate minimiser (the remark after Lemma 1)."""
    if prob.variant not in (ML_K, ML_UD):
        raise ValueError("bcd covers ML-K and ML-UD")
    N, L = prob.N, prob.S.shape[0]
    kappa = prob.g if prob.variant == ML_K else np.ones(N)
    lo, hi = prob.bounds()
    x = np.zeros(N)
    Si = np.eye(L) / prob.sigma2
    for _ in range(sweeps):
        for n in range(N):
            s = prob.S[:, n]
            b = Si @ s
            q = float(np.real(s.conj() @ b))
            r = float(np.real(b.conj() @ prob.Sigma_hat @ b))
            x_new = min(max(x[n] - kappa[n] * (q - r) / (kappa[n] * q) ** 2, lo), hi)
            d = (x_new - x[n]) * kappa[n]
            if d != 0.0:
                Si = Si - d * np.outer(b, b.conj()) / (1.0 + d * q)
            x[n] = x_new
    return x


def problem_from_instance(inst, variant: int, eps: float = 0.01, law: int = AREA_UNIFORM) -> Problem:
    """Wrap a generated instance (fields S, Y, g, p, sigma2, d_lo, d_hi,
    pl_c0, pl_beta) as an oracle Problem; SigmaHat is formed here.  `law` is
    the MAP-UR prior's distance law (reading R4)."""
    Sh = sample_covariance(inst.Y)
    N = inst.S.shape[1]
    kw = dict(Sigma_hat=Sh, S=np.asarray(inst.S, np.complex128), sigma2=float(inst.sigma2),
              M=int(inst.Y.shape[1]), variant=variant)
    if variant in KNOWN_PATHLOSS:
        kw["g"] = np.asarray(inst.g, np.float64)
    if variant == MAP_K:
        kw["p"] = np.full(N, float(inst.p))
    if variant == MAP_UR:
        kw["prior"] = make_prior(inst.p, inst.d_lo, inst.d_hi, inst.pl_c0, inst.pl_beta, eps, law)
    if variant == MAP_K2:
        kw["c1"], kw["C2"] = pairwise_prior(N, inst.c_single, *inst.pair_csr())
    return Problem(**kw)


def pairwise_prior(N: int, c_single: float, ptr, col, val):
    """First-order coefficients c_{n} = c_single and the pairwise matrix C of
    eq. second from its CSR arrays (rows n, entries c_{n,n'})."""
    from scipy.sparse import csr_matrix
    C = csr_matrix((np.asarray(val, np.float64), np.asarray(col), np.asarray(ptr)), shape=(N, N))
    return np.full(N, float(c_single)), C


# ---------------------------------------------------------------------------
# Detection and error rates (threshold module of Sec. III-A; P_MD = P_FA
# operating point)
# ---------------------------------------------------------------------------

def threshold(x: np.ndarray, theta: float) -> np.ndarray:
    """alpha_hat_n = 1[x_n >= theta]."""
    return (np.asarray(x) >= theta).astype(np.uint8)


def miss_false_alarm(scores: np.ndarray, truth: np.ndarray, theta: float):
    """(P_MD, P_FA) at threshold theta, pooled over all entries."""
    truth = np.asarray(truth).astype(bool)
    det = np.asarray(scores) >= theta
    n_act = max(int(truth.sum()), 1)
    n_ina = max(int((~truth).sum()), 1)
    pmd = float(np.sum(truth & ~det)) / n_act
    pfa = float(np.sum(~truth & det)) / n_ina
    return pmd, pfa


def equal_error_rate(scores: np.ndarray, truth: np.ndarray):
    """Threshold where P_MD = P_FA, searched over the candidate set of
    distinct scores: minimise |P_MD - P_FA|, then (P_MD + P_FA)/2, then
    prefer the larger threshold.  Returns (eer, theta, pmd, pfa) with
    eer = (P_MD + P_FA)/2 at that threshold."""
    scores = np.asarray(scores, dtype=np.float64).ravel()
    truth = np.asarray(truth).ravel()
    best = None
    for theta in np.unique(scores):
        pmd, pfa = miss_false_alarm(scores, truth, theta)
        key = (abs(pmd - pfa), 0.5 * (pmd + pfa), -theta)
        if best is None or key < best[0]:
            best = (key, theta, pmd, pfa)
    _, theta, pmd, pfa = best
    return 0.5 * (pmd + pfa), float(theta), pmd, pfa


def error_rate(scores: np.ndarray, truth: np.ndarray, theta: float) -> float:
    """Average error rate ||alpha_hat - alpha||_1 / (N I)."""
    det = threshold(scores, theta)
    return float(np.mean(np.abs(det.astype(np.int64) - np.asarray(truth).astype(np.int64))))


# ---------------------------------------------------------------------------
# Branch sensitivity of the MAP-UR prior (a property of eq. peps, used to
# qualify parity checks at finite precision)
# ---------------------------------------------------------------------------

def branch_margin(prob: Problem, hist) -> np.ndarray:
    """Per device, the smallest relative distance of its iterates x^(k) and
    x^(k+1) over a recorded trajectory to a branch point of p^eps
    (eps, g_l - eps, g_l).  The prior's gradient term has poles at eps from
    below and at g_l - eps from above and jumps at g_l, so a trajectory that
    passes within the working precision of one of them is not a continuous
    function of the inputs there."""
    pr = prob.prior
    pts = np.array([pr.eps, pr.g_l - pr.eps, pr.g_l])
    m = np.full(prob.N, np.inf)
    for rec in hist:
        for arr in (rec.x, rec.x_next):
            d = np.min(np.abs(arr[:, None] - pts[None, :]) / pts[None, :], axis=1)
            m = np.minimum(m, d)
    return m


# ---------------------------------------------------------------------------
# The unrolled network (PSCA-Net, Sec. III-A / IV-A "-Net" subsections): K
# layers, layer k is one iteration of Algorithm 1 with its own step size
# rho_k; loss: binary cross-entropy of the last iterate (eqs. Loss_alpha,
# Loss_gamma).  Gradients by the chain rule, written out per layer.
# ---------------------------------------------------------------------------

def net_forward(prob: Problem, rhos) -> list:
    """x^(0) = 0, ..., x^(K): the iterates of the unrolled network."""
    xs = [np.zeros(prob.N)]
    for rho in rhos:
        xs.append(psca_iteration(prob, xs[-1], float(rho)).x_next)
    return xs


def layer_vjp(prob: Problem, x: np.ndarray, rho: float, v: np.ndarray):
    """Vector-Jacobian product of one layer x' = (1 - rho) x + rho x~(x):
    returns (dL/dx, dL/drho) given v = dL/dx'.

    With kappa = g (known pathloss) or 1, grad = kappa (q - r) - c(x) (c the
    prior term, c' its derivative), curv = (kappa q)^2, pre = x - grad/curv,
    x~ = clip(pre, lo, hi) and mask = [lo <= pre <= hi]:
      d pre/dq = (2 grad - kappa q) / (kappa^2 q^3),  d pre/dr = 1 / (kappa q^2),
      d pre/dx_n (own) = 1 + c'(x_n) / curv_n,
    and, from d Sigma^-1 = -Sigma^-1 s_m s_m^H Sigma^-1 d w_m with w = kappa x,
      dq_n/dx_m = -kappa_m |s_n^H Sigma^-1 s_m|^2,
      dr_n/dx_m = -2 kappa_m Re[(s_n^H Sigma^-1 s_m)(s_m^H Sigma^-1 SigmaHat Sigma^-1 s_n)]."""
    N = prob.N
    known = prob.variant in KNOWN_PATHLOSS
    kappa = prob.g if known else np.ones(N)
    Sigma = model_covariance(prob.S, prob.weights(x), prob.sigma2)
    Si = np.linalg.inv(Sigma)
    q, r = quadratic_forms(prob.S, Si, prob.Sigma_hat)
    grad, curv = gradient_and_curvature(prob, x, q, r)
    lo, hi = prob.bounds()
    pre = x - grad / curv
    xt = np.minimum(np.maximum(pre, lo), hi)
    mask = ((pre >= lo) & (pre <= hi)).astype(np.float64)
    dpre_dq = (2.0 * grad - kappa * q) / (kappa ** 2 * q ** 3)
    dpre_dr = 1.0 / (kappa * q ** 2)
    if prob.variant == MAP_UR:
        cprime = np.array([prob.prior.dlog_ratio(float(xn)) for xn in x]) / prob.M
    else:
        cprime = np.zeros(N)
    own = 1.0 + cprime / curv
    d_rho = float(np.sum(v * (xt - x)))
    a = rho * v * mask * dpre_dq
    b = rho * v * mask * dpre_dr
    Bm = Si @ prob.S                                  # columns Sigma^-1 s_m
    Cm = Si @ prob.Sigma_hat @ Bm                     # columns Sigma^-1 SigmaHat Sigma^-1 s_m
    P = prob.S.conj().T @ Bm                          # P[n, m] = s_n^H Sigma^-1 s_m
    R = prob.S.conj().T @ Cm                          # R[n, m] = s_n^H Sigma^-1 SigmaHat Sigma^-1 s_m
    dq = -(np.abs(P) ** 2) * kappa[None, :]           # dq_n/dx_m
    dr = -2.0 * np.real(P * R.conj()) * kappa[None, :]  # dr_n/dx_m
    dx = v * (1.0 - rho) + rho * v * mask * own + a @ dq + b @ dr
    if prob.variant == MAP_K2:   # d pre_n / d x_m = c_{n,m} / (M curv_n): the pairwise prior couples devices
        dx = dx + rho * (prob.C2.T @ (v * mask / curv)) / prob.M
    return dx, d_rho


def bce_loss(prob: Problem, x: np.ndarray, alpha: np.ndarray, g: np.ndarray, clamp: float = 1e-7):
    """Binary cross-entropy of the detector output against the true activity
    (eq. Loss_alpha on alpha~; eq. Loss_gamma on gamma~/g), averaged over
    devices; the argument is clamped to [clamp, 1 - clamp] (the logarithms
    are undefined at 0 and 1).  Returns (loss, dloss/dx)."""
    known = prob.variant in KNOWN_PATHLOSS
    z = x if known else x / g
    zc = np.clip(z, clamp, 1.0 - clamp)
    N = x.shape[0]
    loss = -np.mean(alpha * np.log(zc) + (1.0 - alpha) * np.log(1.0 - zc))
    inside = ((z >= clamp) & (z <= 1.0 - clamp)).astype(np.float64)
    dz = -(alpha / zc - (1.0 - alpha) / (1.0 - zc)) / N * inside
    dx = dz if known else dz / g
    return float(loss), dx


def net_loss_and_grad(prob: Problem, rhos, alpha: np.ndarray, g: np.ndarray):
    """Loss of the unrolled network and its gradient with respect to every
    step size, by reverse accumulation through layer_vjp."""
    xs = net_forward(prob, rhos)
    loss, v = bce_loss(prob, xs[-1], alpha, g)
    d_rhos = np.zeros(len(rhos))
    for k in range(len(rhos) - 1, -1, -1):
        v, d_rhos[k] = layer_vjp(prob, xs[k], float(rhos[k]), v)
    return loss, d_rhos
