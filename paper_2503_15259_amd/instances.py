"""Seeded synthetic detection instances (system model only; no estimation arithmetic).

This module is the one piece shared by the FP64 oracle tests and the HIP path:
it draws the random quantities of the grant-free access model and nothing
else.  It never forms a covariance, a gradient or an estimate.

System model (paper Sec. II, eq. (signal)):  the base station receives
    Y = sum_n alpha_n sqrt(g_n) s_n h_n^T + Z          (L x M)
which we write as Y = S diag(sqrt(alpha * g)) H + Z with H in C^{N x M}
(the paper's compact forms (signal1)/(signal2) carry H with its transpose
implied).  Small-scale fading H and noise Z are i.i.d. circularly-symmetric
complex Gaussian (Sec. II, Rayleigh fading).

Workload recipe (the sizes come from the workloads this library targets):
  * pilots  S_ln ~ CN(0, 1) / sqrt(L)   (so E||s_n||^2 = 1)
  * distance d_n ~ U[0.05, 0.5] km
  * pathloss in dB  PL(d) = 128.1 + 37.6 log10(d_km), expressed in
    noise-normalised units with the paper's transmit power P = 23 dBm and
    noise power -114 dBm (Sec. V):  g_n = 10^((137 - PL(d_n)) / 10),
    sigma^2 = 1.  Equivalently g = phi(d) = c0 * d^-beta with
    c0 = 10^0.89, beta = 3.76.
  * activity alpha_n ~ Bernoulli(p)
  * H (N x M), Z (L x M) i.i.d. CN(0, 1)

Group-activity workload (the second-order activity model, eq. second): the
devices fall into groups of K_g (a random permutation cut into consecutive
runs); the activity follows p(alpha) proportional to
exp(sum_n a alpha_n + sum_{n<n' same group} b alpha_n alpha_n'), which
factorises over groups, so each group's pattern is drawn exactly from its
2^K_g states.  b > 0 makes devices of a group tend to be active together;
a is set so that every device is active with probability p.

Instance i of workload c uses numpy's Generator(PCG64(SeedSequence([c, i]))).
Draw order: (uneven batches only: N, L, M, p) -> S -> d -> alpha -> H -> Z.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Pathloss map in noise-normalised units: g = C0 * d_km^-BETA.
PL_C0 = 10.0 ** 0.89
PL_BETA = 3.76
D_LO_KM = 0.05
D_HI_KM = 0.5
SIGMA2 = 1.0


def pathloss(d_km: np.ndarray) -> np.ndarray:
    """g = 10^((137 - 128.1 - 37.6 log10 d) / 10)  (noise-normalised)."""
    return 10.0 ** ((137.0 - 128.1 - 37.6 * np.log10(d_km)) / 10.0)


@dataclass
class Instance:
    """One detection instance (all arrays FP64 / complex128, host memory).

    S      : (L, N) complex, pilot matrix, column n is s_n
    Y      : (L, M) complex, received pilots
    g      : (N,)  pathloss (known-pathloss variants take it as input)
    alpha  : (N,)  true activity in {0, 1}
    gamma  : (N,)  true effective pathloss alpha * g
    p      : activity probability used by the generator and the MAP priors
    """
    S: np.ndarray
    Y: np.ndarray
    g: np.ndarray
    alpha: np.ndarray
    d: np.ndarray
    p: float
    sigma2: float = SIGMA2
    d_lo: float = D_LO_KM
    d_hi: float = D_HI_KM
    pl_c0: float = PL_C0
    pl_beta: float = PL_BETA
    seed: tuple = field(default_factory=tuple)
    group: np.ndarray | None = None   # group-activity workload: group index of each device
    c_single: float = 0.0             # its coefficients a (every device) and b (pairs in a group)
    c_pair: float = 0.0

    def pair_csr(self):
        """CSR arrays (row pointers, columns, values) of the pairwise
        coefficients c_{n,n'} = b for n != n' in the same group, else 0."""
        N = self.N
        if self.group is None:
            return np.zeros(N + 1, np.int32), np.zeros(0, np.int32), np.zeros(0)
        members = {}
        for n, k in enumerate(self.group):
            members.setdefault(int(k), []).append(n)
        ptr = [0]
        col = []
        for n in range(N):
            row = [m for m in members[int(self.group[n])] if m != n]
            col.extend(sorted(row))
            ptr.append(len(col))
        return (np.asarray(ptr, np.int32), np.asarray(col, np.int32),
                np.full(len(col), float(self.c_pair)))

    @property
    def L(self) -> int:
        return self.S.shape[0]

    @property
    def N(self) -> int:
        return self.S.shape[1]

    @property
    def M(self) -> int:
        return self.Y.shape[1]

    @property
    def gamma(self) -> np.ndarray:
        return self.alpha * self.g

    def fp32_inputs(self) -> "Instance":
        """The same instance with every input of the detector rounded to
        single precision (and held in FP64 again): the values an FP32
        device path actually receives.  The true activity is unchanged."""
        def r32(a):
            return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)

        def c32(a):
            return np.asarray(a, dtype=np.complex128).astype(np.complex64).astype(np.complex128)

        return Instance(S=c32(self.S), Y=c32(self.Y), g=r32(self.g), alpha=self.alpha.copy(), d=self.d.copy(),
                        p=float(np.float32(self.p)), sigma2=float(np.float32(self.sigma2)),
                        d_lo=float(np.float32(self.d_lo)), d_hi=float(np.float32(self.d_hi)),
                        pl_c0=float(np.float32(self.pl_c0)), pl_beta=float(np.float32(self.pl_beta)),
                        seed=self.seed, group=None if self.group is None else self.group.copy(),
                        c_single=float(np.float32(self.c_single)), c_pair=float(np.float32(self.c_pair)))


def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    """i.i.d. CN(0, 1): independent N(0, 1/2) real and imaginary parts."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


def draw_instance(rng: np.random.Generator, N: int, L: int, M: int, p: float,
                  seed=()) -> Instance:
    """Draw S, d, alpha, H, Z in that order and assemble Y."""
    S = _cn(rng, (L, N)) / math.sqrt(L)
    d = rng.uniform(D_LO_KM, D_HI_KM, size=N)
    alpha = (rng.random(N) < p).astype(np.float64)
    H = _cn(rng, (N, M))
    Z = _cn(rng, (L, M)) * math.sqrt(SIGMA2)
    g = pathloss(d)
    amp = np.sqrt(alpha * g)
    Y = (S * amp[None, :]) @ H + Z
    return Instance(S=S, Y=Y, g=g, alpha=alpha, d=d, p=float(p), seed=tuple(seed))


def group_states(K: int) -> np.ndarray:
    """All 2^K activity patterns of a group, one per row."""
    return ((np.arange(2 ** K)[:, None] >> np.arange(K)[None, :]) & 1).astype(np.float64)


def group_pattern_probs(K: int, a: float, b: float) -> np.ndarray:
    """p(pattern) of one group of K under exp(a sum alpha + b sum_{pairs} alpha alpha)."""
    st = group_states(K)
    k = st.sum(axis=1)
    logw = a * k + b * k * (k - 1) / 2.0
    w = np.exp(logw - logw.max())
    return w / w.sum()


def group_first_order(K: int, p: float, b: float) -> float:
    """The coefficient a for which each device of a group is active with
    probability p (bisection; the marginal grows with a)."""
    lo, hi = -60.0, 60.0
    st = group_states(K)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        marg = float(group_pattern_probs(K, mid, b) @ st[:, 0])
        lo, hi = (mid, hi) if marg < p else (lo, mid)
    return 0.5 * (lo + hi)


def draw_group_instance(rng: np.random.Generator, N: int, L: int, M: int, p: float, K: int, b: float,
                        seed=()) -> Instance:
    """Group-activity instance: draw S, d, the grouping, the activity (exact
    per-group draws), H, Z in that order and assemble Y."""
    S = _cn(rng, (L, N)) / math.sqrt(L)
    d = rng.uniform(D_LO_KM, D_HI_KM, size=N)
    perm = rng.permutation(N)
    group = np.empty(N, np.int64)
    group[perm] = np.arange(N) // K
    a = group_first_order(K, p, b)
    states = group_states(K)
    probs = group_pattern_probs(K, a, b)
    n_groups = int(group.max()) + 1
    alpha = np.zeros(N)
    for k in range(n_groups):
        members = np.flatnonzero(group == k)
        st = states[rng.choice(len(probs), p=probs)] if len(members) == K else None
        if st is None:   # a short last group: its own exact law
            kk = len(members)
            st = group_states(kk)[rng.choice(2 ** kk, p=group_pattern_probs(kk, a, b))]
        alpha[np.sort(members)] = st
    H = _cn(rng, (N, M))
    Z = _cn(rng, (L, M)) * math.sqrt(SIGMA2)
    g = pathloss(d)
    amp = np.sqrt(alpha * g)
    Y = (S * amp[None, :]) @ H + Z
    return Instance(S=S, Y=Y, g=g, alpha=alpha, d=d, p=float(p), seed=tuple(seed), group=group,
                    c_single=a, c_pair=float(b))


def make_group_instance(workload: int, index: int, N: int, L: int, M: int, p: float, K: int,
                        b: float) -> Instance:
    """Group-activity instance `index` of workload `workload`."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload, index])))
    return draw_group_instance(rng, N, L, M, p, K, b, seed=(workload, index))


def make_instance(workload: int, index: int, N: int, L: int, M: int, p: float) -> Instance:
    """Fixed-shape instance `index` of workload `workload`."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload, index])))
    return draw_instance(rng, N, L, M, p, seed=(workload, index))


def make_uneven_instance(workload: int, index: int) -> Instance:
    """Uneven-batch instance: N ~ U{200..2000}, L in {32,48,64,96},
    M in {64,128,256}, p ~ U[0.05, 0.2], drawn before the instance itself."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload, index])))
    N = int(rng.integers(200, 2001))
    L = int(rng.choice([32, 48, 64, 96]))
    M = int(rng.choice([64, 128, 256]))
    p = float(rng.uniform(0.05, 0.2))
    return draw_instance(rng, N, L, M, p, seed=(workload, index))


# Named fixed-shape workloads: (N, L, M, p, iterations)
WORKLOADS = {
    "small": dict(N=100, L=20, M=32, p=0.1, iters=100),          # CPU-checkable case
    "single": dict(N=1000, L=64, M=128, p=0.1, iters=100),       # single instance, four variants
    "large": dict(N=10000, L=200, M=256, p=0.05, iters=200),     # large-scale case
}
WORKLOAD_IDS = {"small": 0, "single": 1, "uneven": 2, "net": 3, "large": 4, "group": 5}

# Group-activity workload (second-order activity model): sizes of the single
# workload, groups of 5, pair coefficient b.
GROUP_WORKLOAD = dict(N=1000, L=64, M=128, p=0.1, K=5, b=2.0, iters=100)


def workload_instance(name: str, index: int) -> Instance:
    w = WORKLOADS[name]
    return make_instance(WORKLOAD_IDS[name], index, w["N"], w["L"], w["M"], w["p"])


def group_instance(index: int, **over) -> Instance:
    """Instance `index` of the group-activity workload (sizes overridable)."""
    w = dict(GROUP_WORKLOAD, **over)
    return make_group_instance(WORKLOAD_IDS["group"], index, w["N"], w["L"], w["M"], w["p"], w["K"], w["b"])
