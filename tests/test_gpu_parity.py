"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2503_15259_amd import instances as I
from parity import (assert_parity, assert_same_support, map_ur_device_parity, parity_report,
                    stepwise_parity)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = [O.ML_K, O.MAP_K, O.ML_UD, O.MAP_UR]
EPS = float(np.float32(0.01))   # the value the FP32 parameter block carries


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15259_amd import psca
    return psca


def dev():
    return torch.device("cuda", 0)


def c64(a):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev())


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).astype(np.float32)).to(dev())


def params_for(P, inst, variant, iters):
    kw = dict(variant=variant, iters=iters, sigma2=inst.sigma2, M=inst.M,
              d_lo=inst.d_lo, d_hi=inst.d_hi, pl_c0=inst.pl_c0, pl_beta=inst.pl_beta, eps=EPS)
    if variant in O.KNOWN_PATHLOSS:
        kw["g"] = f32(inst.g)
    if variant == O.MAP_K:
        kw["p"] = f32(np.full(inst.N, inst.p))
    return P.Params(**kw)


def run_gpu(P, inst, variant, iters):
    Y, S = c64(inst.Y), c64(inst.S)
    status = torch.full((1,), 7, dtype=torch.int32, device=dev())
    x = P.detect_y(Y, S, params_for(P, inst, variant, iters), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return x.cpu().numpy()


def label(inst, variant, iters):
    return f"[{O.VARIANT_NAMES[variant]} N={inst.N} L={inst.L} M={inst.M} seed={inst.seed} iters={iters}]"


def test_sample_covariance(P):
    # M = 33 and 65: a ragged last chunk of Y's columns; L = 256 the largest pilot length
    for (N, L, M) in [(10, 1, 1), (30, 13, 7), (100, 64, 128), (50, 96, 256), (20, 200, 33), (40, 256, 65)]:
        inst = I.make_instance(7, L, N, L, M, 0.2).fp32_inputs()
        print(f"sample_cov L={L} M={M}", flush=True)
        got = P.sample_cov(c64(inst.Y))
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.complex128)
        ref = O.sample_covariance(inst.Y)
        assert np.linalg.norm(got - ref) <= 2e-6 * np.linalg.norm(ref)
        # exact products and FP64 sums, rounded once: within half an FP32 ulp of
        # each entry (real and imaginary parts), up to the FP64 sums' own error
        tol = lambda r: 2.0 ** -24 * (1 + 1e-6) * np.abs(r) + 1e-12 * np.abs(ref).max()
        assert np.all(np.abs(got.real - ref.real) <= tol(ref.real))
        assert np.all(np.abs(got.imag - ref.imag) <= tol(ref.imag))
        assert np.array_equal(got, got.conj().T)        # exactly Hermitian


def test_sample_covariance_batch(P):
    # B instances of one size in one launch, each bit-identical to its own
    # single call (same kernel, same arithmetic) and within half an FP32 ulp
    # of the oracle; padded instance strides; B = 0 launches nothing
    for (B, N, L, M, pad) in [(5, 30, 200, 33, 0), (3, 50, 64, 128, 7), (2, 20, 97, 5, 3)]:
        insts = [I.make_instance(11 + b, L + b, N, L, M, 0.2).fp32_inputs() for b in range(B)]
        print(f"sample_cov_batch B={B} L={L} M={M} pad={pad}", flush=True)
        buf = torch.zeros(B * (L * M + pad), dtype=torch.complex64, device="cuda")
        Yb = buf.as_strided((B, L, M), (L * M + pad, 1, L))
        for b, inst in enumerate(insts):
            Yb[b].copy_(c64(inst.Y))
        got = P.sample_cov_batch(Yb)
        singles = [P.sample_cov(c64(inst.Y)) for inst in insts]
        torch.cuda.synchronize()
        for b, inst in enumerate(insts):
            g = got[b].cpu().numpy()
            assert np.array_equal(g, singles[b].cpu().numpy())
            ref = O.sample_covariance(inst.Y)
            tol = lambda r: 2.0 ** -24 * (1 + 1e-6) * np.abs(r) + 1e-12 * np.abs(ref).max()
            g = g.astype(np.complex128)
            assert np.all(np.abs(g.real - ref.real) <= tol(ref.real))
            assert np.all(np.abs(g.imag - ref.imag) <= tol(ref.imag))
    empty = torch.empty((0, 8, 4), dtype=torch.complex64, device="cuda")
    assert P.sample_cov_batch(empty.as_strided((0, 8, 4), (32, 1, 8))).shape == (0, 8, 8)


@pytest.mark.parametrize("variant", VARIANTS)
def test_first_iteration_from_zero(P, variant):
    inst = I.workload_instance("small", 1).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    rec = O.psca_iteration(prob, np.zeros(inst.N), 0.5)
    Sh = P.sample_cov(c64(inst.Y))
    xn, q, r, xt = P.iterate(Sh, c64(inst.S), f32(np.zeros(inst.N)), 0.5, params_for(P, inst, variant, 1))
    torch.cuda.synchronize()
    for name, got, ref in [("q", q, rec.q), ("r", r, rec.r), ("x~", xt, rec.x_tilde), ("x+", xn, rec.x_next)]:
        got = got.cpu().numpy().astype(np.float64)
        tol = 2e-5 * np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
        assert np.all(np.abs(got - ref) <= tol), (name, np.max(np.abs(got - ref) / np.abs(ref).max()))


@pytest.mark.parametrize("variant", VARIANTS)
def test_iteration_from_a_mid_trajectory_point(P, variant):
    """Factorisation of a realistic Sigma (iterate 15 of the oracle)."""
    inst = I.workload_instance("single", 2).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    x15 = O.psca(prob, 15)
    rho = float(O.step_sizes(16)[15])
    rec = O.psca_iteration(prob, x15, rho)
    Sh = P.sample_cov(c64(inst.Y))
    xn, q, r, xt = P.iterate(Sh, c64(inst.S), f32(x15), rho, params_for(P, inst, variant, 1))
    torch.cuda.synchronize()
    q_gpu = q.cpu().numpy().astype(np.float64)
    qmr_gpu = q_gpu - r.cpu().numpy().astype(np.float64)
    qmr_ref = rec.q - rec.r
    q_err = float(np.max(np.abs(q_gpu - rec.q) / np.abs(rec.q)))
    # q - r nearly cancels near a stationary point, so its error is measured
    # against q, the scale of the two terms it is the difference of
    qmr_err = float(np.max(np.abs(qmr_gpu - qmr_ref) / np.abs(rec.q)))
    print(f"{label(inst, variant, 1)} iterate 15: max rel err q {q_err:.2e}, (q - r) / q {qmr_err:.2e}", flush=True)
    assert q_err < 1e-5 and qmr_err < 1e-5, (q_err, qmr_err)
    assert_parity(xn.cpu().numpy(), rec.x_next, variant, label(inst, variant, 1))


@pytest.mark.parametrize("variant", VARIANTS)
def test_detect_small_workload(P, variant):
    inst = I.workload_instance("small", 0).fp32_inputs()
    iters = 100
    ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
    got = run_gpu(P, inst, variant, iters)
    assert_parity(got, ref, variant, label(inst, variant, iters))
    assert_same_support(got, ref, inst.alpha, variant, label(inst, variant, iters))


@pytest.mark.parametrize("variant", VARIANTS)
def test_detect_single_instance_workload(P, variant):
    """Full-size single-instance workload: N = 1000, L = 64, M = 128, 100 iterations."""
    inst = I.workload_instance("single", 0).fp32_inputs()
    iters = 100
    ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
    print(label(inst, variant, iters), flush=True)
    got = run_gpu(P, inst, variant, iters)
    assert_parity(got, ref, variant, label(inst, variant, iters))
    assert_same_support(got, ref, inst.alpha, variant, label(inst, variant, iters))


@pytest.mark.parametrize("workload,index", [("small", 0), ("single", 0)])
def test_map_ur_with_the_uniform_in_distance_law(P, workload, index):
    """MAP-UR with the prior built on the generator's own distance law
    (uniform in d, dist_law = 1) against the oracle with the same law."""
    inst = I.workload_instance(workload, index).fp32_inputs()
    iters = 100
    prob = O.problem_from_instance(inst, O.MAP_UR, eps=EPS, law=O.UNIFORM_IN_D)
    ref, hist = O.psca(prob, iters, record=True)
    prm = params_for(P, inst, O.MAP_UR, iters)
    prm.dist_law = P.DIST_LINEAR
    status = torch.full((1,), 7, dtype=torch.int32, device=dev())
    x = P.detect_y(c64(inst.Y), c64(inst.S), prm, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    rep = map_ur_device_parity(x.cpu().numpy(), ref, O.branch_margin(prob, hist))
    print(f"MAP-UR uniform-in-d law {label(inst, O.MAP_UR, iters)}: {rep}", flush=True)
    assert rep["n_bad"] == 0, rep
    # the law changes the result (the prior's density piece differs)
    ref_area = O.psca(O.problem_from_instance(inst, O.MAP_UR, eps=EPS), iters)
    assert np.max(np.abs(ref_area - ref)) > 1e-3 * np.max(np.abs(ref))
    bad = params_for(P, inst, O.MAP_UR, 5)
    bad.dist_law = 2
    with pytest.raises(P.PscaError) as e:
        P.detect_y(c64(inst.Y), c64(inst.S), bad)
    assert e.value.code == -1


def test_map_ur_single_workload_every_device_outside_the_prior_poles(P):
    """MAP-UR on instances 0-3 of the N=1000, L=64 workload (100 iterations).
    Devices whose oracle trajectory passes within BRANCH_DELTA of a branch
    point of p^eps are excluded (and counted); every other device meets the
    element-wise bar.  Where the oracle itself is input-sensitive (its
    result moves beyond the bar when only its inputs are rounded to FP32:
    a pole crossing there perturbs every other device through Sigma), the
    whole trajectory is held step by step instead: one oracle iteration
    from each recorded GPU iterate against the GPU's next iterate, on every
    device not within BRANCH_DELTA of a branch point at that step."""
    iters = 100
    rhos = O.step_sizes(iters)
    for idx in range(4):
        inst64 = I.workload_instance("single", idx)
        inst = inst64.fp32_inputs()
        prob = O.problem_from_instance(inst, O.MAP_UR, eps=EPS)
        ref, hist = O.psca(prob, iters, record=True)
        margin = O.branch_margin(prob, hist)
        ref64 = O.psca(O.problem_from_instance(inst64, O.MAP_UR, eps=EPS), iters)
        shift = parity_report(ref64, ref, O.MAP_UR)
        Sh = P.sample_cov(c64(inst.Y))
        status = torch.full((1,), 7, dtype=torch.int32, device=dev())
        hist_gpu = P.net_forward(Sh, c64(inst.S), params_for(P, inst, O.MAP_UR, iters), status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        hist_gpu = hist_gpu.cpu().numpy()
        got = hist_gpu[-1].astype(np.float64)
        rep = map_ur_device_parity(got, ref, margin)
        sensitive = shift["n_bad"] > 0
        print(f"MAP-UR single instance {idx}: {rep['excluded']} devices near a branch point; "
              f"input-sensitive {sensitive}; {rep}", flush=True)
        if not sensitive:
            assert rep["n_bad"] == 0, (idx, rep)
            assert_same_support(got, ref, inst.alpha, O.MAP_UR, f"MAP-UR instance {idx}")
        worst, skipped = stepwise_parity(prob, hist_gpu, rhos)
        print(f"  step by step: {skipped} device-steps skipped near a branch point; worst {worst}", flush=True)
        assert worst["n_bad"] == 0, (idx, worst)


@pytest.mark.parametrize("N,L,M", [(1, 1, 4), (1, 8, 16), (65, 13, 9), (129, 3, 40), (200, 96, 64),
                                   (300, 96, 256), (64, 64, 64), (1000, 33, 128), (250, 72, 64), (90, 80, 32)])
def test_detect_ragged_and_edge_shapes(P, N, L, M):
    inst = I.make_instance(5, N * 1000 + L, N, L, M, 0.2).fp32_inputs()
    for variant in (O.ML_K, O.ML_UD):
        iters = 30
        ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
        print(label(inst, variant, iters), flush=True)
        got = run_gpu(P, inst, variant, iters)
        assert_parity(got, ref, variant, label(inst, variant, iters))


def test_zero_iterations_returns_zero(P):
    inst = I.make_instance(5, 1, 70, 8, 16, 0.2).fp32_inputs()
    got = run_gpu(P, inst, O.ML_UD, 0)
    assert np.array_equal(got, np.zeros(inst.N, np.float32))


def test_explicit_step_sizes_match_schedule(P):
    inst = I.workload_instance("small", 2).fp32_inputs()
    iters = 12
    rho = f32(O.step_sizes(iters))
    prm = params_for(P, inst, O.ML_K, iters)
    prm.rho = rho
    x = P.detect_y(c64(inst.Y), c64(inst.S), prm)
    ref = O.psca(O.problem_from_instance(inst, O.ML_K), iters)
    torch.cuda.synchronize()
    assert_parity(x.cpu().numpy(), ref, O.ML_K)


def test_threshold_bit_exact(P):
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, 1001).astype(np.float32)
    x[::7] = 0.5
    got = P.threshold(f32(x), 0.5)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), O.threshold(x, np.float32(0.5)))


def test_not_positive_definite_is_reported_and_iterate_held(P):
    """A negative iterate makes Sigma indefinite; the device reports it and
    leaves x unchanged (forced from the host: no fault, every kernel exits)."""
    inst = I.make_instance(5, 2, 80, 8, 16, 0.2).fp32_inputs()
    Sh = P.sample_cov(c64(inst.Y))
    x_in = f32(np.full(inst.N, -10.0))
    status = torch.zeros(1, dtype=torch.int32, device=dev())
    xn, _, _, _ = P.iterate(Sh, c64(inst.S), x_in, 0.5, params_for(P, inst, O.ML_UD, 1), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == -2
    assert np.array_equal(xn.cpu().numpy(), x_in.cpu().numpy())
    # a non-finite iterate is reported the same way
    x_nan = f32(np.full(inst.N, np.nan))
    xn, _, _, _ = P.iterate(Sh, c64(inst.S), x_nan, 0.5, params_for(P, inst, O.ML_UD, 1), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == -2


def test_host_validation_errors(P):
    inst = I.make_instance(5, 3, 20, 8, 16, 0.2).fp32_inputs()
    Y, S = c64(inst.Y), c64(inst.S)
    with pytest.raises(P.PscaError) as e:
        P.detect_y(Y, S, P.Params(variant=O.ML_K, iters=5, M=16))          # g missing
    assert e.value.code == -1
    with pytest.raises(P.PscaError):
        P.detect_y(Y, S, P.Params(variant=O.ML_UD, iters=5, M=16, sigma2=0.0))
    with pytest.raises(P.PscaError):
        P.detect_y(Y, S, P.Params(variant=O.ML_UD, iters=5, M=16, rho0=1.5))
    with pytest.raises(P.PscaError):
        P.detect_y(Y, S, P.Params(variant=O.MAP_UR, iters=5, M=16, eps=100.0))   # 2 eps >= g_l
    big = I.make_instance(5, 4, 20, 257, 8, 0.2).fp32_inputs()
    with pytest.raises(P.PscaError) as e:
        P.detect_y(c64(big.Y), c64(big.S), P.Params(variant=O.ML_UD, iters=5, M=8))
    assert e.value.code == -5


def test_batch_mixed_instances_match_oracle_and_single_calls(P):
    """psca_detect_batch over instances of different L, N, M, variant and
    iteration count: each result meets the oracle bar and agrees with the
    same instance run alone to the same bar (the batch may tile the devices
    differently, which changes the summation order of Sigma)."""
    cases = [(O.ML_K, I.workload_instance("single", 0).fp32_inputs(), 40),
             (O.MAP_K, I.make_instance(5, 11, 300, 20, 16, 0.15).fp32_inputs(), 25),
             (O.ML_UD, I.make_instance(5, 12, 700, 96, 64, 0.1).fp32_inputs(), 20),
             (O.MAP_UR, I.workload_instance("small", 0).fp32_inputs(), 60),
             (O.ML_UD, I.make_instance(5, 13, 17, 5, 8, 0.3).fp32_inputs(), 10),
             (O.ML_K, I.make_instance(5, 14, 400, 72, 64, 0.1).fp32_inputs(), 30)]
    probs, refs, singles = [], [], []
    for variant, inst, iters in cases:
        Sh = P.sample_cov(c64(inst.Y))
        prm = params_for(P, inst, variant, iters)
        probs.append(P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=prm,
                               status=torch.full((1,), 7, dtype=torch.int32, device=dev())))
        singles.append(P.detect(Sh, c64(inst.S), prm))
        refs.append(O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters))
    outs = P.detect_batch(probs)
    torch.cuda.synchronize()
    for (variant, inst, iters), pb, x, xs, ref in zip(cases, probs, outs, singles, refs):
        assert int(pb.status.item()) == 0
        got = x.cpu().numpy().astype(np.float64)
        assert_parity(got, ref, variant, "batch " + label(inst, variant, iters))
        assert_parity(got, xs.cpu().numpy().astype(np.float64), variant, "batch vs single " + label(inst, variant, iters))


def test_batch_larger_than_the_gpu_shares_teams(P):
    """Seven N=2000 instances at 16-column tiles would need 7 x 125
    workgroups, more than are co-resident: the persistent launch gives them
    smaller teams that work through several instances each, every result
    to the oracle bar."""
    probs, refs, insts = [], [], []
    for k in range(7):
        inst = I.make_instance(5, 100 + k, 2000, 32, 64, 0.1).fp32_inputs()
        variant = (O.ML_K, O.ML_UD)[k % 2]
        prm = params_for(P, inst, variant, 15)
        probs.append(P.Problem(Sigma_hat=P.sample_cov(c64(inst.Y)), S=c64(inst.S), params=prm,
                               status=torch.full((1,), 7, dtype=torch.int32, device=dev())))
        refs.append((variant, O.psca(O.problem_from_instance(inst, variant, eps=EPS), 15)))
        insts.append(inst)
    print("[batch 7 x N=2000 L=32 M=64 iters=15]", flush=True)
    outs = P.detect_batch(probs)
    torch.cuda.synchronize()
    for pb, x, (variant, ref), inst in zip(probs, outs, refs, insts):
        assert int(pb.status.item()) == 0
        assert_parity(x.cpu().numpy().astype(np.float64), ref, variant, "rounds " + label(inst, variant, 15))


def test_batch_validation_and_empty(P):
    inst = I.make_instance(5, 3, 20, 8, 16, 0.2).fp32_inputs()
    Sh = P.sample_cov(c64(inst.Y))
    assert P.detect_batch([]) == []
    bad = params_for(P, inst, O.ML_K, 5)
    bad.g = None
    with pytest.raises(P.PscaError) as e:
        P.detect_batch([P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=params_for(P, inst, O.ML_UD, 5)),
                        P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=bad)])
    assert e.value.code == -1
    good = [P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=params_for(P, inst, O.ML_UD, 5))]
    for spec in (-7, -144, -1, 100000):   # mixed specs are multiples of 16 up to 128 columns
        with pytest.raises(P.PscaError) as e:
            P.Plan(good, team_size=spec)
        assert e.value.code == -1, spec


def _uneven_batch(P, count, iters, variant=O.ML_UD):
    probs, refs, insts = [], [], []
    for k in range(count):
        inst = I.make_uneven_instance(I.WORKLOAD_IDS["uneven"], k).fp32_inputs()
        prm = params_for(P, inst, variant, iters)
        probs.append(P.Problem(Sigma_hat=P.sample_cov(c64(inst.Y)), S=c64(inst.S), params=prm,
                               status=torch.full((1,), 7, dtype=torch.int32, device=dev())))
        insts.append(inst)
    for inst in insts:
        refs.append(O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters))
    return probs, refs, insts


def test_uneven_batch_matches_oracle_for_every_team_size(P):
    """Uneven batch (N ~ U{200..2000}, L in {32,48,64,96}, M in {64,128,256},
    p ~ U[0.05, 0.2]) in one persistent launch, with the default team size,
    with forced uniform teams and with mixed teams (sized per instance for
    32- and 64-column tiles): every instance meets the oracle bar."""
    probs, refs, insts = _uneven_batch(P, 12, 20)
    print("[uneven batch 12 instances, ML-UD, 20 iterations]", flush=True)
    outs = P.detect_batch(probs)
    torch.cuda.synchronize()
    results = {"default": [x.cpu().numpy().astype(np.float64) for x in outs]}
    for pb in probs:
        assert int(pb.status.item()) == 0
    for T in (32, 80, -32, -64, -96, -112, -128):
        for pb in probs:
            pb.out = None
        plan = P.Plan(probs, team_size=T)
        assert plan.team_size == T
        print(f"[uneven batch, team size {T}]", flush=True)
        outs = plan.launch()
        torch.cuda.synchronize()
        results[T] = [x.cpu().numpy().astype(np.float64) for x in outs]
        plan.close()
    for key, xs in results.items():
        for inst, x, ref in zip(insts, xs, refs):
            assert_parity(x, ref, O.ML_UD, f"team={key} " + label(inst, O.ML_UD, 20))


def test_forward_batch_on_112_column_tiles(P):
    """The training forward's launch shape: N = 1000, L = 64 on a team of 9
    workgroups, i.e. 112-column tiles (seven 16-column blocks per
    workgroup), every recorded iterate of ML-K and MAP-UR against the
    oracle's trajectory."""
    inst = I.workload_instance("single", 1).fp32_inputs()
    iters = 20
    Sh = P.sample_cov(c64(inst.Y))
    for variant in (O.ML_K, O.MAP_UR):
        hist = torch.empty((iters + 1, inst.N), dtype=torch.float32, device=dev())
        status = torch.full((1,), 7, dtype=torch.int32, device=dev())
        pb = P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=params_for(P, inst, variant, iters), hist=hist,
                       status=status)
        plan = P.Plan([pb], team_size=9)
        assert plan.team_size == 9
        print(f"[112-column tiles: {label(inst, variant, iters)}]", flush=True)
        plan.launch()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        _, recs = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters, record=True)
        h = hist.cpu().numpy().astype(np.float64)
        for k, rec in enumerate(recs):
            assert_parity(h[k + 1], rec.x_next, variant, f"112-column tiles, iterate {k + 1} " +
                          label(inst, variant, iters))
        plan.close()


def test_uneven_full_batch_sampled_against_oracle(P):
    """The uneven configuration at full size, launched as the benchmark does:
    4096 ML-UD detections (100 iterations) cycling 64 distinct instances, team
    size from the autotuner.  Every device status is 0; every copy of an
    instance returns the same vector bit for bit (same tiles and reduction
    order wherever it runs); four sampled instances meet the oracle bar."""
    pool, iters, B = 64, 100, 4096
    wid = I.WORKLOAD_IDS["uneven"]
    insts = [I.make_uneven_instance(wid, k).fp32_inputs() for k in range(pool)]
    Ss = [c64(x.S) for x in insts]
    Shs = [P.sample_cov(c64(x.Y)) for x in insts]
    status = torch.full((B,), 7, dtype=torch.int32, device=dev())
    probs = [P.Problem(Sigma_hat=Shs[b % pool], S=Ss[b % pool],
                       params=P.Params(variant=O.ML_UD, iters=iters, sigma2=insts[b % pool].sigma2,
                                       M=insts[b % pool].M),
                       status=status[b:b + 1]) for b in range(B)]
    print(f"[uneven full batch: {B} instances, ML-UD, {iters} iterations]", flush=True)
    T = P.autotune_batch(probs, tune_iters=4)
    plan = P.Plan(probs, team_size=T)
    outs = plan.launch()
    torch.cuda.synchronize()
    assert int((status != 0).sum().item()) == 0
    got = torch.cat(outs)
    first = torch.cat([outs[b % pool] for b in range(B)])
    assert torch.equal(got, first)
    assert bool(torch.isfinite(got).all()) and bool((got >= 0).all())
    for k in (0, 17, 40, 63):
        ref = O.psca(O.problem_from_instance(insts[k], O.ML_UD, eps=EPS), iters)
        assert_parity(outs[k].cpu().numpy().astype(np.float64), ref, O.ML_UD,
                      f"full batch, team={T} " + label(insts[k], O.ML_UD, iters))
    plan.close()


def test_plan_replays_inside_a_captured_graph(P):
    """A planned batch captured into a graph and replayed three times, with
    eager work and synchronisation between replays: every replay reproduces
    the eager launch exactly."""
    probs, refs, insts = _uneven_batch(P, 6, 15)
    plan = P.Plan(probs)
    eager = [x.clone() for x in plan.launch()]
    torch.cuda.synchronize()
    for inst, x, ref in zip(insts, eager, refs):
        assert_parity(x.cpu().numpy().astype(np.float64), ref, O.ML_UD, "eager plan " + label(inst, O.ML_UD, 15))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    print("[capture plan launch]", flush=True)
    with torch.cuda.graph(graph):
        plan.launch()
    for rep in range(3):
        for x in plan.outs:
            x.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for x, e in zip(plan.outs, eager):
            assert torch.equal(x, e), f"replay {rep}"
        for pb in probs:
            assert int(pb.status.item()) == 0
    del graph
    plan.close()


def test_autotuner_choice_is_used_and_exact(P):
    probs, refs, insts = _uneven_batch(P, 5, 12)
    T = P.autotune_batch(probs, tune_iters=2)
    assert 1 <= T <= 256 or (T < 0 and -T % 16 == 0 and -T <= 128), T
    for pb in probs:
        pb.out = None
    outs = P.detect_batch(probs)
    torch.cuda.synchronize()
    for inst, x, ref in zip(insts, outs, refs):
        assert_parity(x.cpu().numpy().astype(np.float64), ref, O.ML_UD, f"tuned T={T} " + label(inst, O.ML_UD, 12))


def test_long_team_lists_finish_without_barrier_timeouts(P):
    """Forty uneven instances on 32-workgroup teams (each team works through
    several instances of different sizes in one launch): every instance
    reports OK and meets the oracle bar."""
    probs, refs, insts = _uneven_batch(P, 40, 10)
    plan = P.Plan(probs, team_size=32)
    print("[40 uneven instances on teams of 32]", flush=True)
    outs = plan.launch()
    torch.cuda.synchronize()
    for pb in probs:
        assert int(pb.status.item()) == 0
    for inst, x, ref in zip(insts, outs, refs):
        assert_parity(x.cpu().numpy().astype(np.float64), ref, O.ML_UD, "team lists " + label(inst, O.ML_UD, 10))
    plan.close()


@pytest.mark.parametrize("N,L,M", [(50, 97, 32), (300, 130, 64), (200, 200, 256), (129, 256, 40)])
def test_large_pilot_lengths_match_oracle(P, N, L, M):
    """L above 96 (the cooperative factorisation in device memory)."""
    inst = I.make_instance(5, 7000 + N + L, N, L, M, 0.2).fp32_inputs()
    for variant in (O.ML_K, O.ML_UD, O.MAP_UR):
        iters = 15
        ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
        print(label(inst, variant, iters), flush=True)
        got = run_gpu(P, inst, variant, iters)
        assert_parity(got, ref, variant, label(inst, variant, iters))


def test_large_scale_workload_size(P):
    """The large-scale size, N = 10^4 devices, L = 200, M = 256 (p = 0.05):
    ten iterations of ML-K and MAP-UR, every device against the oracle."""
    inst = I.workload_instance("large", 0).fp32_inputs()
    for variant in (O.ML_K, O.MAP_UR):
        iters = 10
        ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
        print(label(inst, variant, iters), flush=True)
        got = run_gpu(P, inst, variant, iters)
        assert_parity(got, ref, variant, label(inst, variant, iters))


def _large_case(P, inst, variant, iters):
    Sh = P.sample_cov(c64(inst.Y))
    prm = params_for(P, inst, variant, iters)
    status = torch.full((1,), 7, dtype=torch.int32, device=dev())
    return P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=prm, status=status)


@pytest.mark.parametrize("team", [0, 1, 2, 5])
def test_large_pilot_length_batch_matches_oracle_and_single_calls(P, team):
    """Batches with 97 <= L <= 256 (Sigma factored in memory by each
    instance's team): instances of different L, N, M, variant and iteration
    count in one persistent launch, on default and forced team sizes (a team
    of one workgroup holds every tile and column block of its instance).
    Each result meets the oracle bar and agrees with the same instance run
    alone to the same bar."""
    cases = [(O.ML_K, I.make_instance(5, 31, 300, 97, 32, 0.2).fp32_inputs(), 12),
             (O.ML_UD, I.make_instance(5, 32, 1000, 130, 64, 0.1).fp32_inputs(), 9),
             (O.MAP_UR, I.make_instance(5, 33, 777, 200, 256, 0.1).fp32_inputs(), 8),
             (O.MAP_K, I.make_instance(5, 34, 129, 256, 40, 0.2).fp32_inputs(), 7),
             (O.ML_K, I.make_instance(5, 35, 33, 113, 16, 0.3).fp32_inputs(), 10)]
    probs = [_large_case(P, inst, v, it) for v, inst, it in cases]
    for pb, (v, inst, _) in zip(probs, cases):
        if v == O.MAP_K:
            pb.params.p = f32(np.full(inst.N, inst.p))
    singles = [P.detect(pb.Sigma_hat, pb.S, pb.params) for pb in probs]
    print(f"[large-L batch, team {team}]", flush=True)
    if team == 0:
        outs = P.detect_batch(probs)
    else:
        plan = P.Plan(probs, team_size=team)
        assert plan.team_size == team
        outs = plan.launch()
    torch.cuda.synchronize()
    for (variant, inst, iters), pb, x, xs in zip(cases, probs, outs, singles):
        assert int(pb.status.item()) == 0
        ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
        got = x.cpu().numpy().astype(np.float64)
        assert_parity(got, ref, variant, f"large batch team={team} " + label(inst, variant, iters))
        assert_parity(got, xs.cpu().numpy().astype(np.float64), variant, "large batch vs single " +
                      label(inst, variant, iters))
    if team:
        plan.close()


def test_large_pilot_length_batch_validation(P):
    small = I.make_instance(5, 36, 50, 64, 16, 0.2).fp32_inputs()
    big = I.make_instance(5, 37, 50, 100, 16, 0.2).fp32_inputs()
    probs = [_large_case(P, small, O.ML_UD, 3), _large_case(P, big, O.ML_UD, 3)]
    with pytest.raises(P.PscaError) as e:   # one launch takes one of the two kernels
        P.detect_batch(probs)
    assert e.value.code == -5
    with pytest.raises(P.PscaError) as e:   # large-L plans take uniform teams only
        P.Plan(probs[1:], team_size=-64)
    assert e.value.code == -1


def test_large_pilot_length_iterate_and_network_forward(P):
    """One iteration from a mid-trajectory point at L = 200 (q, q - r and
    x~ against the oracle), and a network forward with explicit step sizes
    whose recorded iterates follow the oracle's."""
    inst = I.make_instance(5, 38, 2000, 200, 256, 0.05).fp32_inputs()
    prob = O.problem_from_instance(inst, O.ML_K, eps=EPS)
    x8 = O.psca(prob, 8)
    rho = 0.37
    rec = O.psca_iteration(prob, x8, rho)
    Sh = P.sample_cov(c64(inst.Y))
    xn, q, r, xt = P.iterate(Sh, c64(inst.S), f32(x8), rho, params_for(P, inst, O.ML_K, 1))
    torch.cuda.synchronize()
    qg = q.cpu().numpy().astype(np.float64)
    qmr = qg - r.cpu().numpy().astype(np.float64)
    q_err = float(np.max(np.abs(qg - rec.q) / np.abs(rec.q)))
    qmr_err = float(np.max(np.abs(qmr - (rec.q - rec.r)) / np.abs(rec.q)))
    print(f"L=200 iterate: q {q_err:.2e}, (q - r) / q {qmr_err:.2e}", flush=True)
    assert q_err < 1e-5 and qmr_err < 1e-5
    assert_parity(xt.cpu().numpy(), rec.x_tilde, O.ML_K, "L=200 x~")
    assert_parity(xn.cpu().numpy(), rec.x_next, O.ML_K, "L=200 x+")
    rhos = np.array([0.5, 0.7, 0.3, 0.45, 0.6, 0.2], dtype=np.float32)
    prm = params_for(P, inst, O.ML_K, len(rhos))
    prm.rho = f32(rhos)
    hist = P.net_forward(Sh, c64(inst.S), prm).cpu().numpy().astype(np.float64)
    _, recs = O.psca(prob, len(rhos), rho=rhos.astype(np.float64), record=True)
    for k, rc in enumerate(recs):
        assert_parity(hist[k + 1], rc.x_next, O.ML_K, f"L=200 network layer {k}")


@pytest.mark.parametrize("N,L,M,variant", [(300, 32, 64, O.ML_K), (500, 64, 128, O.MAP_K), (400, 130, 64, O.ML_UD)])
def test_detection_from_a_given_starting_iterate(P, N, L, M, variant):
    """params.x0: a detection that starts from x^(0) = x0 (here the oracle's
    6th iterate from zero) equals the oracle's iterations from x0 with the
    same schedule, single and batched (L <= 96 and L > 96); x0 may not alias
    the output."""
    inst = I.make_instance(5, 900 + N + L, N, L, M, 0.1).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    x0 = O.psca(prob, 6).astype(np.float32).astype(np.float64)   # the start the kernel sees
    iters = 12
    x_ref = x0.copy()
    for rho in O.step_sizes(iters):
        x_ref = O.psca_iteration(prob, x_ref, float(rho)).x_next
    Sh = P.sample_cov(c64(inst.Y))
    prm = params_for(P, inst, variant, iters)
    prm.x0 = f32(x0)
    status = torch.full((1,), 7, dtype=torch.int32, device=dev())
    print(f"[x0 start {O.VARIANT_NAMES[variant]} N={N} L={L}]", flush=True)
    x = P.detect(Sh, c64(inst.S), prm, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert_parity(x.cpu().numpy(), x_ref, variant, "x0 single")
    st2 = torch.full((2,), 7, dtype=torch.int32, device=dev())
    probs = [P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=prm, status=st2[0:1]),
             P.Problem(Sigma_hat=Sh, S=c64(inst.S), params=params_for(P, inst, variant, iters), status=st2[1:2])]
    xs = P.detect_batch(probs)
    torch.cuda.synchronize()
    assert st2.cpu().tolist() == [0, 0]
    assert_parity(xs[0].cpu().numpy(), x_ref, variant, "x0 batch")
    assert_parity(xs[1].cpu().numpy(), O.psca(prob, iters), variant, "zero start in the same batch")
    with pytest.raises(P.PscaError) as e:   # the start may not be the output
        P.detect(Sh, c64(inst.S), prm, out=prm.x0)
    assert e.value.code == -1


def test_large_pilot_length_batch_beyond_the_gpu(P):
    """300 instances with 97 <= L <= 128 on teams of one workgroup: more
    instances than co-resident workgroups, so teams work through lists of
    several instances (longest first).  Every status is clean, every result
    agrees with the same instance alone (its own launch) at the bar, and
    sampled instances meet the oracle bar."""
    rng = np.random.default_rng(31)
    probs, insts, variants = [], [], []
    for k in range(300):
        N = int(rng.integers(97, 301))
        L = int(rng.choice([97, 112, 128]))
        inst = I.make_instance(6, k, N, L, 32, 0.1).fp32_inputs()
        variant = (O.ML_K, O.ML_UD)[k % 2]
        probs.append(P.Problem(Sigma_hat=P.sample_cov(c64(inst.Y)), S=c64(inst.S),
                               params=params_for(P, inst, variant, 5),
                               status=torch.full((1,), 7, dtype=torch.int32, device=dev())))
        insts.append(inst)
        variants.append(variant)
    print("[large-L batch of 300 on teams of 1]", flush=True)
    plan = P.Plan(probs, team_size=1)
    outs = [x.clone() for x in plan.launch()]
    torch.cuda.synchronize()
    plan.close()
    assert all(int(pb.status.item()) == 0 for pb in probs)
    for k in range(0, 300, 23):   # against the instance run alone
        x1 = P.detect(probs[k].Sigma_hat, probs[k].S, probs[k].params)
        torch.cuda.synchronize()
        assert_parity(outs[k].cpu().numpy(), x1.cpu().numpy().astype(np.float64), variants[k], f"alone {k}")
    for k in (0, 151, 299):   # against the oracle
        ref = O.psca(O.problem_from_instance(insts[k], variants[k], eps=EPS), 5)
        assert_parity(outs[k].cpu().numpy(), ref, variants[k], f"oracle {k}")
