"""Unrolled network (PSCA-Net) on the GPU against the FP64 oracle: the
per-layer backward kernel, the recorded forward pass, the step-size gradient
and a short training run (needs an MI355X)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2503_15259_amd import instances as I
from parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = [O.ML_K, O.MAP_K, O.ML_UD, O.MAP_UR]
EPS = float(np.float32(0.01))


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


def params_for(P, inst, variant, iters=1):
    kw = dict(variant=variant, iters=iters, sigma2=inst.sigma2, M=inst.M, d_lo=inst.d_lo, d_hi=inst.d_hi,
              pl_c0=inst.pl_c0, pl_beta=inst.pl_beta, eps=EPS)
    if variant in O.KNOWN_PATHLOSS:
        kw["g"] = f32(inst.g)
    if variant == O.MAP_K:
        kw["p"] = f32(np.full(inst.N, inst.p))
    return P.Params(**kw)


CASES = [(20, 8, 64), (100, 20, 32), (300, 64, 128)]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("N,L,M", CASES)
def test_layer_backward_matches_oracle_vjp(P, variant, N, L, M):
    inst = I.make_instance(3, 500 + N + L, N, L, M, 0.2).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    _, hist = O.psca(prob, 6, record=True)
    x = np.asarray(hist[5].x, np.float32).astype(np.float64)   # the input the kernel sees
    rho = 0.3
    v = np.random.default_rng(N + L + variant).standard_normal(N)
    v = v.astype(np.float32).astype(np.float64)
    dx_ref, drho_ref = O.layer_vjp(prob, x, rho, v)
    Sh = P.sample_cov(c64(inst.Y))
    status = torch.full((1,), 7, dtype=torch.int32, device=dev())
    print(f"[layer backward {O.VARIANT_NAMES[variant]} N={N} L={L} M={M}]", flush=True)
    gx, gr = P.layer_backward(Sh, c64(inst.S), params_for(P, inst, variant), rho, f32(x), f32(v), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    gx = gx.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(dx_ref))
    err = np.max(np.abs(gx - dx_ref)) / scale
    assert err < 2e-3, (O.VARIANT_NAMES[variant], N, L, err)
    assert float(gr.item()) == pytest.approx(drho_ref, rel=2e-3, abs=1e-6 * np.sum(np.abs(v)) * np.max(np.abs(x)))


@pytest.mark.parametrize("variant", VARIANTS)
def test_net_forward_records_the_oracle_trajectory(P, variant):
    inst = I.workload_instance("small", 3).fp32_inputs()
    rhos = np.random.default_rng(variant).uniform(0.2, 0.8, 8).astype(np.float32)
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    ref = O.net_forward(prob, rhos.astype(np.float64))
    prm = params_for(P, inst, variant, iters=8)
    prm.rho = torch.from_numpy(rhos).to(dev())
    hist = P.net_forward(P.sample_cov(c64(inst.Y)), c64(inst.S), prm)
    torch.cuda.synchronize()
    assert hist.shape == (9, inst.N)
    assert torch.count_nonzero(hist[0]) == 0
    for k in range(1, 9):
        assert_parity(hist[k].cpu().numpy().astype(np.float64), ref[k], variant, f"layer {k}")


@pytest.mark.parametrize("variant", [O.ML_K, O.MAP_K, O.ML_UD])
def test_network_step_size_gradient_matches_oracle(P, variant):
    """Whole-network gradient against the oracle's reverse accumulation.  MAP-UR
    is covered layer by layer above: after a few layers many gamma~/g sit at
    the BCE clamp and near the prior's branch points, where the FP32 and FP64
    trajectories need not take the same branch."""
    from paper_2503_15259_amd import net as NET
    inst = I.make_instance(3, 900 + variant, 60, 16, 64, 0.2).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    K = 5
    rhos = np.asarray(NET.schedule(K), np.float32).astype(np.float64)
    loss_ref, g_ref = O.net_loss_and_grad(prob, rhos, inst.alpha, inst.g)
    model = NET.PscaNet(K, params_for(P, inst, variant))
    Sh = P.sample_cov(c64(inst.Y))
    x = model(Sh, c64(inst.S))
    loss = NET.bce(x, f32(inst.alpha), f32(inst.g), model.known)
    loss.backward()
    torch.cuda.synchronize()
    assert loss.item() == pytest.approx(loss_ref, rel=1e-3)
    got = model.rho.grad.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, g_ref, rtol=5e-3, atol=5e-3 * np.max(np.abs(g_ref)))


def test_training_lowers_the_loss(P):
    """A few Adam steps of an ML-UD network on generated instances lower the
    training loss and keep every step size in [0, 1]."""
    from paper_2503_15259_amd import net as NET
    insts = [I.make_instance(I.WORKLOAD_IDS["net"], 10 + k, 100, 20, 32, 0.1).fp32_inputs() for k in range(4)]
    model = NET.PscaNet(6, params_for(P, insts[0], O.ML_UD))
    batch = []
    for inst in insts:
        prm = params_for(P, inst, O.ML_UD)
        batch.append((P.sample_cov(c64(inst.Y)), c64(inst.S), prm, f32(inst.alpha), f32(inst.g)))
    opt = torch.optim.Adam(model.parameters(), lr=2e-2)
    losses = [NET.train_step(model, opt, batch) for _ in range(12)]
    torch.cuda.synchronize()
    assert losses[-1] < losses[0], losses
    r = model.rho.detach().cpu().numpy()
    assert np.all(r >= 0.0) and np.all(r <= 1.0)


def test_layer_backward_batch_matches_oracle_and_single_calls(P):
    """psca_layer_backward_batch over instances of different N, L and variant
    (one step size): each result meets the oracle bar of the single-instance
    backward and agrees with the single call to the same bar."""
    cases = [(O.ML_K, 300, 64, 128), (O.MAP_K, 100, 20, 32), (O.ML_UD, 700, 48, 64), (O.MAP_UR, 60, 16, 64),
             (O.ML_UD, 20, 8, 64), (O.ML_K, 1000, 64, 128)]
    rho = 0.35
    items, refs, singles = [], [], []
    for k, (variant, N, L, M) in enumerate(cases):
        inst = I.make_instance(3, 800 + k, N, L, M, 0.2).fp32_inputs()
        prob = O.problem_from_instance(inst, variant, eps=EPS)
        _, hist = O.psca(prob, 6, record=True)
        x = np.asarray(hist[5].x, np.float32).astype(np.float64)
        v = np.random.default_rng(k).standard_normal(N).astype(np.float32).astype(np.float64)
        refs.append((O.layer_vjp(prob, x, rho, v), x, v))
        Sh = P.sample_cov(c64(inst.Y))
        prm = params_for(P, inst, variant)
        items.append((Sh, c64(inst.S), prm, f32(x), f32(v)))
        singles.append(P.layer_backward(Sh, c64(inst.S), prm, rho, f32(x), f32(v)))
    status = torch.full((len(cases),), 7, dtype=torch.int32, device=dev())
    print("[layer backward batch of 6]", flush=True)
    gxs, gr = P.layer_backward_batch(items, rho, status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * len(cases)
    for k, (variant, N, L, M) in enumerate(cases):
        (dx_ref, drho_ref), x, v = refs[k]
        gx = gxs[k].cpu().numpy().astype(np.float64)
        scale = np.max(np.abs(dx_ref))
        assert np.max(np.abs(gx - dx_ref)) / scale < 2e-3, (k, O.VARIANT_NAMES[variant])
        assert np.max(np.abs(gx - singles[k][0].cpu().numpy())) / scale < 2e-3, k
        tol = 1e-6 * np.sum(np.abs(v)) * np.max(np.abs(x))
        assert float(gr[k].item()) == pytest.approx(drho_ref, rel=2e-3, abs=tol), k
        assert float(gr[k].item()) == pytest.approx(float(singles[k][1].item()), rel=2e-3, abs=tol), k


def test_layer_backward_batch_full_minibatch_sampled(P):
    """One layer's batched backward over a full training minibatch (512 MAP-UR
    instances at N=1000, L=64, M=128), at seeded iterates: every status is 0,
    three sampled instances agree with the single-instance backward, and two
    of them meet the oracle's vector-Jacobian product."""
    B, N, L, M, rho = 512, 1000, 64, 128, 0.3
    wid = I.WORKLOAD_IDS["net"]
    items, xs, vs, insts = [], [], [], []
    rng = np.random.default_rng(2024)
    for k in range(B):
        inst = I.make_instance(wid, k, N, L, M, 0.1).fp32_inputs()
        x = (inst.g * rng.uniform(0.0, 0.3, N)).astype(np.float32).astype(np.float64)
        v = rng.standard_normal(N).astype(np.float32).astype(np.float64)
        items.append((P.sample_cov(c64(inst.Y)), c64(inst.S), params_for(P, inst, O.MAP_UR), f32(x), f32(v)))
        xs.append(x)
        vs.append(v)
        insts.append(inst)
    status = torch.full((B,), 7, dtype=torch.int32, device=dev())
    print(f"[layer backward batch of {B}, MAP-UR N={N} L={L} M={M}]", flush=True)
    gxs, gr = P.layer_backward_batch(items, rho, status=status)
    torch.cuda.synchronize()
    assert int((status != 0).sum().item()) == 0
    for k in (0, 255, 511):
        Sh, S, prm, x_t, v_t = items[k]
        gx1, gr1 = P.layer_backward(Sh, S, prm, rho, x_t, v_t)
        torch.cuda.synchronize()
        gx = gxs[k].cpu().numpy().astype(np.float64)
        scale = np.max(np.abs(gx1.cpu().numpy()))
        assert np.max(np.abs(gx - gx1.cpu().numpy())) / scale < 2e-3, k
        tol = 1e-6 * np.sum(np.abs(vs[k])) * np.max(np.abs(xs[k]))
        assert float(gr[k].item()) == pytest.approx(float(gr1.item()), rel=2e-3, abs=tol), k
    for k in (0, 511):
        dx_ref, drho_ref = O.layer_vjp(O.problem_from_instance(insts[k], O.MAP_UR, eps=EPS), xs[k], rho, vs[k])
        gx = gxs[k].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(gx - dx_ref)) / np.max(np.abs(dx_ref)) < 2e-3, k
        tol = 1e-6 * np.sum(np.abs(vs[k])) * np.max(np.abs(xs[k]))
        assert float(gr[k].item()) == pytest.approx(drho_ref, rel=2e-3, abs=tol), k


def test_layer_backward_batch_validation(P):
    inst = I.make_instance(3, 5, 30, 80, 16, 0.2).fp32_inputs()
    Sh = P.sample_cov(c64(inst.Y))
    item = (Sh, c64(inst.S), params_for(P, inst, O.ML_UD), f32(np.zeros(30)), f32(np.ones(30)))
    inst2 = I.make_instance(3, 6, 30, 16, 16, 0.2).fp32_inputs()
    item2 = (P.sample_cov(c64(inst2.Y)), c64(inst2.S), params_for(P, inst2, O.ML_UD), f32(np.zeros(30)),
             f32(np.ones(30)))
    with pytest.raises(P.PscaError) as e:   # one launch takes L <= 64 (LDS) or L > 64 (memory), not both
        P.layer_backward_batch([item, item2], 0.5)
    assert e.value.code == -5
    with pytest.raises(P.PscaError) as e:
        P.layer_backward_batch([item2], 1.5)
    assert e.value.code == -1   # rho outside [0, 1]


# (N, L, M, p, scale of the iterate).  The L > 64 backward is held to the bar
# of the L <= 64 one where single precision can meet it: shapes with N >> L
# as in the configurations (kappa(Sigma) of a few hundred), and shapes with
# N < L at iterates scaled down to kappa(Sigma) ~ 100.  With N close to or
# below L at full-scale iterates kappa(Sigma) reaches 1e5, and the same
# formulas evaluated in single precision on the host (NumPy complex64)
# already miss the FP64 vector-Jacobian product by 0.3 % to 20 %.
LARGE_CASES = [(2000, 200, 256, 0.05, 1.0), (1200, 100, 64, 0.05, 1.0), (600, 72, 64, 0.1, 1.0),
               (400, 256, 40, 0.05, 1.0), (1000, 130, 128, 0.1, 1.0), (33, 256, 40, 0.2, 1e-3), (40, 72, 64, 0.2, 1e-3)]


def _large_back_case(variant, N, L, M, p, scale):
    inst = I.make_instance(3, 700 + N + L, N, L, M, p).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    _, hist = O.psca(prob, 6, record=True)
    x = (scale * np.asarray(hist[5].x)).astype(np.float32).astype(np.float64)   # the input the kernel sees
    v = np.random.default_rng(N + L + variant).standard_normal(N).astype(np.float32).astype(np.float64)
    return inst, prob, x, v


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("N,L,M,p,scale", LARGE_CASES)
def test_large_pilot_length_layer_backward_matches_oracle_vjp(P, variant, N, L, M, p, scale):
    """Layer backward with L > 64 (Sigma and the two Gram matrices in memory,
    column blocks in registers) against the oracle's vector-Jacobian product
    at the bar of the L <= 64 backward."""
    inst, prob, x, v = _large_back_case(variant, N, L, M, p, scale)
    rho = 0.4
    dx_ref, drho_ref = O.layer_vjp(prob, x, rho, v)
    Sh = P.sample_cov(c64(inst.Y))
    status = torch.full((1,), 7, dtype=torch.int32, device=dev())
    print(f"[large-L layer backward {O.VARIANT_NAMES[variant]} N={N} L={L} M={M}]", flush=True)
    gx, gr = P.layer_backward(Sh, c64(inst.S), params_for(P, inst, variant), rho, f32(x), f32(v), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    gx = gx.cpu().numpy().astype(np.float64)
    err = np.max(np.abs(gx - dx_ref)) / np.max(np.abs(dx_ref))
    print(f"  max |dL/dx error| / max |dL/dx| = {err:.2e}", flush=True)
    assert err < 2e-3, (O.VARIANT_NAMES[variant], N, L, err)
    assert float(gr.item()) == pytest.approx(drho_ref, rel=2e-3, abs=1e-6 * np.sum(np.abs(v)) * np.max(np.abs(x)))


def test_large_pilot_length_layer_backward_batch(P):
    """psca_layer_backward_batch with every L above 64, of different N, L and
    variant: each result agrees with the single call and the oracle."""
    cases = [(O.ML_K, 1200, 100, 64, 0.05, 1.0), (O.MAP_UR, 600, 72, 64, 0.1, 1.0),
             (O.ML_UD, 2000, 200, 256, 0.05, 1.0), (O.MAP_K, 33, 256, 40, 0.2, 1e-3)]
    rho = 0.35
    items, refs, singles = [], [], []
    for variant, N, L, M, p, scale in cases:
        inst, prob, x, v = _large_back_case(variant, N, L, M, p, scale)
        refs.append((O.layer_vjp(prob, x, rho, v), x, v))
        Sh = P.sample_cov(c64(inst.Y))
        prm = params_for(P, inst, variant)
        items.append((Sh, c64(inst.S), prm, f32(x), f32(v)))
        singles.append(P.layer_backward(Sh, c64(inst.S), prm, rho, f32(x), f32(v)))
    status = torch.full((len(cases),), 7, dtype=torch.int32, device=dev())
    print("[large-L layer backward batch of 4]", flush=True)
    gxs, gr = P.layer_backward_batch(items, rho, status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * len(cases)
    for k, (variant, N, L, M, p, scale) in enumerate(cases):
        (dx_ref, drho_ref), x, v = refs[k]
        gx = gxs[k].cpu().numpy().astype(np.float64)
        scale_dx = np.max(np.abs(dx_ref))
        assert np.max(np.abs(gx - dx_ref)) / scale_dx < 2e-3, (k, O.VARIANT_NAMES[variant])
        assert np.max(np.abs(gx - singles[k][0].cpu().numpy())) / scale_dx < 2e-3, k
        tol = 1e-6 * np.sum(np.abs(v)) * np.max(np.abs(x))
        assert float(gr[k].item()) == pytest.approx(drho_ref, rel=2e-3, abs=tol), k


@pytest.mark.parametrize("variant,L,seed", [(O.ML_K, 100, 0), (O.MAP_UR, 16, 0), (O.MAP_UR, 16, 9)])
def test_network_gradient_large_pilot_length_and_map_ur(P, variant, L, seed):
    """Whole-network step-size gradient against the oracle's reverse
    accumulation: ML-K at L = 100 (the backward in memory), and MAP-UR on
    instances whose every iterate stays at least 1e-3 (relative) away from
    the branch points of p^eps and whose gamma~/g stays clear of the BCE
    clamp (there both paths take the same branches)."""
    from paper_2503_15259_amd import net as NET
    inst = I.make_instance(3, 1200 + seed if variant == O.MAP_UR else 1500, 60 if variant == O.MAP_UR else 120, L,
                           64, 0.2).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    K = 5
    rhos = np.asarray(NET.schedule(K), np.float32).astype(np.float64)
    x, recs = np.zeros(prob.N), []
    for r in rhos:
        recs.append(O.psca_iteration(prob, x, float(r)))
        x = recs[-1].x_next
    if variant == O.MAP_UR:
        assert O.branch_margin(prob, recs).min() >= 1e-3
    loss_ref, g_ref = O.net_loss_and_grad(prob, rhos, inst.alpha, inst.g)
    model = NET.PscaNet(K, params_for(P, inst, variant))
    xg = model(P.sample_cov(c64(inst.Y)), c64(inst.S))
    loss = NET.bce(xg, f32(inst.alpha), f32(inst.g), model.known)
    loss.backward()
    torch.cuda.synchronize()
    model.status.check()
    assert loss.item() == pytest.approx(loss_ref, rel=1e-3)
    got = model.rho.grad.cpu().numpy().astype(np.float64)
    print(f"network gradient {O.VARIANT_NAMES[variant]} L={L}: max rel err "
          f"{np.max(np.abs(got - g_ref)) / np.max(np.abs(g_ref)):.2e}", flush=True)
    np.testing.assert_allclose(got, g_ref, rtol=5e-3, atol=5e-3 * np.max(np.abs(g_ref)))


@pytest.mark.parametrize("variant", [O.ML_K, O.ML_UD])
def test_batched_network_gradient_matches_oracle(P, variant):
    """Forward (one batch launch with recorded iterates) and backward (one
    batched launch per layer) of a minibatch: the mean loss and its step-size
    gradient against the oracle's reverse accumulation, instance by instance."""
    from paper_2503_15259_amd import net as NET
    K = 5
    insts = [I.make_instance(3, 950 + 10 * variant + k, n, 16, 64, 0.2).fp32_inputs()
             for k, n in enumerate((60, 90, 40))]
    rhos = np.asarray(NET.schedule(K), np.float32).astype(np.float64)
    refs = [O.net_loss_and_grad(O.problem_from_instance(inst, variant, eps=EPS), rhos, inst.alpha, inst.g)
            for inst in insts]
    loss_ref = np.mean([r[0] for r in refs])
    g_ref = np.mean([r[1] for r in refs], axis=0)
    model = NET.PscaNet(K, params_for(P, insts[0], variant))
    batch = [(P.sample_cov(c64(inst.Y)), c64(inst.S), params_for(P, inst, variant), f32(inst.alpha), f32(inst.g))
             for inst in insts]
    print(f"[batched network gradient {O.VARIANT_NAMES[variant]}]", flush=True)
    xs = model.forward_batch([(Sh, S, prm) for Sh, S, prm, _, _ in batch])
    loss = sum(NET.bce(x, a, g, model.known) for x, (_, _, _, a, g) in zip(xs, batch)) / len(batch)
    loss.backward()
    torch.cuda.synchronize()
    assert loss.item() == pytest.approx(loss_ref, rel=1e-3)
    got = model.rho.grad.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, g_ref, rtol=5e-3, atol=5e-3 * np.max(np.abs(g_ref)))
    # the training step's form: one weighted sum over the concatenated devices
    model.rho.grad = None
    loss2 = NET.batch_loss(model, batch)
    loss2.backward()
    torch.cuda.synchronize()
    assert loss2.item() == pytest.approx(loss_ref, rel=1e-3)
    assert loss2.item() == pytest.approx(loss.item(), rel=1e-12)
    got2 = model.rho.grad.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got2, g_ref, rtol=5e-3, atol=5e-3 * np.max(np.abs(g_ref)))
    np.testing.assert_allclose(got2, got, rtol=1e-5, atol=1e-6 * np.max(np.abs(got)))


@pytest.mark.parametrize("variant,tol", [(O.ML_K, 1e-2), (O.ML_UD, 1e-2), (O.ML_K, 1e9)])
def test_network_with_plain_psca_as_judge_and_fallback(P, variant, tol):
    """detect_with_fallback: the network's output is judged by its
    stationarity residual from one PSCA iteration (against the oracle's);
    above tol, plain PSCA continues from it with the schedule and the result
    equals the oracle's network followed by the same PSCA iterations, with
    a smaller residual; at a tolerance it meets, the output is the
    network's own."""
    from paper_2503_15259_amd import net as NET
    inst = I.make_instance(3, 2100 + variant, 300, 32, 64, 0.1).fp32_inputs()
    prob = O.problem_from_instance(inst, variant, eps=EPS)
    K, extra = 3, 40
    model = NET.PscaNet(K, params_for(P, inst, variant))   # the schedule: far from stationary after 3 layers
    rhos = model.rho.detach().numpy().astype(np.float64)
    xk = O.net_forward(prob, rhos)[-1]
    rec = O.psca_iteration(prob, xk, 1.0)
    res_ref = np.max(np.abs(rec.x_tilde - xk)) / max(np.max(np.abs(xk)), 1e-30)
    x, rep = NET.detect_with_fallback(model, P.sample_cov(c64(inst.Y)), c64(inst.S), tol=tol, extra_iters=extra)
    torch.cuda.synchronize()
    print(f"[fallback {O.VARIANT_NAMES[variant]} tol={tol:g}] {rep}; oracle residual {res_ref:.4g}", flush=True)
    assert rep["residual_net"] == pytest.approx(res_ref, rel=1e-3)
    if tol < res_ref:
        assert rep["fallback"]
        x_ref = xk.copy()
        for rho in O.step_sizes(extra):
            x_ref = O.psca_iteration(prob, x_ref, float(rho)).x_next
        assert_parity(x.cpu().numpy(), x_ref, variant, "network + fallback")
        assert rep["residual_after"] < rep["residual_net"]
    else:
        assert not rep["fallback"]
        assert_parity(x.cpu().numpy(), xk, variant, "network alone")
