"""psca_detect_noalloc (the entry point that allocates nothing, for callers
under graph capture or in loops that forbid allocation) against psca_detect
through the C ABI (needs an MI355X): two calls in a row on one GPU, the
second smaller, each bit-identical to psca_detect on the same inputs and
within the oracle bar; sizes beyond the fixed scratch are refused before
any launch."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2503_15259_amd import instances as I
from parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = float(np.float32(0.01))


def _case(P, dev, workload_or_shape, index, variant, iters):
    if isinstance(workload_or_shape, str):
        inst = I.workload_instance(workload_or_shape, index).fp32_inputs()
    else:
        N, L, M = workload_or_shape
        inst = I.make_instance(5, 900 + index, N, L, M, 0.1).fp32_inputs()
    S = P.colmajor(torch.from_numpy(inst.S.astype(np.complex64)).to(dev))
    Y = P.colmajor(torch.from_numpy(inst.Y.astype(np.complex64)).to(dev))
    kw = dict(variant=variant, iters=iters, sigma2=inst.sigma2, M=inst.M, d_lo=inst.d_lo, d_hi=inst.d_hi,
              pl_c0=inst.pl_c0, pl_beta=inst.pl_beta, eps=EPS)
    if variant in O.KNOWN_PATHLOSS:
        kw["g"] = torch.from_numpy(inst.g.astype(np.float32)).to(dev)
    return inst, P.sample_cov(Y), S, P.Params(**kw)


def test_no_alloc_detect_matches_detect_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15259_amd import psca as P
    dev = torch.device("cuda", 0)
    ctx = P.Context(0)
    cases = [("single", 0, O.MAP_UR, 60), ((300, 48, 64), 1, O.ML_K, 40)]   # the second call is smaller
    for what, index, variant, iters in cases:
        inst, Sh, S, prm = _case(P, dev, what, index, variant, iters)
        ref_gpu = P.detect(Sh, S, prm, ctx=ctx)
        out = torch.full((inst.N,), float("nan"), dtype=torch.float32, device=dev)
        status = torch.full((1,), 7, dtype=torch.int32, device=dev)
        print(f"[no-alloc detect: {O.VARIANT_NAMES[variant]} N={inst.N} L={inst.L} iters={iters}]", flush=True)
        P.detect_noalloc(Sh, S, prm, out, ctx=ctx, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert torch.equal(out, ref_gpu), "not bit-identical to psca_detect"
        ref = O.psca(O.problem_from_instance(inst, variant, eps=EPS), iters)
        if variant == O.MAP_UR:   # devices near a branch point of the prior are not held to the bar
            prob = O.problem_from_instance(inst, variant, eps=EPS)
            _, hist = O.psca(prob, iters, record=True)
            keep = O.branch_margin(prob, hist) >= 1e-4
            assert_parity(out.cpu().numpy()[keep], ref[keep], variant, "no-alloc")
        else:
            assert_parity(out.cpu().numpy(), ref, variant, "no-alloc")
    # beyond the fixed scratch's reach: refused before any launch
    inst, Sh, S, prm = _case(P, dev, (64, 120, 16), 2, O.ML_UD, 5)
    out = torch.empty(inst.N, dtype=torch.float32, device=dev)
    with pytest.raises(P.PscaError) as e:
        P.detect_noalloc(Sh, S, prm, out, ctx=ctx)
    assert e.value.code == -5
    ctx.close()
