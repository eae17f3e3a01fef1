"""Python binding of the PSCA C ABI (argument marshalling only).

Every computation runs in the HIP kernels of libpsca.so; torch provides the
device memory and the stream.  Complex matrices are torch.complex64 tensors
with the mathematical shape (L x N for S, L x M for Y, L x L for SigmaHat);
the ABI wants them column-major, i.e. with strides (1, L).  `colmajor()`
produces that layout (a no-op for a tensor that already has it).
"""
from __future__ import annotations

import atexit
import ctypes
import sys
from dataclasses import dataclass
from typing import Optional

import torch

from . import _native as N
from ._native import ML_K, MAP_K, ML_UD, MAP_UR, MAP_K2, MAX_L, DIST_AREA, DIST_LINEAR, PscaError  # noqa: F401

VARIANTS = {"ML-K": ML_K, "MAP-K": MAP_K, "ML-UD": ML_UD, "MAP-UR": MAP_UR, "MAP-K2": MAP_K2}


def colmajor(t: torch.Tensor) -> torch.Tensor:
    """Same matrix, column-major storage (strides (1, rows))."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    if t.stride(0) == 1 and t.stride(1) == t.shape[0]:
        return t
    return t.mT.contiguous().mT


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device, stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream(device) if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(device: torch.device, stream, temporaries) -> None:
    """Before a launch on a caller-given `stream`: order it after the work
    torch queued on the current stream (the column-major copies the call may
    have made there), and tell the caching allocator that those copies are
    in use on `stream` until its work is done."""
    if stream is None:
        return
    cur = torch.cuda.current_stream(device)
    if stream != cur:
        stream.wait_stream(cur)
    for t in temporaries:
        t.record_stream(stream)


def _need(t: torch.Tensor, dtype, device, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device:
        raise TypeError(f"{name} must be a {dtype} tensor on {device}")


class Context:
    """Owns a psca_ctx (work buffers) on one GPU."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self._lib = N.load()
        h = ctypes.c_void_p()
        N.check(self._lib.psca_create(ctypes.byref(h), self.device.index), "psca_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.psca_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down: the runtime (or a
        # profiler attached to it) may already be finalising
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


@atexit.register
def _close_default_contexts():
    """Free the default contexts while the HIP runtime is still up."""
    for c in list(_default_ctx.values()):
        try:
            c.close()
        except Exception:
            pass
    _default_ctx.clear()


def default_context(device=None) -> Context:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = dev.index or 0
    if key not in _default_ctx:
        _default_ctx[key] = Context(key)
    return _default_ctx[key]


@dataclass
class Params:
    """psca_params (include/psca.h).  Tensors must live on the context's GPU."""
    variant: int
    iters: int = 100
    sigma2: float = 1.0
    M: int = 1
    g: Optional[torch.Tensor] = None
    p: Optional[torch.Tensor] = None
    rho0: float = 0.5
    rho_decay: float = 0.5
    rho: Optional[torch.Tensor] = None
    d_lo: float = 0.05
    d_hi: float = 0.5
    pl_c0: float = 10.0 ** 0.89
    pl_beta: float = 3.76
    eps: float = 0.01
    dist_law: int = 0   # MAP-UR distance law: 0 area-uniform (eq. dispdf), 1 uniform in d
    # MAP-K2: first-order coefficients [N] and the pairwise coefficients as
    # CSR (row pointers [N+1] int32, columns [nnz] int32, values [nnz] float32)
    c1: Optional[torch.Tensor] = None
    c2_ptr: Optional[torch.Tensor] = None
    c2_col: Optional[torch.Tensor] = None
    c2_val: Optional[torch.Tensor] = None
    x0: Optional[torch.Tensor] = None   # starting iterate [N] (None: zeros)

    def to_c(self) -> N.PscaParams:
        c = N.PscaParams()
        c.variant = int(self.variant)
        c.iters = int(self.iters)
        c.rho0 = float(self.rho0)
        c.rho_decay = float(self.rho_decay)
        c.rho = None if self.rho is None else self.rho.data_ptr()
        c.sigma2 = float(self.sigma2)
        c.M = int(self.M)
        c.g = None if self.g is None else self.g.data_ptr()
        c.p = None if self.p is None else self.p.data_ptr()
        c.d_lo, c.d_hi = float(self.d_lo), float(self.d_hi)
        c.pl_c0, c.pl_beta, c.eps = float(self.pl_c0), float(self.pl_beta), float(self.eps)
        c.c1 = None if self.c1 is None else self.c1.data_ptr()
        c.c2_ptr = None if self.c2_ptr is None else self.c2_ptr.data_ptr()
        c.c2_col = None if self.c2_col is None else self.c2_col.data_ptr()
        c.c2_val = None if self.c2_val is None else self.c2_val.data_ptr()
        c.c2_nnz = 0 if self.c2_col is None else int(self.c2_col.numel())
        c.dist_law = int(self.dist_law)
        c.x0 = None if self.x0 is None else self.x0.data_ptr()
        return c

    def check_tensors(self, device, n):
        for name in ("g", "p", "x0"):
            t = getattr(self, name)
            if t is not None:
                _need(t, torch.float32, device, name)
                if t.numel() != n or not t.is_contiguous():
                    raise ValueError(f"{name} must be a contiguous float32 vector of length N")
        if self.c1 is not None:
            _need(self.c1, torch.float32, device, "c1")
            if self.c1.numel() != n or not self.c1.is_contiguous():
                raise ValueError("c1 must be a contiguous float32 vector of length N")
        if self.c2_ptr is not None:
            _need(self.c2_ptr, torch.int32, device, "c2_ptr")
            if self.c2_ptr.numel() != n + 1 or not self.c2_ptr.is_contiguous():
                raise ValueError("c2_ptr must be a contiguous int32 vector of length N + 1")
            for name, dt in (("c2_col", torch.int32), ("c2_val", torch.float32)):
                t = getattr(self, name)
                if t is None:
                    raise ValueError(f"{name} is required with c2_ptr")
                _need(t, dt, device, name)
                if not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous")
            if self.c2_col.numel() != self.c2_val.numel():
                raise ValueError("c2_col and c2_val must have the same length")
        if self.rho is not None:
            _need(self.rho, torch.float32, device, "rho")
            if self.rho.numel() < self.iters or not self.rho.is_contiguous():
                raise ValueError("rho must hold `iters` contiguous float32 step sizes")


def sample_cov(Y: torch.Tensor, ctx: Optional[Context] = None, stream=None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """SigmaHat = Y Y^H / M on the GPU (psca_sample_cov).  `out`, if given,
    is a column-major complex64 L x L tensor that receives it."""
    ctx = ctx or default_context(Y.device)
    _need(Y, torch.complex64, ctx.device, "Y")
    Y = colmajor(Y)
    L, M = Y.shape
    if out is None:
        out = torch.empty((L, L), dtype=torch.complex64, device=ctx.device).mT
    else:
        _need(out, torch.complex64, ctx.device, "out")
        if out.shape != (L, L) or out.stride() != (1, L):
            raise ValueError("out must be a column-major L x L complex64 tensor")
    N.check(ctx._lib.psca_sample_cov(ctx.handle, _ptr(Y), L, M, _ptr(out), _stream(ctx.device, stream)),
            "psca_sample_cov")
    return out


def sample_cov_batch(Y: torch.Tensor, ctx: Optional[Context] = None, stream=None,
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """SigmaHat of B instances of one size in one launch (psca_sample_cov_batch).
    Y: complex64 B x L x M whose instances are column-major (Y[b].stride() ==
    (1, L)), such as torch.empty(B, M, L).transpose(1, 2).  Returns (or fills
    `out`, of the same kind) B x L x L with column-major instances."""
    ctx = ctx or default_context(Y.device)
    _need(Y, torch.complex64, ctx.device, "Y")
    if Y.dim() != 3:
        raise ValueError("Y must be B x L x M")
    B, L, M = Y.shape
    if Y.stride(1) != 1 or Y.stride(2) != L:
        raise ValueError("every instance of Y must be column-major (strides (1, L))")
    if out is None:
        out = torch.empty((B, L, L), dtype=torch.complex64, device=ctx.device).transpose(1, 2)
    else:
        _need(out, torch.complex64, ctx.device, "out")
        if out.shape != (B, L, L) or out.stride(1) != 1 or out.stride(2) != L:
            raise ValueError("out must be B x L x L with column-major instances")
    N.check(ctx._lib.psca_sample_cov_batch(ctx.handle, B, _ptr(Y), Y.stride(0) if B > 1 else L * M, L, M,
                                           _ptr(out), out.stride(0) if B > 1 else L * L,
                                           _stream(ctx.device, stream)), "psca_sample_cov_batch")
    return out


def detect(Sigma_hat: torch.Tensor, S: torch.Tensor, params: Params, ctx: Optional[Context] = None,
           stream=None, out: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None):
    """Algorithm 1 from x = params.x0 (zeros when None) for params.iters
    iterations (psca_detect).  Returns x (float32, length N).  `status`, if given, is a device int32[1]
    that receives 0 or PSCA_ENOTPD."""
    ctx = ctx or default_context(S.device)
    _need(S, torch.complex64, ctx.device, "S")
    _need(Sigma_hat, torch.complex64, ctx.device, "Sigma_hat")
    S = colmajor(S)
    Sigma_hat = colmajor(Sigma_hat)
    L, n = S.shape
    if Sigma_hat.shape != (L, L):
        raise ValueError("Sigma_hat must be L x L")
    params.check_tensors(ctx.device, n)
    x = torch.empty(n, dtype=torch.float32, device=ctx.device) if out is None else out
    c = params.to_c()
    _on_stream(ctx.device, stream, (Sigma_hat, S))
    N.check(ctx._lib.psca_detect(ctx.handle, _ptr(Sigma_hat), _ptr(S), L, n, ctypes.byref(c), _ptr(x),
                                 _ptr(status), _stream(ctx.device, stream)), "psca_detect")
    return x


def detect_noalloc(Sigma_hat: torch.Tensor, S: torch.Tensor, params: Params, out: torch.Tensor,
                   ctx: Optional[Context] = None, stream=None, status: Optional[torch.Tensor] = None):
    """psca_detect_noalloc: psca_detect with the library's fixed per-GPU
    scratch array (no device allocation in the call; L <= 96).  Sigma_hat
    and S must already be column-major and `out` given: this wrapper makes
    no copies.  Calls on one GPU must not overlap in time."""
    ctx = ctx or default_context(S.device)
    _need(S, torch.complex64, ctx.device, "S")
    _need(Sigma_hat, torch.complex64, ctx.device, "Sigma_hat")
    _need(out, torch.float32, ctx.device, "out")
    L, n = S.shape
    if S.stride() != (1, L) or Sigma_hat.shape != (L, L) or Sigma_hat.stride() != (1, L):
        raise ValueError("S and Sigma_hat must be column-major (see colmajor)")
    if out.numel() != n or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 vector of length N")
    params.check_tensors(ctx.device, n)
    c = params.to_c()
    _on_stream(ctx.device, stream, ())
    N.check(ctx._lib.psca_detect_noalloc(ctx.handle, _ptr(Sigma_hat), _ptr(S), L, n, ctypes.byref(c), _ptr(out),
                                         _ptr(status), _stream(ctx.device, stream)), "psca_detect_noalloc")
    return out


def detect_y(Y: torch.Tensor, S: torch.Tensor, params: Params, ctx: Optional[Context] = None,
             stream=None, out: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None):
    """psca_detect_y: SigmaHat from Y (M = Y.shape[1]) then Algorithm 1."""
    ctx = ctx or default_context(S.device)
    _need(S, torch.complex64, ctx.device, "S")
    _need(Y, torch.complex64, ctx.device, "Y")
    S = colmajor(S)
    Y = colmajor(Y)
    L, n = S.shape
    if Y.shape[0] != L or Y.shape[1] != params.M:
        raise ValueError("Y must be L x M with M = params.M")
    params.check_tensors(ctx.device, n)
    x = torch.empty(n, dtype=torch.float32, device=ctx.device) if out is None else out
    c = params.to_c()
    _on_stream(ctx.device, stream, (Y, S))
    N.check(ctx._lib.psca_detect_y(ctx.handle, _ptr(Y), _ptr(S), L, n, ctypes.byref(c), _ptr(x),
                                   _ptr(status), _stream(ctx.device, stream)), "psca_detect_y")
    return x


@dataclass
class Problem:
    """One instance of a batch (psca_problem): SigmaHat, S, parameters and the
    output vector (allocated by detect_batch when None)."""
    Sigma_hat: torch.Tensor
    S: torch.Tensor
    params: Params
    out: Optional[torch.Tensor] = None
    status: Optional[torch.Tensor] = None
    hist: Optional[torch.Tensor] = None   # optional [(iters + 1), N]: every iterate


def _problem_array(problems, ctx):
    """psca_problem[] for `problems`; allocates missing outputs.  Returns the
    array, the output tensors and the tensors that must stay alive."""
    arr = (N.PscaProblem * len(problems))()
    keep, outs = [], []
    for k, pb in enumerate(problems):
        _need(pb.S, torch.complex64, ctx.device, "S")
        _need(pb.Sigma_hat, torch.complex64, ctx.device, "Sigma_hat")
        S = colmajor(pb.S)
        Sh = colmajor(pb.Sigma_hat)
        L, n = S.shape
        if Sh.shape != (L, L):
            raise ValueError("Sigma_hat must be L x L")
        pb.params.check_tensors(ctx.device, n)
        if pb.out is None:
            pb.out = torch.empty(n, dtype=torch.float32, device=ctx.device)
        x = pb.out
        if x.numel() != n or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("out must be a contiguous float32 vector of length N")
        keep += [S, Sh]
        outs.append(x)
        e = arr[k]
        e.Sigma_hat = Sh.data_ptr()
        e.S = S.data_ptr()
        e.L, e.N = L, n
        e.prm = pb.params.to_c()
        e.x_out = x.data_ptr()
        e.status = None if pb.status is None else pb.status.data_ptr()
        if pb.hist is not None:
            _need(pb.hist, torch.float32, ctx.device, "hist")
            if pb.hist.numel() < (pb.params.iters + 1) * n or not pb.hist.is_contiguous():
                raise ValueError("hist must be a contiguous float32 tensor of (iters + 1) x N")
        e.x_hist = None if pb.hist is None else pb.hist.data_ptr()
    return arr, outs, keep


def detect_batch(problems, ctx: Optional[Context] = None, stream=None):
    """psca_detect_batch: independent detections in one persistent launch.
    Returns the list of x vectors (each problem's `out`)."""
    if not problems:
        return []
    ctx = ctx or default_context(problems[0].S.device)
    arr, outs, keep = _problem_array(problems, ctx)
    _on_stream(ctx.device, stream, keep)
    N.check(ctx._lib.psca_detect_batch(ctx.handle, len(problems), arr, _stream(ctx.device, stream)),
            "psca_detect_batch")
    return outs


def autotune_batch(problems, tune_iters: int = 4, ctx: Optional[Context] = None, stream=None) -> int:
    """psca_autotune_batch: times the candidate team sizes for this batch and
    remembers the fastest in the context.  Returns the chosen team size."""
    ctx = ctx or default_context(problems[0].S.device)
    arr, _outs, keep = _problem_array(problems, ctx)
    _on_stream(ctx.device, stream, keep)
    t = ctypes.c_int(0)
    N.check(ctx._lib.psca_autotune_batch(ctx.handle, len(problems), arr, int(tune_iters), ctypes.byref(t),
                                         _stream(ctx.device, stream)), "psca_autotune_batch")
    return t.value


class Plan:
    """psca_plan: a batch planned once and launched many times (launches may be
    captured into a CUDA/HIP graph).  Keep the problems' tensors alive.
    team_size: > 0 uniform teams of that many workgroups; < 0 mixed teams,
    each instance's team sized for tiles of -team_size columns (a multiple
    of 16 up to 128); 0 the autotuned choice, else the default."""

    def __init__(self, problems, team_size: int = 0, ctx: Optional[Context] = None):
        self.ctx = ctx or default_context(problems[0].S.device)
        self.problems = problems
        arr, self.outs, self._keep = _problem_array(problems, self.ctx)
        h = ctypes.c_void_p()
        N.check(self.ctx._lib.psca_plan_create(self.ctx.handle, len(problems), arr, int(team_size),
                                               ctypes.byref(h)), "psca_plan_create")
        self.handle = h

    @property
    def team_size(self) -> int:
        return self.ctx._lib.psca_plan_team_size(self.handle)

    def launch(self, stream=None):
        N.check(self.ctx._lib.psca_plan_launch(self.handle, _stream(self.ctx.device, stream)), "psca_plan_launch")
        return self.outs

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.ctx._lib.psca_plan_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def iterate(Sigma_hat: torch.Tensor, S: torch.Tensor, x: torch.Tensor, rho: float, params: Params,
            ctx: Optional[Context] = None, stream=None, status: Optional[torch.Tensor] = None):
    """One iteration (psca_iterate).  Returns (x_next, q, r, x_tilde)."""
    ctx = ctx or default_context(S.device)
    _need(S, torch.complex64, ctx.device, "S")
    _need(Sigma_hat, torch.complex64, ctx.device, "Sigma_hat")
    _need(x, torch.float32, ctx.device, "x")
    S = colmajor(S)
    Sigma_hat = colmajor(Sigma_hat)
    L, n = S.shape
    if x.numel() != n or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 vector of length N")
    params.check_tensors(ctx.device, n)
    x_next, q, r, xt = (torch.empty(n, dtype=torch.float32, device=ctx.device) for _ in range(4))
    c = params.to_c()
    _on_stream(ctx.device, stream, (Sigma_hat, S))
    N.check(ctx._lib.psca_iterate(ctx.handle, _ptr(Sigma_hat), _ptr(S), L, n, ctypes.byref(c),
                                  ctypes.c_float(rho), _ptr(x), _ptr(x_next), _ptr(q), _ptr(r), _ptr(xt),
                                  _ptr(status), _stream(ctx.device, stream)), "psca_iterate")
    return x_next, q, r, xt


def net_forward(Sigma_hat: torch.Tensor, S: torch.Tensor, params: Params, ctx: Optional[Context] = None,
                stream=None, status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """psca_net_forward: params.iters layers (step sizes params.rho, or the
    schedule), every iterate recorded.  Returns x_hist [(iters + 1), N]."""
    ctx = ctx or default_context(S.device)
    _need(S, torch.complex64, ctx.device, "S")
    _need(Sigma_hat, torch.complex64, ctx.device, "Sigma_hat")
    S = colmajor(S)
    Sigma_hat = colmajor(Sigma_hat)
    L, n = S.shape
    params.check_tensors(ctx.device, n)
    hist = torch.empty((params.iters + 1, n), dtype=torch.float32, device=ctx.device)
    c = params.to_c()
    _on_stream(ctx.device, stream, (Sigma_hat, S))
    N.check(ctx._lib.psca_net_forward(ctx.handle, _ptr(Sigma_hat), _ptr(S), L, n, ctypes.byref(c), _ptr(hist),
                                      _ptr(status), _stream(ctx.device, stream)), "psca_net_forward")
    return hist


def layer_backward(Sigma_hat: torch.Tensor, S: torch.Tensor, params: Params, rho: float, x_in: torch.Tensor,
                   v: torch.Tensor, ctx: Optional[Context] = None, stream=None,
                   status: Optional[torch.Tensor] = None):
    """psca_layer_backward: (dL/dx, dL/drho) of one layer from v = dL/dx'.
    dL/drho is returned as a one-element device tensor."""
    ctx = ctx or default_context(S.device)
    _need(S, torch.complex64, ctx.device, "S")
    _need(Sigma_hat, torch.complex64, ctx.device, "Sigma_hat")
    _need(x_in, torch.float32, ctx.device, "x_in")
    _need(v, torch.float32, ctx.device, "v")
    S = colmajor(S)
    Sigma_hat = colmajor(Sigma_hat)
    L, n = S.shape
    if x_in.numel() != n or v.numel() != n or not x_in.is_contiguous() or not v.is_contiguous():
        raise ValueError("x_in and v must be contiguous float32 vectors of length N")
    params.check_tensors(ctx.device, n)
    gx = torch.empty(n, dtype=torch.float32, device=ctx.device)
    gr = torch.empty(1, dtype=torch.float32, device=ctx.device)
    c = params.to_c()
    _on_stream(ctx.device, stream, (Sigma_hat, S))
    N.check(ctx._lib.psca_layer_backward(ctx.handle, _ptr(Sigma_hat), _ptr(S), L, n, ctypes.byref(c),
                                         ctypes.c_float(rho), _ptr(x_in), _ptr(v), _ptr(gx), _ptr(gr),
                                         _ptr(status), _stream(ctx.device, stream)), "psca_layer_backward")
    return gx, gr


class BackBatch:
    """A minibatch for psca_layer_backward_batch: the instances (Sigma_hat, S,
    params) are validated and marshalled once; run() supplies each layer's
    inputs x_in and upstream gradients v."""

    def __init__(self, items, ctx: Optional[Context] = None, status=None):
        if not items:
            raise ValueError("empty minibatch")
        self.ctx = ctx or default_context(items[0][1].device)
        self.B = len(items)
        self.arr = (N.PscaBackProblem * self.B)()
        self.keep, self.n = [], []
        self.gr = torch.empty(self.B, dtype=torch.float32, device=self.ctx.device)
        for k, (Sh, S, params) in enumerate(items):
            _need(S, torch.complex64, self.ctx.device, "S")
            _need(Sh, torch.complex64, self.ctx.device, "Sigma_hat")
            S = colmajor(S)
            Sh = colmajor(Sh)
            L, n = S.shape
            if Sh.shape != (L, L):
                raise ValueError("Sigma_hat must be L x L")
            params.check_tensors(self.ctx.device, n)
            self.keep += [S, Sh]
            self.n.append(n)
            e = self.arr[k]
            e.Sigma_hat, e.S, e.L, e.N = Sh.data_ptr(), S.data_ptr(), L, n
            e.prm = params.to_c()
            e.grad_rho = self.gr.data_ptr() + 4 * k
            e.status = None if status is None else status[k].data_ptr()

    def set_status(self, status):
        """Point every instance's status word at status[k] (a device int32
        tensor of B words), or at nothing when status is None."""
        if status is not None and (status.dtype != torch.int32 or status.numel() < self.B):
            raise ValueError("status must hold B int32 words")
        for k in range(self.B):
            self.arr[k].status = None if status is None else status[k].data_ptr()
        self.status_words = status

    def run(self, x_ins, vs, rho: float, stream=None):
        """Returns ([dL/dx per instance], dL/drho per instance as a tensor [B])."""
        gxs, hold = [], []
        for k, (x_in, v) in enumerate(zip(x_ins, vs)):
            n = self.n[k]
            _need(x_in, torch.float32, self.ctx.device, "x_in")
            _need(v, torch.float32, self.ctx.device, "v")
            if x_in.numel() != n or v.numel() != n or not x_in.is_contiguous() or not v.is_contiguous():
                raise ValueError("x_in and v must be contiguous float32 vectors of length N")
            gx = torch.empty(n, dtype=torch.float32, device=self.ctx.device)
            gxs.append(gx)
            hold += [x_in, v]
            e = self.arr[k]
            e.x_in, e.v, e.grad_x = x_in.data_ptr(), v.data_ptr(), gx.data_ptr()
        _on_stream(self.ctx.device, stream, self.keep)
        N.check(self.ctx._lib.psca_layer_backward_batch(self.ctx.handle, self.B, self.arr, ctypes.c_float(rho),
                                                        _stream(self.ctx.device, stream)),
                "psca_layer_backward_batch")
        return gxs, self.gr.clone()


def layer_backward_batch(items, rho: float, ctx: Optional[Context] = None, stream=None, status=None):
    """psca_layer_backward_batch: one layer's backward over a minibatch in one
    persistent launch.  items: list of (Sigma_hat, S, params, x_in, v).
    Returns ([dL/dx per item], dL/drho per item as a device tensor [B])."""
    if not items:
        return [], None
    bb = BackBatch([(Sh, S, prm) for Sh, S, prm, _, _ in items], ctx=ctx, status=status)
    return bb.run([it[3] for it in items], [it[4] for it in items], rho, stream=stream)


def threshold(x: torch.Tensor, theta: float, stream=None) -> torch.Tensor:
    """support = 1[x >= theta] (psca_threshold)."""
    lib = N.load()
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous float32 CUDA tensor")
    out = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
    N.check(lib.psca_threshold(_ptr(x), x.numel(), ctypes.c_float(theta), _ptr(out), _stream(x.device, stream)),
            "psca_threshold")
    return out
