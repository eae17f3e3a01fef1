"""The unrolled PSCA network (PSCA-Net): K layers, layer k one iteration of
Algorithm 1 with its own learned step size rho_k in [0, 1]; trained end to
end on the binary cross-entropy of the last iterate against the true
activity (eq. Loss_alpha on alpha~ for known pathloss, eq. Loss_gamma on
gamma~ / g for unknown pathloss), with Adam; the detection threshold is
chosen afterwards on validation data.

Forward and backward run in the HIP kernels: psca_net_forward records every
iterate; the backward pass calls psca_layer_backward from the last layer to
the first, recomputing Sigma^-1 from each layer's input instead of storing
it.  torch only carries the step-size parameters, the optimiser and the
scalar loss.
"""
from __future__ import annotations

import math
from dataclasses import replace
from typing import Optional

import numpy as np
import torch

from . import psca as P


def schedule(K: int, rho0: float = 0.5, decay: float = 0.5) -> list:
    """rho_0 = rho0, rho_{k+1} = rho_k (1 - decay rho_k): the initial step sizes."""
    out, rho = [], rho0
    for _ in range(K):
        out.append(rho)
        rho = rho * (1.0 - decay * rho)
    return out


class StatusLog:
    """Device status words of the launches behind one training step (forward
    and backward).  Every launch writes its own words; check() reads them
    all back at once and raises on any non-zero code (PSCA_ENOTPD: a
    factorisation failed and that instance's iterates stopped advancing;
    PSCA_ESYNC: a device-wide wait gave up), so no optimiser step is taken
    on results the device has flagged."""

    def __init__(self):
        self.words = []

    def new(self, n: int, device) -> torch.Tensor:
        w = torch.zeros(n, dtype=torch.int32, device=device)
        self.words.append(w)
        return w

    def check(self):
        if not self.words:
            return
        bad = torch.cat(self.words)
        self.words = []
        codes = sorted({int(c) for c in bad[bad != 0].tolist()})
        if codes:
            raise P.PscaError(codes[0], "unrolled network: device status " + ", ".join(map(str, codes)))


class _Unrolled(torch.autograd.Function):
    """x^(K) of the unrolled network as a function of the step sizes."""

    @staticmethod
    def forward(fctx, rhos, Sigma_hat, S, params, pctx, log):
        rho_dev = rhos.detach().to(S.device, torch.float32).contiguous()
        prm = replace(params, iters=rhos.numel(), rho=rho_dev)
        hist = P.net_forward(Sigma_hat, S, prm, ctx=pctx, status=log.new(1, S.device))
        fctx.save_for_backward(rho_dev.clone(), hist)
        fctx.rho_device = rhos.device
        fctx.inputs = (Sigma_hat, S, params, pctx, log)
        return hist[-1].clone()

    @staticmethod
    def backward(fctx, grad_out):
        rhos, hist = fctx.saved_tensors
        Sigma_hat, S, params, pctx, log = fctx.inputs
        host_rhos = rhos.cpu().tolist()
        v = grad_out.contiguous().float()
        grads = []
        status = log.new(len(host_rhos), S.device)   # one word per layer launch
        for k in range(len(host_rhos) - 1, -1, -1):
            v, g = P.layer_backward(Sigma_hat, S, params, float(host_rhos[k]), hist[k].contiguous(), v, ctx=pctx,
                                    status=status[k:k + 1])
            grads.append(g)
        d_rho = torch.cat(grads[::-1]).to(fctx.rho_device)
        return d_rho, None, None, None, None, None


class _UnrolledBatch(torch.autograd.Function):
    """x^(K) of every instance of a minibatch, concatenated, as a function of
    the shared step sizes: the forward is one persistent batch launch with
    every iterate recorded (psca_detect_batch), the backward one batched
    launch per layer (psca_layer_backward_batch)."""

    @staticmethod
    def forward(fctx, rhos, items, pctx, log):
        K = rhos.numel()
        dev = items[0][1].device
        rho_dev = rhos.detach().to(dev, torch.float32).contiguous()
        status = log.new(len(items), dev)
        probs = []
        for b, (Sh, S, params) in enumerate(items):
            hist = torch.empty((K + 1, S.shape[1]), dtype=torch.float32, device=dev)
            probs.append(P.Problem(Sigma_hat=Sh, S=S, params=replace(params, iters=K, rho=rho_dev), hist=hist,
                                   status=status[b:b + 1]))
        P.detect_batch(probs, ctx=pctx)
        fctx.log = log
        fctx.hists = [pb.hist for pb in probs]
        fctx.sizes = [pb.hist.shape[1] for pb in probs]
        fctx.host_rhos = rhos.detach().float().cpu().tolist()   # the FP32 values the kernels use
        fctx.rho_device = rhos.device
        fctx.items = items
        fctx.pctx = pctx
        return torch.cat([pb.hist[-1] for pb in probs])

    @staticmethod
    def backward(fctx, grad):
        host_rhos = fctx.host_rhos   # taken in the forward: no device round trip here
        if grad is None:
            grad = torch.zeros(sum(fctx.sizes), dtype=torch.float32, device=fctx.hists[0].device)
        vs = list(grad.contiguous().float().split(fctx.sizes))   # contiguous pieces
        grads = []
        K = len(host_rhos)
        # one status word per instance and layer: a layer's launch writes
        # every instance's word, so each layer gets its own
        status = fctx.log.new(K * len(fctx.items), fctx.hists[0].device).view(K, -1)
        bb = P.BackBatch(fctx.items, ctx=fctx.pctx)
        for k in range(K - 1, -1, -1):
            bb.set_status(status[k])
            vs, gr = bb.run([h[k] for h in fctx.hists], vs, float(host_rhos[k]))
            grads.append(gr.sum().reshape(1))
        d_rho = torch.cat(grads[::-1]).to(fctx.rho_device)
        return d_rho, None, None, None


def bce_terms(x: torch.Tensor, alpha: torch.Tensor, g: Optional[torch.Tensor], known: bool,
              clamp: float = 1e-7) -> torch.Tensor:
    """Per-device terms of eq. Loss_alpha (known pathloss: z = alpha~) or
    eq. Loss_gamma (z = gamma~ / g); z clamped to [clamp, 1 - clamp].
    Evaluated in float64: in float32, 1 - 1e-7 rounds to 1 - 1.19e-7."""
    x = x.double()
    z = x if known else x / g.double()
    z = z.clamp(clamp, 1.0 - clamp)
    a = alpha.double()
    return -(a * torch.log(z) + (1.0 - a) * torch.log(1.0 - z))


def bce(x: torch.Tensor, alpha: torch.Tensor, g: Optional[torch.Tensor], known: bool, clamp: float = 1e-7):
    """The loss of one instance: the mean of its per-device terms."""
    return bce_terms(x, alpha, g, known, clamp).mean()


def batch_loss(net: "PscaNet", batch) -> torch.Tensor:
    """Mean over a minibatch of (Sigma_hat, S, params, alpha, g) of each
    instance's loss, from one concatenated forward: the device terms of
    instance b are weighted 1 / (B N_b), so instances of different N count
    equally, as in the mean of per-instance losses."""
    x = net.forward_batch_cat([(Sh, S, prm) for Sh, S, prm, _, _ in batch])
    alpha = torch.cat([a for _, _, _, a, _ in batch])
    g = None if net.known else torch.cat([gg for _, _, _, _, gg in batch])
    sizes = np.array([S.shape[1] for _, S, _, _, _ in batch])
    w = np.repeat(1.0 / (len(batch) * sizes), sizes)
    return (bce_terms(x, alpha, g, net.known) * torch.from_numpy(w).to(x.device)).sum()


class PscaNet(torch.nn.Module):
    """K-layer unrolled PSCA for one estimator (params.variant)."""

    def __init__(self, K: int, params: P.Params, ctx: Optional[P.Context] = None):
        super().__init__()
        self.params = params
        self.ctx = ctx
        self.rho = torch.nn.Parameter(torch.tensor(schedule(K), dtype=torch.float32))
        self.theta = 0.5
        self.status = StatusLog()

    @property
    def known(self) -> bool:
        return self.params.variant in (P.ML_K, P.MAP_K)

    def forward(self, Sigma_hat: torch.Tensor, S: torch.Tensor, params: Optional[P.Params] = None):
        prm = params or self.params
        return _Unrolled.apply(self.rho, Sigma_hat, S, prm, self.ctx or P.default_context(S.device), self.status)

    def forward_batch_cat(self, items) -> torch.Tensor:
        """x^(K) of every (Sigma_hat, S, params) of a minibatch, concatenated
        in order, in batched launches."""
        return _UnrolledBatch.apply(self.rho, list(items), self.ctx or P.default_context(items[0][1].device),
                                    self.status)

    def forward_batch(self, items):
        """x^(K) of every (Sigma_hat, S, params) of a minibatch, one tensor per
        instance (views of the concatenation)."""
        if not items:
            return ()
        return tuple(self.forward_batch_cat(items).split([S.shape[1] for _, S, _ in items]))

    def project(self):
        """Keep every step size in [0, 1] after an optimiser step."""
        with torch.no_grad():
            self.rho.clamp_(0.0, 1.0)


def train_step(net: PscaNet, opt: torch.optim.Optimizer, batch, batched: bool = True) -> float:
    """One Adam step on a minibatch of (Sigma_hat, S, params, alpha, g): the
    mean BCE over the minibatch.  batched: forward and backward of the whole
    minibatch in batched launches, else instance by instance."""
    opt.zero_grad()
    if batched:
        loss = batch_loss(net, batch)
        loss.backward()
        total = loss.detach()
    else:
        total = None
        for Sh, S, prm, alpha, g in batch:
            x = net(Sh, S, prm)
            loss = bce(x, alpha, g, net.known) / len(batch)
            loss.backward()
            total = loss.detach() if total is None else total + loss.detach()
    net.status.check()   # raises before the optimiser step if any launch flagged an instance
    opt.step()
    net.project()
    return float(total) if total is not None else 0.0


def stationarity_residual(Sigma_hat, S, params: P.Params, x: torch.Tensor, ctx=None) -> float:
    """How far x is from a stationary point of the estimator's objective,
    judged by plain PSCA: one iteration from x gives the coordinate
    minimisers x~ (Lemmas 1-4), and x~ = x exactly at a stationary point
    (Theorems 2-5).  Returns max|x~ - x| / max(max|x|, 1e-30)."""
    _, _, _, xt = P.iterate(Sigma_hat, S, x, 1.0, replace(params, x0=None), ctx=ctx)
    scale = torch.clamp(x.abs().max(), min=1e-30)
    return float(((xt - x).abs().max() / scale).item())


def detect_with_fallback(net: "PscaNet", Sigma_hat, S, params: Optional[P.Params] = None, tol: float = 1e-2,
                         extra_iters: int = 100, ctx=None):
    """The unrolled network with plain PSCA as its judge and its fallback:
    the network's output x^(K) is accepted when its stationarity residual
    (stationarity_residual) is at most tol; otherwise plain PSCA continues
    from x^(K) for extra_iters iterations with the schedule (one launch,
    params.x0 = x^(K)).  Returns (x, report) with the residual before and
    after and whether the fallback ran."""
    prm = params or net.params
    ctx = ctx or net.ctx
    with torch.no_grad():
        x = net(Sigma_hat, S, prm)
        net.status.check()
        res = stationarity_residual(Sigma_hat, S, prm, x, ctx=ctx)
        report = {"residual_net": res, "fallback": res > tol}
        if res > tol:
            status = torch.zeros(1, dtype=torch.int32, device=x.device)
            x = P.detect(Sigma_hat, S, replace(prm, iters=extra_iters, rho=None, x0=x), ctx=ctx, status=status)
            if int(status.item()) != 0:
                raise P.PscaError(int(status.item()), "fallback PSCA")
            report["residual_after"] = stationarity_residual(Sigma_hat, S, prm, x, ctx=ctx)
    return x, report


def choose_threshold(scores, truths) -> float:
    """Threshold minimising the average error rate ||alpha^ - alpha||_1 / n
    over validation data (detection is score >= threshold)."""
    import numpy as np
    s = np.concatenate([np.asarray(t.detach().cpu(), dtype=np.float64).ravel() for t in scores])
    a = np.concatenate([np.asarray(t.detach().cpu(), dtype=np.float64).ravel() for t in truths]) > 0.5
    order = np.argsort(s, kind="stable")
    s, a = s[order], a[order]
    n = s.size
    miss_before = np.concatenate([[0], np.cumsum(a)])            # actives below index i
    inactive_from = (~a)[::-1].cumsum()[::-1]                    # inactives at index >= i
    first = np.concatenate([[True], s[1:] != s[:-1]])            # first index of each distinct score
    idx = np.nonzero(first)[0]
    err = (miss_before[idx] + inactive_from[idx]) / n
    return float(s[idx[int(np.argmin(err))]])
