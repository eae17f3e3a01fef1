"""Shared helpers of the GPU parity tests (no GPU needed to import)."""
from __future__ import annotations

import numpy as np

import oracle as O

# Tolerances of the HIP path (complex FP32, FP32 accumulation) against the
# FP64 oracle, after a fixed number of iterations:
#   gamma (unknown pathloss): |err| <= REL_GAMMA * |x_ref| on entries with
#       |x_ref| >= FLOOR_FRAC * max|x_ref|, else <= ABS_SMALL_GAMMA * max|x_ref|
#   alpha (known pathloss, values in [0, 1]): |err| <= ABS_ALPHA
REL_GAMMA = 1e-4
FLOOR_FRAC = 1e-3
ABS_SMALL_GAMMA = 1e-6
ABS_ALPHA = 1e-4


def parity_report(x_gpu, x_ref, variant):
    x_gpu = np.asarray(x_gpu, dtype=np.float64)
    x_ref = np.asarray(x_ref, dtype=np.float64)
    err = np.abs(x_gpu - x_ref)
    if variant in O.KNOWN_PATHLOSS:
        bad = err > ABS_ALPHA
        return {"max_abs": float(err.max()), "n_bad": int(bad.sum()), "bad": np.nonzero(bad)[0]}
    scale = float(np.max(np.abs(x_ref))) if x_ref.size else 0.0
    big = (np.abs(x_ref) >= FLOOR_FRAC * scale) & (np.abs(x_ref) > 0)
    tol = np.where(big, REL_GAMMA * np.abs(x_ref), ABS_SMALL_GAMMA * scale)
    bad = err > tol
    rel = err[big] / np.abs(x_ref[big]) if (big.any() and scale > 0) else np.zeros(1)
    return {"max_rel_big": float(rel.max()), "max_abs_small_over_scale":
            float((err[~big].max() / scale) if (~big).any() and scale > 0 else 0.0),
            "n_bad": int(bad.sum()), "bad": np.nonzero(bad)[0]}


def assert_parity(x_gpu, x_ref, variant, what=""):
    rep = parity_report(x_gpu, x_ref, variant)
    assert rep["n_bad"] == 0, f"{what} {O.VARIANT_NAMES[variant]}: {rep}"
    return rep


def assert_same_support(x_gpu, x_ref, truth, variant, what=""):
    """Identical detected support at the oracle's equal-error threshold (and at
    0.5 for the known-pathloss variants), excluding devices whose oracle score
    lies within a relative 1e-4 of the threshold; the excluded devices are
    counted and printed.  Returns {threshold: (excluded, flips among them)}."""
    x_gpu = np.asarray(x_gpu, dtype=np.float64)
    x_ref = np.asarray(x_ref, dtype=np.float64)
    _, theta, _, _ = O.equal_error_rate(x_ref, truth)
    thetas = [theta] + ([0.5] if variant in O.KNOWN_PATHLOSS else [])
    scale = float(np.max(np.abs(x_ref)))
    counts = {}
    for th in thetas:
        near = np.abs(x_ref - th) <= 1e-4 * max(scale, abs(th))
        flips = (x_gpu >= th) != (x_ref >= th)
        n_flip = int(np.sum(flips & ~near))
        counts[float(th)] = (int(near.sum()), int(np.sum(flips & near)))
        assert n_flip == 0, f"{what} {O.VARIANT_NAMES[variant]}: {n_flip} support flips at theta={th}"
    print(f"  support identity {what} {O.VARIANT_NAMES[variant]}: "
          + ", ".join(f"theta={th:.4g}: {n} near-threshold devices excluded ({f} of them flipped)"
                      for th, (n, f) in counts.items()), flush=True)
    return counts


# MAP-UR devices whose iterates pass within this relative distance of a
# branch point of p^eps (eps, g_l - eps, g_l) are not held to the element-wise
# bar: the prior term has poles at the first two and a jump at the third, so
# there an FP32 trajectory cannot follow the FP64 one (see branch_margin).
BRANCH_DELTA = 1e-4


def map_ur_device_parity(x_gpu, x_ref, margin, delta=BRANCH_DELTA):
    """Element-wise MAP-UR parity on the devices whose oracle trajectory keeps
    a relative distance >= delta from every branch point.  Returns the
    report of the kept devices and the number excluded."""
    keep = np.asarray(margin) >= delta
    rep = parity_report(np.asarray(x_gpu)[keep], np.asarray(x_ref)[keep], O.MAP_UR)
    rep["excluded"] = int((~keep).sum())
    return rep


def stepwise_parity(prob, hist_gpu, rhos, delta=BRANCH_DELTA, errors=None):
    """One oracle iteration from each GPU iterate x^(k) (rounded values taken
    as exact) against the GPU's x^(k+1), element by element at the parity
    bar.  MAP-UR devices whose x^(k) lies within delta (relative) of a branch
    point of p^eps are skipped at that step.  Returns (worst report, total
    skipped device-steps); with a list `errors`, appends each step's
    |x_gpu^(k+1) - step(x_gpu^(k))| (float32, every device) to it."""
    hist = np.asarray(hist_gpu, dtype=np.float64)
    worst, skipped = None, 0
    for k, rho in enumerate(rhos):
        rec = O.psca_iteration(prob, hist[k], float(rho))
        if errors is not None:
            errors.append(np.abs(hist[k + 1] - rec.x_next).astype(np.float32))
        keep = np.ones(prob.N, dtype=bool)
        if prob.variant == O.MAP_UR:
            pr = prob.prior
            pts = np.array([pr.eps, pr.g_l - pr.eps, pr.g_l])
            d = np.min(np.abs(hist[k][:, None] - pts[None, :]) / pts[None, :], axis=1)
            keep = d >= delta
        skipped += int((~keep).sum())
        rep = parity_report(hist[k + 1][keep], rec.x_next[keep], prob.variant)
        rep["step"] = k
        err = rep.get("max_abs", rep.get("max_rel_big", 0.0))
        if worst is None or (rep["n_bad"], err) > (worst["n_bad"], worst.get("max_abs", worst.get("max_rel_big", 0.0))):
            worst = rep
        if (k + 1) % 25 == 0:
            print(f"  step-by-step check: {k + 1}/{len(rhos)} steps", flush=True)
    return worst, skipped
