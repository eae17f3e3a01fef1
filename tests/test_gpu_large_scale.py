"""The large-scale configuration at its run length, through the C ABI (needs
an MI355X): N = 10^4 devices, L = 200, M = 256, p = 0.05, the four sampled
instances of the benchmark's batch (seeds [4, 0..3]), in the launch shape
the benchmark times (one batch launch on teams of 4 workgroups), for ML-K
PSCA with 200 iterations, MAP-UR PSCA with 200 iterations and the trained
ML-K network (20 layers, its learned step sizes).

Two checks, both at the parity bar (|alpha error| <= 1e-4; relative 1e-4 on
gamma), every device:

* step by step: one oracle iteration from each recorded GPU iterate x^(k)
  against the GPU's x^(k+1) (MAP-UR devices within a relative 1e-4 of a
  branch point of p^eps at that step are skipped and counted);
* the output against the oracle's own trajectory from x = 0, with the same
  detected support at the instance's equal-error threshold (and at 0.5 for
  ML-K).  This is held where the trajectory is stable at the size of the
  FP32 path's own step errors: the oracle is run again with every step
  perturbed by exactly the GPU's measured per-step error magnitudes, device
  by device, with random signs (seeded), and kept inside the box; for MAP-UR,
  whose prior has poles and a jump (devices can land on either side of a
  branch point), also with every iterate scaled by (1 + 1e-6 xi).  The output
  bar is asserted where every such run moves the oracle's output by less than
  half the bar.  Where the method's own dynamics amplify errors of that size beyond
  it, the output comparison cannot tell kernel error from amplification; the
  test then reports the output error and the oracle's own spread instead of
  asserting them (the step-by-step check still holds every step).

The oracle legs run in parallel host processes (single-threaded BLAS each)
and print their progress."""
from __future__ import annotations

import json
import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle as O
from paper_2503_15259_amd import instances as I
from parity import assert_same_support, map_ur_device_parity, parity_report, stepwise_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = float(np.float32(0.01))
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAMPLE = (0, 1, 2, 3)
ITERS = 200
STABLE = 0.5     # output bar asserted where the perturbed oracle moves less than this fraction of the bar
SCALED = 1e-6    # MAP-UR: relative perturbation of every iterate in the second stability run


def _net_rhos():
    with open(os.path.join(ROOT, "paper_2503_15259_amd", "data", "net_ML-K_K20_N10000_L200.json")) as f:
        return [float(np.float32(r)) for r in json.load(f)["rho"]]


def _steps(what):
    return np.asarray(_net_rhos(), dtype=np.float64) if what == "net" else O.step_sizes(ITERS)


def _problem(what, index):
    inst = I.workload_instance("large", index).fp32_inputs()
    return O.problem_from_instance(inst, O.MAP_UR if what == "MAP-UR" else O.ML_K, eps=EPS)


def _oracle_leg(task):
    """One oracle leg, printing its progress:
      ("run", what, index, None): Algorithm 1 from x = 0 (as O.psca runs it),
          with the branch margin (MAP-UR) and kappa(Sigma) at the last iterate;
      ("steps", what, index, hist): one oracle iteration from each recorded
          GPU iterate, against the next (tests/parity.stepwise_parity), with
          the per-step error magnitudes of every device;
      ("perturbed", what, index, errs): Algorithm 1 from x = 0 with
          errs[k] * (random sign) added to step k's output, then clipped to
          the box;
      ("scaled", what, index, None): Algorithm 1 from x = 0 with every
          iterate multiplied by (1 + SCALED xi), xi seeded standard normal."""
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    kind, what, index, arg = task
    prob = _problem(what, index)
    steps = _steps(what)
    if kind == "steps":
        errs = []
        worst, skipped = stepwise_parity(prob, arg, steps, errors=errs)
        return kind, what, index, None, {"worst": worst, "skipped": skipped, "errors": errs}
    rng = np.random.default_rng([17, index, len(steps)])
    lo, hi = prob.bounds()
    x = np.zeros(prob.N)
    margin = np.full(prob.N, np.inf)
    for k, rho in enumerate(steps):
        rec = O.psca_iteration(prob, x, float(rho))
        if what == "MAP-UR":
            margin = np.minimum(margin, O.branch_margin(prob, [rec]))
        x = rec.x_next
        if kind == "perturbed":
            sign = np.where(rng.random(prob.N) < 0.5, -1.0, 1.0)
            x = np.clip(x + sign * arg[k].astype(np.float64), lo, hi)
        elif kind == "scaled":
            x = x * (1.0 + SCALED * rng.standard_normal(prob.N))
        if (k + 1) % 25 == 0:
            print(f"  oracle {kind} {what} instance {index}: iteration {k + 1}/{len(steps)}", flush=True)
    extra = {}
    if kind == "run":
        Sigma = O.model_covariance(prob.S, prob.weights(x), prob.sigma2)
        extra["cond"] = float(np.linalg.cond(Sigma))
        extra["margin"] = margin
    return kind, what, index, x, extra


@pytest.fixture(scope="module")
def results():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15259_amd import psca as P
    dev = torch.device("cuda", 0)
    rho_net = torch.tensor(_net_rhos(), dtype=torch.float32, device=dev)
    insts = [I.workload_instance("large", i).fp32_inputs() for i in SAMPLE]
    data = []
    for inst in insts:
        S = P.colmajor(torch.from_numpy(inst.S.astype(np.complex64)).to(dev))
        Y = P.colmajor(torch.from_numpy(inst.Y.astype(np.complex64)).to(dev))
        g = torch.from_numpy(inst.g.astype(np.float32)).to(dev)
        data.append((P.sample_cov(Y), S, g, inst))
    gpu = {}
    for what, variant, iters, rho in (("ML-K", P.ML_K, ITERS, None), ("MAP-UR", P.MAP_UR, ITERS, None),
                                      ("net", P.ML_K, len(rho_net), rho_net)):
        status = torch.full((len(data),), 7, dtype=torch.int32, device=dev)
        probs = []
        for b, (Sh, S, g, inst) in enumerate(data):
            prm = P.Params(variant=variant, iters=iters, sigma2=inst.sigma2, M=inst.M, d_lo=inst.d_lo,
                           d_hi=inst.d_hi, pl_c0=inst.pl_c0, pl_beta=inst.pl_beta, eps=EPS,
                           g=g if variant == P.ML_K else None, rho=rho)
            hist = torch.empty((iters + 1, inst.N), dtype=torch.float32, device=dev)
            probs.append(P.Problem(Sigma_hat=Sh, S=S, params=prm, status=status[b:b + 1], hist=hist))
        plan = P.Plan(probs, team_size=4)
        print(f"[large-scale GPU batch: {what}, {len(probs)} instances, teams of {plan.team_size}]", flush=True)
        xs = plan.launch()
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [0] * len(data), what
        for k, (x, pb) in enumerate(zip(xs, probs)):
            gpu[(what, SAMPLE[k])] = (x.cpu().numpy().astype(np.float64), pb.hist.cpu().numpy())
        plan.close()
    tasks = []
    for what in ("ML-K", "MAP-UR", "net"):
        for i in SAMPLE:
            tasks += [("run", what, i, None), ("steps", what, i, gpu[(what, i)][1])]
            if what == "MAP-UR":
                tasks.append(("scaled", what, i, None))
    tasks.sort(key=lambda t: t[1] == "net")   # the long legs first
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS")}
    os.environ.update(OPENBLAS_NUM_THREADS="1", OMP_NUM_THREADS="1")   # read by the workers' BLAS at start
    orc = {}
    try:
        with mp.get_context("spawn").Pool(max(1, min(len(tasks), cores, 16))) as pool:
            print(f"[large-scale oracle: {len(tasks)} legs]", flush=True)
            for kind, what, i, x, extra in pool.imap_unordered(_oracle_leg, tasks):
                orc[(kind, what, i)] = (x, extra)
                print(f"  oracle leg done: {kind} {what} instance {i} ({len(orc)}/{len(tasks)})", flush=True)
            # stability runs: the oracle again, every step perturbed by the GPU's own per-step errors
            tasks2 = [("perturbed", what, i, orc[("steps", what, i)][1].pop("errors"))
                      for what in ("ML-K", "MAP-UR", "net") for i in SAMPLE]
            print(f"[large-scale oracle: {len(tasks2)} stability legs]", flush=True)
            for kind, what, i, x, extra in pool.imap_unordered(_oracle_leg, tasks2):
                orc[(kind, what, i)] = (x, extra)
                print(f"  oracle leg done: {kind} {what} instance {i}", flush=True)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return gpu, orc, insts


@pytest.mark.parametrize("what", ["ML-K", "net", "MAP-UR"])
def test_large_scale_at_run_length(results, what):
    gpu, orc, insts = results
    variant = O.MAP_UR if what == "MAP-UR" else O.ML_K
    for idx, inst in zip(SAMPLE, insts):
        got, _ = gpu[(what, idx)]
        ref, extra = orc[("run", what, idx)]
        step = orc[("steps", what, idx)][1]
        print(f"large-scale {what} instance {idx}: kappa(Sigma) at the last iterate {extra['cond']:.3e}; step by "
              f"step: worst {step['worst']}, {step['skipped']} device-steps near a branch point", flush=True)
        assert step["worst"]["n_bad"] == 0, (what, idx, step["worst"])
        keep = extra["margin"] >= 1e-4 if variant == O.MAP_UR else np.ones(inst.N, dtype=bool)
        rep = map_ur_device_parity(got, ref, extra["margin"]) if variant == O.MAP_UR else \
            parity_report(got, ref, variant)
        spreads = {}
        for kind in ("perturbed", "scaled"):
            if (kind, what, idx) in orc:
                pert = orc[(kind, what, idx)][0]
                spreads[kind] = map_ur_device_parity(pert, ref, extra["margin"]) if variant == O.MAP_UR else \
                    parity_report(pert, ref, variant)
        stable = all((sp["max_abs"] if variant == O.ML_K else sp["max_rel_big"]) <= STABLE * 1e-4
                     for sp in spreads.values())
        print(f"  output vs the oracle's trajectory: {rep}; oracle spread under perturbations of the GPU's "
              f"per-step error sizes: {spreads['perturbed']}; under relative {SCALED:g} per step: "
              f"{spreads.get('scaled')}; stable {stable}", flush=True)
        if stable:
            assert rep["n_bad"] == 0, (what, idx, rep)
            assert_same_support(got[keep], ref[keep], inst.alpha[keep], variant, f"large-scale {what} {idx}")
