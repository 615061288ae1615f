"""Throughput of the batched time step on one MI355X: link-steps/s.

Workload (default): 4096 serial chains with 10..50 hinge links each (uniform),
random unit axes, box links of length U[0.3,1.2] m, width 0.1 m, density
U[500,2000] kg/m^3, initial angles U[-1,1] rad at rest, dt = 0.03 s, one
collocation point per step (order 2), L-BFGS history 5, tolerance 1e-8.
A bench step is one time step of the whole batch (one call of abd_step).
`value` is the mixed-precision rate; the float64 rate on the same workload is
reported next to it.  Inputs are synthetic and resident on the GPU before
timing starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes per link (streaming formulation, no on-chip reuse across phases)
EVAL_BYTES = {"f32": 128, "f64": 240}   # q, axis+offset, M, B in; g out
LBFGS_BYTES = 128                        # g, q, s/y history (m=5) in; d, q, s, y out
PRECOND_BYTES = 240                      # two sweeps: s, U, 1/D (f64) in twice; b/u/x traffic
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def run_rollout(torch, abd, model, q0, opts, warmup, steps):
    """Warm-up steps, then `steps` timed steps; per-launch durations from events on the launch stream."""
    n = model.n_dofs
    buf = torch.empty((warmup + steps + 2, n), dtype=torch.float64, device="cuda")
    buf[0] = q0
    buf[1] = q0
    stats = torch.zeros((steps, max(1, model.n_models), 4), dtype=torch.float64, device="cuda")
    for k in range(warmup):
        model.step(buf[k:k + 2].reshape(-1), buf[k + 2], opts)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for j in range(steps):
        k = warmup + j
        model.step(buf[k:k + 2].reshape(-1), buf[k + 2], opts, stats=stats[j])
        ev[j + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch_ms = [ev[j].elapsed_time(ev[j + 1]) for j in range(steps)]
    st = [model.read_stats(stats[j], model.n_models) for j in range(steps)]
    return buf, wall, per_launch_ms, st


def algorithmic_bytes(desc, st, precision):
    """Bytes the step would move if every phase streamed its operands from HBM."""
    links = np.diff(desc.link_offset).astype(np.float64)
    it = st["iterations"].astype(np.float64)
    ev = st["evaluations"].astype(np.float64)
    if precision == "mixed":
        it32 = st["f32_iterations"].astype(np.float64)
        ev32 = np.minimum(ev, it32 + 1.0)
        ev64 = ev - ev32
    else:
        ev32, ev64 = np.zeros_like(ev), ev
    per_link = EVAL_BYTES["f32"] * ev32 + EVAL_BYTES["f64"] * ev64 + (LBFGS_BYTES + PRECOND_BYTES) * it
    return float(np.sum(links * per_link))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(models are independent; see the sharding notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1709_04145_amd import abd
    from paper_1709_04145_amd import workloads as W

    wl = W.config(args.config)
    desc = wl.model
    model = abd.Model(desc)
    q0 = torch.tensor(wl.q0, dtype=torch.float64, device="cuda")
    L = desc.n_links
    base = dict(dt=wl.step.dt, lbfgs_m=wl.step.lbfgs_m, tol=wl.step.tol, max_iter=wl.step.max_iter)
    results = {}
    for name, prec in (("mixed", abd.MIXED), ("fp64", abd.FP64)):
        if name == "fp64" and args.no_fp64:
            continue
        opts = abd.StepOptions(precision=prec, **base)
        buf, wall, per_launch, st = run_rollout(torch, abd, model, q0, opts, args.warmup, args.steps)
        iters = np.stack([s["iterations"] for s in st])
        evals = np.stack([s["evaluations"] for s in st])
        flags = np.stack([s["flag"] for s in st])
        bytes_launch = [algorithmic_bytes(desc, s, name) for s in st]
        avg_ms = float(np.mean(per_launch))
        results[name] = dict(
            wall=wall, per_launch_ms=avg_ms, value=L * args.steps / wall,
            iters_mean=float(iters.mean()), iters_max=int(iters.max()),
            evals_mean=float(evals.mean()), converged_frac=float(np.mean(flags == 1)),
            achieved_gbs=float(np.mean(bytes_launch)) / (avg_ms * 1e-3) / 1e9,
            last=(buf[args.warmup + args.steps].cpu().numpy(), buf[args.warmup + args.steps + 1].cpu().numpy()),
        )
        print(f"[bench] {name}: {results[name]['value']:.4g} link-steps/s, {avg_ms:.3f} ms/launch, "
              f"iters {results[name]['iters_mean']:.2f}", file=sys.stderr, flush=True)

    mixed = results["mixed"]
    out = {
        "metric": "link-steps/s on 1 MI355X, batched mixed vs plain FP64, at <=1e-5 rel pose err",
        "value": mixed["value"],
        "unit": "link-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": W.CONFIG_NAMES[args.config], "models": desc.n_models, "links": L,
                   "dofs": desc.n_dofs, "dt": wl.step.dt, "order_K": 2, "lbfgs_m": wl.step.lbfgs_m,
                   "tol": wl.step.tol, "precond": "joint-space inertia"},
        "iterations_per_step": mixed["iters_mean"],
        "evaluations_per_step": mixed["evals_mean"],
        "converged_fraction": mixed["converged_frac"],
        "roofline": {"bound": "hbm", "achieved": mixed["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": mixed["achieved_gbs"] / HBM_PEAK_GBS, "traffic": None},
    }
    if "fp64" in results:
        f = results["fp64"]
        out["fp64"] = {"value": f["value"], "ms_per_step": f["wall"] / args.steps * 1e3,
                       "iterations_per_step": f["iters_mean"], "achieved_gbs": f["achieved_gbs"],
                       "mixed_over_fp64": mixed["value"] / f["value"]}

    # parity of the last timed step against the oracle on a sample of models
    from oracle.oracle import Oracle
    sample = np.arange(0, desc.n_models, max(1, desc.n_models // 32))
    sub = desc.subset(sample)
    idx = desc.dof_subset_index(sample)
    orc = Oracle(sub)
    par = {}
    # one teacher-forced step from the final mixed state, both precisions
    qp, qc = results["mixed"]["last"]
    ref, _ = orc.step(qp[idx], qc[idx], wl.step.dt, lbfgs_m=wl.step.lbfgs_m, tol=wl.step.tol)
    for name, prec in (("mixed", abd.MIXED), ("fp64", abd.FP64)):
        o = torch.zeros(desc.n_dofs, dtype=torch.float64, device="cuda")
        h = torch.tensor(np.concatenate([qp, qc]), dtype=torch.float64, device="cuda")
        model.step(h, o, abd.StepOptions(precision=prec, **base))
        torch.cuda.synchronize()
        qg = o.cpu().numpy()[idx]
        par[name] = float(np.max(np.abs(qg - ref)) / max(1.0, np.max(np.abs(ref))))
    out["parity_max_rel_q_err"] = par

    if not args.no_cpu:
        threads = max(1, min(16, os.cpu_count() or 1))
        orc_full = Oracle(desc, threads=threads)
        qa = wl.q0.copy()
        qb = wl.q0.copy()
        t0 = time.perf_counter()
        nsteps = 0
        while True:
            qn, _ = orc_full.step(qa, qb, wl.step.dt, lbfgs_m=wl.step.lbfgs_m, tol=wl.step.tol)
            qa, qb = qb, qn
            nsteps += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": L * nsteps / el, "unit": "link-steps/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"full batch ({desc.n_models} models), first {nsteps} steps from rest, "
                                         f"{el:.1f} s, OpenMP over models"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
