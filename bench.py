"""Throughput of batched position-based time integration on one MI355X: link-steps/s.

Workload (default, "chains4096_uneven10to50"): 4096 serial chains with 10..50
hinge links each (uniform), random unit axes, box links of length U[0.3,1.2] m,
width 0.1 m, density U[500,2000] kg/m^3, initial angles U[-1,1] rad at rest,
dt = 0.03 s, one collocation point per step (order 2), L-BFGS history 5,
relative gradient tolerance 1e-8, inertia-preconditioned L-BFGS.

A bench step is one time step of the whole batch.  The warm-up steps run as one
rollout launch (abd_rollout) from rest; the K timed steps run as one more
rollout launch from where the warm-up ended, with the inputs already on the
GPU.  `value` is the mixed-precision rate; the float64 rate on the same
workload is reported next to it.

Also reported:
  roofline     algorithmic bytes of the timed launch (per-link figures below,
               times the float32 and float64 evaluations and the iterations the
               launch performed, as counted by the kernel) over the launch's
               duration measured with HIP events on the launch stream, against
               the 8 TB/s HBM peak; the preconditioner's and the step setup's
               bytes are reported beside it (extra_bytes), not in it;
  cpu_baseline the oracle (C, OpenMP over models) on a sample of the models
               over the same steps, and (cpu_baseline.parity) the oracle's
               solution of one teacher-forced step from the final state on a
               sample of models next to the GPU's (both precisions, both solved
               to a 1e-12 relative gradient, at most 2000 iterations): q and
               pose errors over the models where both sides converge to the
               same minimum (equal objective to 1e-9 of its scale); the step
               objective is non-convex on this workload, so models where the two
               reach different local minima, and models where either side stops
               at the iteration cap, are counted separately.  The oracle runs in
               this leg only (--no-cpu skips it).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic bytes per link (one DOF per link), streaming form: every operand
# read from and every result written to HBM once per use, no on-chip reuse.
# evaluation, float32 terms: read q 8, axis+offset 24, M 40, B 48; write g 8
# evaluation, float64 terms: read q 8, axis+offset 48, M 80, B 96; write g 8
# These and the L-BFGS figure are the method's work per link-iteration; the
# roofline fraction counts them only.
EVAL_BYTES = {"f32": 128, "f64": 240}
LBFGS_BYTES = 128                       # read g, q, s/y history (m=5); write d, q, s, y
# Work of this implementation's choices, reported separately (extra_bytes):
PRECOND_BYTES = 240                     # per iteration: two sweeps over the recursion records (s, U, 1/D) + b/u/x
SETUP_BYTES = 328                       # per step: read q_{k-1}, q_k, axis/offset, M; write B (f64+f32), records
HBM_PEAK_GBS = 8000.0
# committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of the order-2 rollout kernel, one per workload
TRAFFIC_PROFILE_GLOB = os.path.join(ROOT, "profiles", "k_rollout_*_hbm_traffic.md")


# tolerance of the parity sample: at 1e-12 a step's result is implied to ~3e-11
# (the oracle's own results at 1e-12 and 1e-13 differ by that), at 1e-11 only to ~1e-9
PARITY_TOL = 1e-12
PARITY_MAX_ITER = 2000
# CG of the rollout derivative; iteration cap of the order-K oracle sample
VJP_TOL = 1e-10
VJP_MAX_ITER = 200
HOC_CPU_ITERS = 20

# sources the order-2 rollout kernel is built from (the traffic summary is keyed to them)
ROLLOUT_SOURCES = ("abd_device.h", "abd_internal.h", "rollout.hip")


def kernel_source_digest():
    """sha256 over the order-2 rollout kernel's sources (in ROLLOUT_SOURCES order)."""
    import hashlib
    h = hashlib.sha256()
    for name in ROLLOUT_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1709_04145_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, precision, warmup, steps):
    """HBM bytes of the timed launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summaries: their machine-readable blocks (one per measured launch, separated by
    blank lines) are searched for one taken on this kernel source, workload,
    precision and step window; None if there is none."""
    import glob
    text = ""
    for path in sorted(glob.glob(TRAFFIC_PROFILE_GLOB)):
        with open(path) as f:
            text += f.read() + "\n\n"
    digest = kernel_source_digest()
    want = {"source_sha256": digest, "workload": workload, "precision": precision,
            "warmup": str(warmup), "steps": str(steps)}
    blocks, kv = [], {}
    for line in text.splitlines() + [""]:
        if ": " in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(": ", 1)
            kv[k.strip()] = v.strip()
        elif not line.strip() and kv:
            blocks.append(kv)
            kv = {}
    for kv in blocks:
        if all(kv.get(k) == v for k, v in want.items()) and "traffic_bytes" in kv:
            return float(kv["traffic_bytes"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--solver", choices=("auto", "lbfgs", "lm"), default="auto",
                    help="step optimizer: auto = Levenberg-Marquardt for order K = 3 (the sum-of-squares "
                         "Eq. EQHOC), L-BFGS otherwise; lm at order 2 runs float64 only")
    ap.add_argument("--order", type=int, default=0,
                    help="collocation order K instead of the configuration's (0: the configuration's)")
    ap.add_argument("--schedule", choices=("auto", "wave", "tile"), default="auto",
                    help="how models map onto wavefronts (auto: the library's autotuner)")
    ap.add_argument("--dt", type=float, default=0.0, help="time step instead of the configuration's (0: the "
                                                             "configuration's)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-parity", action="store_true", help="skip the teacher-forced parity sample")
    ap.add_argument("--cpu-models", type=int, default=4096, help="models in the CPU baseline sample")
    ap.add_argument("--vjp", action="store_true",
                    help="also time the rollout's reverse-mode derivative (abd_rollout_vjp; on for configuration 5)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB of float64 device to device three times (the known-size kernel "
                         "that calibrates rocprofv3's FETCH_SIZE and WRITE_SIZE counters), then exit")
    return ap.parse_args()


def copy_probe(torch):
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {x.numel() * 8} bytes three times", flush=True)


def timed_rollout(torch, model, q0, opts, warmup, steps, torque=None):
    """Warm-up rollout from rest, then `steps` timed steps in one launch
    (torque: [warmup + steps, n_dofs] joint forces, or None)."""
    n = model.n_dofs
    K = opts.order_K
    q0c = torch.as_tensor(q0, dtype=torch.float64, device="cuda")
    init = torch.cat([q0c, q0c]).contiguous()
    tw = tt = None
    if torque is not None:
        tq = torch.as_tensor(torque, dtype=torch.float64, device="cuda")
        tw, tt = tq[:warmup].contiguous(), tq[warmup:warmup + steps].contiguous()
    if warmup > 0:
        wtraj, _ = model.rollout(init, warmup, opts, torque=tw)
        if K == 2:
            prev = wtraj[warmup - 2] if warmup >= 2 else q0c
            init = torch.cat([prev, wtraj[warmup - 1]]).contiguous()
        else:  # known points of the next step: the last step's alpha_{K-2} point and q_{k+1}
            init = torch.cat([wtraj[warmup - 1, K - 3], wtraj[warmup - 1, K - 2]]).contiguous()
    traj = torch.empty((steps, n) if K == 2 else (steps, K - 1, n), dtype=torch.float64, device="cuda")
    stats = model.new_rollout_stats(steps)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    model.rollout(init, steps, opts, torque=tt, q_traj=traj, stats=stats)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1)
    st = model.read_rollout_stats(stats, steps)
    return init, traj, st, wall, kernel_ms


def algorithmic_bytes(desc, st):
    """Bytes the timed launch would move in the streaming formulation of the
    method: per link, EVAL_BYTES per evaluation (float32 or float64, as the
    kernel counted them) and LBFGS_BYTES per iteration.  Returns (bytes,
    extra_bytes), extra_bytes being the preconditioner's and the step setup's."""
    links = np.diff(desc.link_offset).astype(np.float64)[None, :]
    it = st["iterations"].astype(np.float64)
    ev = st["evaluations"].astype(np.float64)
    ev32 = st["f32_evaluations"].astype(np.float64)
    ev64 = ev - ev32
    per_link = EVAL_BYTES["f32"] * ev32 + EVAL_BYTES["f64"] * ev64 + LBFGS_BYTES * it
    extra = PRECOND_BYTES * it + SETUP_BYTES
    return float(np.sum(links * per_link)), float(np.sum(links * extra))


def pose_error(orc, desc, q, ref):
    """Relative pose error: max over links of |x - x_ref| / reach of the link's model
    (sum of its link lengths), and max |R - R_ref|_F."""
    A, B = orc.poses(q), orc.poses(ref)
    lo = desc.link_offset
    ex, eR = 0.0, 0.0
    for i in range(desc.n_models):
        sl = slice(lo[i], lo[i + 1])
        if lo[i + 1] == lo[i]:
            continue
        reach = np.sum(np.linalg.norm(desc.offset[sl], axis=1)) + 2.0 * np.max(
            desc.mass_moment[sl, 3] / desc.mass_moment[sl, 9])
        ex = max(ex, float(np.max(np.linalg.norm(A[sl, :, 3] - B[sl, :, 3], axis=1)) / reach))
        eR = max(eR, float(np.max(np.linalg.norm(A[sl, :, :3] - B[sl, :, :3], axis=(1, 2)))))
    return ex, eR


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the models are independent, "
              "so a multi-GPU run would shard them and gather the results once (see the sharding notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe:
        copy_probe(torch)
        return

    from paper_1709_04145_amd import abd
    from paper_1709_04145_amd import workloads as W

    wl = W.config(args.config)
    if args.dt > 0.0:
        wl.step.dt = args.dt
    desc = wl.model
    if wl.torque is not None and args.warmup + args.steps > wl.torque.shape[0]:
        print(f"configuration {args.config} defines joint forces for {wl.torque.shape[0]} steps: "
              f"--warmup + --steps must not exceed that", file=sys.stderr)
        sys.exit(2)
    model = abd.Model(desc)
    L = desc.n_links
    K = args.order if args.order > 0 else wl.step.order_K
    solver = {"lbfgs": abd.SOLVER_LBFGS, "lm": abd.SOLVER_LM}.get(args.solver,
                                                                  abd.SOLVER_LM if K == 3 else abd.SOLVER_LBFGS)
    schedule = {"auto": abd.SCHEDULE_AUTO, "wave": abd.SCHEDULE_WAVE, "tile": abd.SCHEDULE_TILE}[args.schedule]
    base = dict(dt=wl.step.dt, lbfgs_m=wl.step.lbfgs_m, tol=wl.step.tol, max_iter=wl.step.max_iter, order_K=K,
                solver=solver, schedule=schedule)
    runs = {}
    lm = solver == abd.SOLVER_LM
    for name, prec in (("mixed", abd.MIXED), ("fp64", abd.FP64)):
        if name == "fp64" and args.no_fp64 and K == 2 and not lm:
            continue
        if name == "mixed" and lm:
            continue  # Levenberg-Marquardt runs in float64 only
        opts = abd.StepOptions(precision=prec, **base)
        init, traj, st, wall, kms = timed_rollout(torch, model, wl.q0, opts, args.warmup, args.steps, wl.torque)
        nbytes, xbytes = algorithmic_bytes(desc, st)
        links = np.diff(desc.link_offset)[None, :]
        runs[name] = dict(
            init=init, traj=traj, st=st, wall=wall, kernel_ms=kms, value=L * args.steps / wall,
            iters_mean=float(st["iterations"].mean()), iters_max=int(st["iterations"].max()),
            evals_mean=float(st["evaluations"].mean()),
            f32_eval_share=float(np.sum(links * st["f32_evaluations"]) / max(1, np.sum(links * st["evaluations"]))),
            converged_frac=float(np.mean(st["flag"] == abd.FLAG_CONVERGED)),
            link_iters=float(np.sum(links * st["iterations"])),
            achieved_gbs=nbytes / (kms * 1e-3) / 1e9, bytes=nbytes, extra_bytes=xbytes)
        print(f"[bench] {name}: {runs[name]['value']:.4g} link-steps/s, kernel {kms:.2f} ms for {args.steps} "
              f"steps, iters/step {runs[name]['iters_mean']:.2f} (max {runs[name]['iters_max']})",
              file=sys.stderr, flush=True)

    mixed = runs["mixed"] if "mixed" in runs else runs["fp64"]
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
        "dtype": "f32+f64" if "mixed" in runs else "f64",
        "data": "synthetic",
        "config": {"workload": W.CONFIG_NAMES[args.config], "models": desc.n_models, "links": L,
                   "dofs": desc.n_dofs, "dt": wl.step.dt, "order_K": K, "lbfgs_m": wl.step.lbfgs_m,
                   "tol": wl.step.tol,
                   "solver": "levenberg-marquardt" if solver == abd.SOLVER_LM else "l-bfgs",
                   "precond": "joint-space inertia" if solver == abd.SOLVER_LBFGS else None,
                   "schedule": args.schedule,
                   "launch": "one rollout per K steps"},
        "iterations_per_step": mixed["iters_mean"],
        "iterations_per_step_max": mixed["iters_max"],
        "evaluations_per_step": mixed["evals_mean"],
        "converged_fraction": mixed["converged_frac"],
        "link_iterations_per_s": mixed["link_iters"] / mixed["wall"],
        "roofline": {"bound": "hbm", "achieved": mixed["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": mixed["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(W.CONFIG_NAMES[args.config], "mixed" if "mixed" in runs else "fp64",
                                                 args.warmup, args.steps) if args.dt == 0.0 else None,
                     "kernel": ("k_rollout_hoc<MIXED>" if K > 2 else "k_rollout<MIXED, extras>" if desc.has_extras
                                else "k_rollout<MIXED>") if "mixed" in runs else
                     ("k_rollout_lm2" if lm and K == 2 else "k_rollout_lm" if lm else
                      "k_rollout<FP64>" if K == 2 else "k_rollout_hoc"),
                     "kernel_ms": mixed["kernel_ms"],
                     "algorithmic_bytes": mixed["bytes"],
                     "extra_bytes": mixed["extra_bytes"],
                     "bytes_per_link": {"eval_f32": EVAL_BYTES["f32"], "eval_f64": EVAL_BYTES["f64"],
                                        "lbfgs_iteration": LBFGS_BYTES}},
        "float32_evaluation_share": mixed["f32_eval_share"],
    }
    if "fp64" in runs and "mixed" in runs:
        f = runs["fp64"]
        out["fp64"] = {"value": f["value"], "ms_per_step": f["wall"] / args.steps * 1e3,
                       "iterations_per_step": f["iters_mean"], "iterations_per_step_max": f["iters_max"],
                       "converged_fraction": f["converged_frac"], "kernel_ms": f["kernel_ms"],
                       "achieved_gbs": f["achieved_gbs"], "mixed_over_fp64": mixed["value"] / f["value"]}

    if (args.vjp or args.config == 5) and K == 2 and "fp64" in runs:
        out["vjp"] = time_vjp(torch, abd, model, desc, wl, runs["fp64"], args)

    if K == 2:
        src = runs["fp64"] if "fp64" in runs else runs["mixed"]
        out["energy"] = energy_drift(torch, model, desc, wl, src, args)

    tf = None
    if not args.no_parity and not args.no_cpu and K == 2 and not lm:
        tf = teacher_forced_gpu(torch, abd, model, desc, wl, runs, base, args)

    if not args.no_cpu and K == 2 and lm:
        out["cpu_baseline"] = eq_lm_cpu_baseline(desc, wl, runs["fp64"], args.warmup)
    if not args.no_cpu and K == 2 and not lm:
        from oracle.oracle import Oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        nsub = max(1, min(desc.n_models, args.cpu_models))
        sample = np.arange(0, desc.n_models, max(1, desc.n_models // nsub))[:nsub]
        sub = desc.subset(sample)
        idx = desc.dof_subset_index(sample)
        orc = Oracle(sub, threads=threads)
        qa = wl.q0[idx].copy()
        qb = qa.copy()
        kw = dict(lbfgs_m=wl.step.lbfgs_m, tol=wl.step.tol, max_iter=wl.step.max_iter)
        tq = (lambda k: None) if wl.torque is None else (lambda k: wl.torque[k][idx])
        for k in range(args.warmup):
            qn, _ = orc.step(qa, qb, wl.step.dt, tq(k), **kw)
            qa, qb = qb, qn
            print(f"[bench] cpu baseline: warm-up step {k} done", file=sys.stderr, flush=True)
        qa0, qb0 = qa.copy(), qb.copy()  # the state the timed steps start from
        t0 = time.perf_counter()
        nsteps = 0
        while nsteps < args.steps:
            qn, _ = orc.step(qa, qb, wl.step.dt, tq(args.warmup + nsteps), **kw)
            qa, qb = qb, qn
            nsteps += 1
            if nsteps % 10 == 0 or time.perf_counter() - t0 > 30.0:
                print(f"[bench] cpu baseline: {nsteps} timed steps done", file=sys.stderr, flush=True)
            if time.perf_counter() - t0 > 30.0:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": sub.n_links * nsteps / el, "unit": "link-steps/s", "cores": threads,
                               "kind": "oracle", "host_cores": os.cpu_count(),
                               "sample": f"{len(sample)} of {desc.n_models} models ({sub.n_links} links), steps "
                                         f"{args.warmup}..{args.warmup + nsteps - 1} after a {args.warmup}-step "
                                         f"warm-up from rest, float64, OpenMP over models, {el:.1f} s"}
        # one core: the same timed steps, from the same state, on the first models
        # of the sample, as many as one core steps in about 2 s by the rate above
        cpu_s_per_link_step = el * threads / (sub.n_links * nsteps)
        links = np.cumsum(np.diff(sub.link_offset))
        n1 = max(1, int(np.searchsorted(links, 2.0 / cpu_s_per_link_step, side="right")))
        sub1 = sub.subset(np.arange(n1))
        idx1 = sub.dof_subset_index(np.arange(n1))
        orc1 = Oracle(sub1, threads=1)
        qa1, qb1 = qa0[idx1].copy(), qb0[idx1].copy()
        tq1 = (lambda k: None) if wl.torque is None else (lambda k: wl.torque[k][idx][idx1])
        t0 = time.perf_counter()
        n1steps = 0
        while n1steps < args.steps and time.perf_counter() - t0 < 15.0:
            qn, _ = orc1.step(qa1, qb1, wl.step.dt, tq1(args.warmup + n1steps), **kw)
            qa1, qb1 = qb1, qn
            n1steps += 1
        el1 = time.perf_counter() - t0
        out["cpu_baseline"]["single_core"] = {
            "value": sub1.n_links * n1steps / el1, "unit": "link-steps/s", "cores": 1,
            "sample": f"{n1} models ({sub1.n_links} links), steps {args.warmup}..{args.warmup + n1steps - 1}, "
                      f"{el1:.1f} s"}
        print(f"[bench] cpu baseline: single core done ({n1steps} steps)", file=sys.stderr, flush=True)
        if tf is not None:
            print("[bench] parity: oracle solving the teacher-forced step", file=sys.stderr, flush=True)
            out["cpu_baseline"]["parity"] = parity_vs_oracle(abd, desc, wl, tf)
    if not args.no_cpu and K > 2:
        out["cpu_baseline"] = (hoc_lm_cpu_baseline(desc, wl, runs["fp64"], K) if solver == abd.SOLVER_LM
                               else hoc_cpu_baseline(desc, wl, runs["fp64"], K))
    print(json.dumps(out), flush=True)


def model_energy(poses, prev_poses, desc, dt):
    """Reported energy per model: (1/2 dt^2) sum_l tr(dA_l M_l dA_l^T) + V(q_k),
    dA = A(q_k) - A(q_{k-1}), V = -sum_l g^T A_l M_l e4, from world poses
    [n_links, 3, 4] (host arithmetic on the GPU's forward kinematics)."""
    mm = desc.mass_moment
    M = np.zeros((desc.n_links, 4, 4))
    iu = np.triu_indices(4)
    M[:, iu[0], iu[1]] = mm
    M[:, iu[1], iu[0]] = mm
    dA = poses - prev_poses
    ke = 0.5 * np.einsum("lij,ljk,lik->l", dA, M, dA) / (dt * dt)
    pot = -np.einsum("i,lij,lj->l", desc.gravity, poses, M[:, :, 3])
    lo = desc.link_offset
    return np.add.reduceat(ke + pot, lo[:-1]) if desc.n_links else np.zeros(desc.n_models)


def energy_drift(torch, model, desc, wl, run, args):
    """Energy at the start and at the end of the timed launch (float64 run)."""
    n = desc.n_dofs
    init = run["init"]
    tr = run["traj"]
    P = lambda q: model.poses(q.contiguous()).cpu().numpy().reshape(desc.n_links, 3, 4)
    h0 = model_energy(P(init[n:]), P(init[:n]), desc, wl.step.dt)
    last_prev = tr[-2] if args.steps >= 2 else init[n:]
    h1 = model_energy(P(tr[-1]), P(last_prev), desc, wl.step.dt)
    ok = np.nonzero(np.diff(desc.link_offset) > 0)[0]
    # the potential's zero level is the world origin, so only changes are meaningful
    return {"definition": "(1/2dt^2) sum tr(dA M dA^T) + V(q_k), per model, float64 run",
            "mean_J_start": float(np.mean(h0[ok])), "mean_J_end": float(np.mean(h1[ok])),
            "mean_change_per_step_J": float(np.mean(h1[ok] - h0[ok])) / max(1, args.steps),
            "models_losing_energy": float(np.mean(h1[ok] < h0[ok]))}


def parity_tol(args, wl):
    """Tolerance of the teacher-forced parity sample: PARITY_TOL for the chains,
    trees and ropes; for the swimmers and spiders (drag, contact), whose float64
    gradient floor lies higher, 1/100 of the workload's tolerance."""
    return PARITY_TOL if args.config <= 5 else 1e-2 * wl.step.tol


def teacher_forced_gpu(torch, abd, model, desc, wl, runs, base, args):
    """One step of every model from the final float64 state (both precisions
    start from the same float64 (q_{k-1}, q_k)), solved to PARITY_TOL on the GPU."""
    src = runs["fp64"] if "fp64" in runs else runs["mixed"]
    tr = src["traj"].cpu().numpy()
    qp, qc = (tr[-2], tr[-1]) if args.steps >= 2 else (src["init"].cpu().numpy()[:desc.n_dofs], tr[-1])
    hist = torch.tensor(np.concatenate([qp, qc]), dtype=torch.float64, device="cuda")
    res = {"qp": qp, "qc": qc, "tol": parity_tol(args, wl)}
    for name, prec in (("fp64", abd.FP64), ("mixed", abd.MIXED)):
        o = torch.zeros(desc.n_dofs, dtype=torch.float64, device="cuda")
        st = model.new_stats()
        model.step(hist, o, abd.StepOptions(precision=prec, **dict(base, tol=parity_tol(args, wl),
                                                                     max_iter=PARITY_MAX_ITER)), stats=st)
        torch.cuda.synchronize()
        res[name] = (o.cpu().numpy(), model.read_stats(st, desc.n_models))
    return res


def parity_vs_oracle(abd, desc, wl, tf):
    """The oracle's solution of the same teacher-forced step on a sample of models
    next to the GPU's (part of the CPU-baseline leg)."""
    from oracle.oracle import Oracle
    qp, qc = tf["qp"], tf["qc"]
    sample = np.arange(0, desc.n_models, max(1, desc.n_models // 64))
    sub = desc.subset(sample)
    idx = desc.dof_subset_index(sample)
    orc = Oracle(sub)
    ref, rst = orc.step(qp[idx], qc[idx], wl.step.dt, lbfgs_m=wl.step.lbfgs_m, tol=tf["tol"],
                        max_iter=PARITY_MAX_ITER)
    E_ref, _, S_ref = orc.objective_grad(ref, qp[idx], qc[idx], wl.step.dt)
    par = {}
    for name in ("fp64", "mixed"):
        qfull, st = tf[name]
        gst = st[sample]
        qg = qfull[idx]
        E_g, _, _ = orc.objective_grad(qg, qp[idx], qc[idx], wl.step.dt)
        conv = (gst["flag"] == abd.FLAG_CONVERGED) & (rst["flag"] == 1)
        same = conv & (np.abs(E_g - E_ref) <= 1e-9 * S_ref)
        qerr, perr = 0.0, 0.0
        keep = np.nonzero(same)[0]
        if len(keep):
            sd = sub.subset(keep)
            si = sub.dof_subset_index(keep)
            qerr = float(np.max(np.abs(qg[si] - ref[si])) / max(1.0, np.max(np.abs(ref[si]))))
            perr = pose_error(Oracle(sd), sd, qg[si], ref[si])[0]
        distinct = conv & ~same
        par[name] = {"models_same_minimum": int(same.sum()), "max_rel_q_err": qerr, "max_rel_pose_err": perr,
                     "models_distinct_minima": int(distinct.sum()),
                     "max_rel_objective_gap_distinct": float(np.max(np.abs(E_g - E_ref)[distinct] / S_ref[distinct]))
                     if distinct.any() else 0.0,
                     "models_not_converged": int((~conv).sum())}
    return {"sample_models": int(len(sample)), "tol": tf["tol"], **par}


def time_vjp(torch, abd, model, desc, wl, run, args):
    """The rollout's reverse-mode derivative for a seed on the last configuration
    (implicit differentiation, abd_rollout_vjp), timed with HIP events on the
    launch stream after one untimed call; the oracle's dense implicit
    differentiation of the same trajectory timed on a sample of models."""
    n, T = desc.n_dofs, args.steps
    seed = np.zeros((T, n))
    seed[-1] = np.random.default_rng(7).standard_normal(n)
    dl = torch.as_tensor(seed, dtype=torch.float64, device="cuda")
    st = model.new_rollout_stats(T)
    kw = dict(tol=VJP_TOL, max_iter=VJP_MAX_ITER)
    model.rollout_vjp(run["init"], run["traj"], dl, wl.step.dt, stats=st, **kw)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    model.rollout_vjp(run["init"], run["traj"], dl, wl.step.dt, stats=st, **kw)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s = model.read_rollout_stats(st, T)
    res = {"value": desc.n_links * T / (ms * 1e-3), "unit": "link-steps/s", "kernel": "k_rollout_vjp",
           "kernel_ms": ms, "cg_iterations_per_step": float(s["iterations"].mean()),
           "cg_iterations_max": int(s["iterations"].max()),
           "converged_fraction": float(np.mean(s["flag"] == abd.FLAG_CONVERGED)), "cg_tol": VJP_TOL}
    if not args.no_cpu:
        from oracle.oracle import Oracle
        nsub = min(desc.n_models, 64)
        sample = np.arange(0, desc.n_models, max(1, desc.n_models // nsub))[:nsub]
        sub = desc.subset(sample)
        idx = desc.dof_subset_index(sample)
        qi = run["init"].cpu().numpy()
        tr = run["traj"].cpu().numpy()[:, idx]
        threads = max(1, min(16, os.cpu_count() or 1))
        t0 = time.perf_counter()
        Oracle(sub, threads=threads).rollout_vjp(qi[:n][idx], qi[n:][idx], tr, wl.step.dt, seed[:, idx])
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": sub.n_links * T / el, "unit": "link-steps/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{nsub} of {desc.n_models} models ({sub.n_links} links), the same {T} "
                                         f"steps, dense Hessians and solves, {el:.1f} s"}
    return res


def hoc_cpu_baseline(desc, wl, run, K):
    """The oracle's order-K step on a bounded sample: one step of a few models from
    the GPU's timed starting state with the iterations capped, as link-iterations/s
    (the steps of this workload do not converge within the cap in either
    implementation, so link-steps/s would only measure the cap)."""
    from oracle.oracle import Oracle
    n = desc.n_dofs
    threads = max(1, min(16, os.cpu_count() or 1))
    nsub = min(desc.n_models, threads)
    sample = np.arange(0, desc.n_models, max(1, desc.n_models // nsub))[:nsub]
    sub = desc.subset(sample)
    idx = desc.dof_subset_index(sample)
    init = run["init"].cpu().numpy()
    t0 = time.perf_counter()
    _, st = Oracle(sub, threads=threads).step_hoc(K, init[:n][idx], init[n:][idx], wl.step.dt,
                                                  lbfgs_m=wl.step.lbfgs_m, tol=wl.step.tol,
                                                  max_iter=HOC_CPU_ITERS)
    el = time.perf_counter() - t0
    li = float(np.sum(np.diff(sub.link_offset) * st["iterations"]))
    return {"value": li / el, "unit": "link-iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"one step of {nsub} of {desc.n_models} models ({sub.n_links} links) from the timed "
                      f"launch's starting state, at most {HOC_CPU_ITERS} iterations, float64, {el:.1f} s; "
                      f"compare with link_iterations_per_s"}


def hoc_lm_cpu_baseline(desc, wl, run, K):
    """The oracle's Levenberg-Marquardt step (dense written-out Jacobian, Cholesky)
    on a bounded sample: the first timed step of a few models from the GPU's
    starting state, and the largest distance of the GPU's result from the
    oracle's on them (both solved to the workload's tolerance)."""
    from oracle.oracle import Oracle
    n = desc.n_dofs
    threads = max(1, min(16, os.cpu_count() or 1))
    nsub = min(desc.n_models, threads)
    sample = np.arange(0, desc.n_models, max(1, desc.n_models // nsub))[:nsub]
    sub = desc.subset(sample)
    idx = desc.dof_subset_index(sample)
    init = run["init"].cpu().numpy()
    t0 = time.perf_counter()
    ref, st = Oracle(sub, threads=threads).step_lm(K, init[:n][idx], init[n:][idx], wl.step.dt, tol=wl.step.tol,
                                                  max_iter=wl.step.max_iter)
    el = time.perf_counter() - t0
    got = run["traj"][0].cpu().numpy()[:, idx]
    return {"value": sub.n_links / el, "unit": "link-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the first timed step of {nsub} of {desc.n_models} models ({sub.n_links} links) from the "
                      f"timed launch's starting state, Levenberg-Marquardt with dense Jacobians, float64, {el:.1f} s",
            "converged_fraction": float(np.mean(st["flag"] == 1)),
            "iterations_per_step": float(st["iterations"].mean()),
            "max_abs_q_diff_vs_gpu": float(np.max(np.abs(got - ref)))}


def eq_lm_cpu_baseline(desc, wl, run, warmup):
    """The oracle's order-2 Levenberg-Marquardt step (H_q from its pose derivatives,
    dense Cholesky) on a bounded sample: the first timed step of a few models from
    the GPU's starting state, and the largest distance of the GPU's result from the
    oracle's on them (both solved to the workload's tolerance)."""
    from oracle.oracle import Oracle
    n = desc.n_dofs
    threads = 1  # the oracle's LM runs its dense algebra in numpy, model by model
    nsub = min(desc.n_models, 64)
    sample = np.arange(0, desc.n_models, max(1, desc.n_models // nsub))[:nsub]
    sub = desc.subset(sample)
    idx = desc.dof_subset_index(sample)
    init = run["init"].cpu().numpy()
    t0 = time.perf_counter()
    tau = None if wl.torque is None else wl.torque[warmup][idx]
    ref, st = Oracle(sub, threads=threads).step_lm_eq(init[:n][idx], init[n:][idx], wl.step.dt, tau,
                                                      tol=wl.step.tol, max_iter=wl.step.max_iter)
    el = time.perf_counter() - t0
    got = run["traj"][0].cpu().numpy()[idx]
    gst = run["st"][0][sample]
    return {"value": sub.n_links / el, "unit": "link-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the first timed step of {nsub} of {desc.n_models} models ({sub.n_links} links) from the "
                      f"timed launch's starting state, Levenberg-Marquardt with dense H_q, float64, {el:.1f} s",
            "converged_fraction": float(np.mean(st["flag"] == 1)),
            "iterations_per_step": float(st["iterations"].mean()),
            "iterations_equal_gpu_fraction": float(np.mean(st["iterations"] == gst["iterations"])),
            "max_abs_q_diff_vs_gpu": float(np.max(np.abs(got - ref)))}


if __name__ == "__main__":
    main()
