#!/usr/bin/env python
"""Gauss-Newton Hessian matvecs/s and Newton time-to-solution on one MI355X.

Workload: 2D 512x512, nt = 32 RK2 steps, H2 regulariser, beta = 1e-4 (after
continuation from 1e-1), stationary velocity, FP32 transport and FFTs with FP64
reductions; the reference image is the template transported by a seeded
band-limited velocity scaled to CFL 0.1 at nt = 32. One timed step is one
GN-PCG inner iteration at the first Newton iterate: Hessian matvec (incremental
state + incremental adjoint transport, body force, spectral finalize),
preconditioner, FP64 dot products and vector updates.

Prints one JSON line on stdout; progress goes to stderr.
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timed_pcg_steps(prob, rhs, steps, torch):
    """Run exactly `steps` PCG iterations (restarting if PCG stops early); return seconds."""
    done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < steps:
        _, it, _, _ = prob.pcg(rhs, 0.0, steps - done)
        if it == 0:
            raise RuntimeError("PCG made no progress")
        done += it
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kernel", default="col_deriv",
                    help="kernel whose launches are timed for the roofline (see Problem.KERNELS)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the Newton time-to-solution runs")
    ap.add_argument("--cpu-matvecs", type=int, default=16, help="oracle matvecs in the CPU sample")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (got --gpus {args.gpus}).",
              file=sys.stderr)
        return 2

    import torch
    import synth
    import paper_1408_6299_amd as nk

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS["c2lit"]
    shape, nt = spec.shape, spec.nt
    mT_h, vstar_h = synth.make_inputs(spec)
    log(f"workload {spec.name}; max|v*^i| = {np.abs(vstar_h).max():.4f}")

    def to(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev).to(dt).contiguous()

    # reference image: template transported by v* (FP64 solve in the library)
    gen = nk.Problem(shape, nt, 1, spec.reg, False, spec.beta, precision=64)
    zero64 = torch.zeros((shape[0], shape[1]), dtype=torch.float64, device=dev)
    gen.set_images(to(mT_h, torch.float64), zero64)
    mR64 = gen.forward(to(vstar_h, torch.float64))
    torch.cuda.synchronize()
    mR_h = mR64.cpu().numpy()
    gen.close()

    results = {}
    for prec in (32, 64):
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(shape, nt, 1, spec.reg, False, spec.beta, precision=prec)
        G.set_images(to(mT_h, dt), to(mR_h, dt))
        J, Jd, Jr, g = G.objective_gradient(G.zeros_v())
        rhs = (-g).contiguous()
        steps = args.steps if prec == 32 else max(10, args.steps // 4)
        timed_pcg_steps(G, rhs, args.warmup, torch)
        secs = timed_pcg_steps(G, rhs, steps, torch)   # matvecs replay their captured HIP graph
        r = {"steps": steps, "seconds": secs, "matvecs_per_s": steps / secs, "ms_per_step": 1e3 * secs / steps,
             "launch": G.describe()}
        if prec == 32:
            # second timed region, same workload: HIP events around every launch of the
            # dominant kernel (the library launches eagerly while its timer is armed)
            ksteps = max(5, steps // 4)
            G.timer_arm(args.kernel, capacity=512 * ksteps)
            ksecs = timed_pcg_steps(G, rhs, ksteps, torch)
            launches, avg_ms, bytes_per = G.timer_read()
            r["kernel"] = {"name": args.kernel, "launches": launches, "avg_us": 1e3 * avg_ms,
                           "bytes_per_launch": bytes_per, "eager_ms_per_step": 1e3 * ksecs / ksteps}
        log(f"FP{prec}: {r['matvecs_per_s']:.1f} matvecs/s ({r['ms_per_step']:.3f} ms per PCG iteration)")
        if not args.no_solve:
            # time-to-solution: beta continuation 1e-1 -> 1e-4, warm-started, relative gradient 1e-3
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v, reps = G.continuation(spec.beta_levels, G.zeros_v(), gtol=1e-3, max_outer=50)
            torch.cuda.synchronize()
            tsol = time.perf_counter() - t0
            rep = reps[-1]
            tot_cg = sum(x.cg_iterations for x in reps)
            tot_it = sum(x.iterations for x in reps)
            tot_pde = sum(x.n_pde for x in reps)
            mis = 2.0 * rep.J_dist / (G.hd * float(np.sum((mR_h - mT_h) ** 2)))
            r["newton"] = {"seconds": tsol, "outer_iterations": tot_it, "matvecs": tot_cg, "n_pde": tot_pde,
                           "levels": [{"beta": b, "outer": x.iterations, "matvecs": x.cg_iterations,
                                       "converged": x.converged} for b, x in zip(spec.beta_levels, reps)],
                           "relative_mismatch": mis, "converged": all(x.converged for x in reps),
                           "grad_rel": rep.gnorm_inf / reps[0].gnorm0_inf if reps[0].gnorm0_inf else 0.0}
            log(f"FP{prec}: Newton solve {tsol:.3f} s, {tot_it} outer / {tot_cg} matvecs, mismatch {mis:.3e}")
            G.beta = spec.beta
        results[prec] = r
        G.close()

    out = {
        "metric": "GN Hessian matvecs/s (512^2, nt=32, FP32 transport/FFT, FP64 reductions) + Newton solve time",
        "value": results[32]["matvecs_per_s"],
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": results[32]["steps"],
        "warmup": args.warmup,
        "ms_per_step": results[32]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded smooth image; reference = template transported by a seeded band-limited velocity)",
        "config": {"workload": spec.name, "grid": list(shape), "nt": nt, "nc": 1, "reg": "H2",
                   "beta": spec.beta, "incompressible": False, "step": "one GN-PCG iteration (matvec-dominated)"},
        "launch": results[32]["launch"],
        "fp64": {"matvecs_per_s": results[64]["matvecs_per_s"], "ms_per_step": results[64]["ms_per_step"],
                 "fp32_speedup": results[32]["matvecs_per_s"] / results[64]["matvecs_per_s"]},
    }
    if not args.no_solve:
        out["newton_fp32"] = results[32]["newton"]
        out["newton_fp64"] = results[64]["newton"]
    k = results[32]["kernel"]
    if k["launches"] > 0 and k["avg_us"] > 0:
        ach = k["bytes_per_launch"] / (k["avg_us"] * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": k["name"], "launches": k["launches"],
                           "avg_us": k["avg_us"], "bytes_per_launch": k["bytes_per_launch"],
                           "timing": "HIP events around each launch, eager pass of the same workload "
                                     f"({k['eager_ms_per_step']:.3f} ms per step without graph replay)",
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                           "traffic": None}
    if not args.no_cpu:
        from oracle import reduced as ord_
        from oracle import spectral as osp
        P = ord_.Problem(mT_h, mR_h, nt, 1, spec.reg, 0, spec.beta)
        S = ord_.objective_gradient(P, np.zeros(P.vshape()))
        w = -S.g
        n = max(1, args.cpu_matvecs)
        t0 = time.perf_counter()
        for _ in range(n):
            hw = ord_.hessian_matvec(P, S, w)
            z = ord_.precond(P, hw)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / tc, "unit": "matvecs/s", "cores": osp.WORKERS, "kind": "oracle",
                               "sample": f"{n} oracle GN Hessian matvecs + preconditioner applications "
                                         f"(FP64 NumPy/SciPy) at the same 512^2 nt=32 state, {tc:.1f} s"}
        log(f"CPU oracle: {n / tc:.3f} matvecs/s on {osp.WORKERS} threads")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
