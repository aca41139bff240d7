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
COUNTERS = os.path.join(ROOT, "profiles", "col_deriv_512sq_256cube_fp32_fetch_write_counters.md")


# The sources that define the kernels and their launch geometry; host-side sequencing
# (problem.hpp, the ABI) does not change what one dispatch reads and writes.
KERNEL_SOURCES = ("common.hpp", "kernels.hpp", "kernels_wave.hpp", "spectral.hpp", "wave_fft.hpp")


def source_digest() -> str:
    """SHA-256 over the kernel sources; counter readings are only valid for the code they measured."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1408_6299_amd", "csrc")
    for fn in KERNEL_SOURCES:
        h.update(fn.encode())
        h.update(open(os.path.join(d, fn), "rb").read())
    return h.hexdigest()


def measured_traffic(symbol: str):
    """L2-to-fabric bytes (FETCH_SIZE + WRITE_SIZE, calibrated) per launch of `symbol` from the
    committed counter summary, or None when the
    summary is missing, covers another kernel, or was taken on different sources."""
    try:
        text = open(COUNTERS).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    k = rec.get("kernels", {}).get(symbol)
    return None if k is None else k["traffic_bytes_per_launch"]


def sleep_cycles_for(ms: float, torch) -> int:
    """Cycles of torch's device spin kernel that take about `ms` milliseconds."""
    cyc = 1_000_000
    torch.cuda._sleep(cyc)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.cuda._sleep(cyc)
    e1.record()
    torch.cuda.synchronize()
    return max(1, int(cyc * ms / max(e0.elapsed_time(e1), 1e-3)))


def kernel_pass(G, kernel, vt, out, reps, torch, cap=4096):
    """Times every launch of `kernel` in `reps` eager matvecs. Each matvec's launches are
    queued behind a device spin of a few milliseconds, so they run back to back as in a
    graph replay instead of trickling in at the host's launch rate."""
    cyc = sleep_cycles_for(8.0, torch)
    G.timer_arm(kernel, capacity=cap)
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.cuda._sleep(cyc)
        G.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    launches, avg_ms, bytes_per = G.timer_read()
    return {"name": kernel, "launches": launches, "avg_us": 1e3 * avg_ms, "bytes_per_launch": bytes_per,
            "matvecs": reps, "seconds": secs}


def symbol_of(kernel: str, launch: dict) -> str:
    """Kernel symbol of a timed kernel, as rocprof names it (column passes: the variant the
    handle's autotuner chose, from its description; the first axis's symbol in 3D)."""
    if kernel == "col_deriv":
        return launch["col_deriv_symbols"][0]
    return kernel


def matvec_roofline(G, vt, ms_per_matvec: float) -> dict:
    """The whole matvec against the HBM roofline: algorithmic bytes of all its launches
    (the library's tally) over the graph-replayed matvec time."""
    b, launches = G.matvec_bytes(vt)
    ach = b / (ms_per_matvec * 1e-3) / 1e9
    return {"bound": "hbm", "bytes_per_matvec": b, "launches": launches, "matvec_ms": ms_per_matvec,
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}


def time_matvecs(G, vt, reps, torch) -> float:
    """Milliseconds per graph-replayed Hessian matvec (one warm-up replay)."""
    out = G.empty_v()
    G.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def roofline(kernel: str, symbol: str, rec: dict, traffic=None) -> dict:
    ach = rec["bytes_per_launch"] / (rec["avg_us"] * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": kernel, "symbol": symbol, "launches": rec["launches"], "matvecs": rec["matvecs"],
            "avg_us": rec["avg_us"], "bytes_per_launch": rec["bytes_per_launch"],
            "timing": "HIP events stamped by each dispatch (hipExtLaunchKernelGGL) over eager matvecs of the "
                      "same workload, each queued behind a device spin so its launches run back to back",
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_counts": "bytes per launch between the L2 caches and the memory fabric (rocprofv3 FETCH_SIZE + "
                              "WRITE_SIZE, scaled by a plain device copy); the Infinity Cache is on the fabric side, "
                              "so this bounds the HBM bytes from above"}


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it), from /proc/cpuinfo."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


# Column pass of each counter workload: the autotuner's choice on the GPU (per-column at
# 512^2, tiled at 256^3), fixed here so a counter run never captures or times a graph.
COUNTER_COLUMN_PASS = {"c2lit": "8", "c4": "tiled"}


def counter_pass(nk, synth, torch, name: str) -> int:
    """Three eager FP32 matvecs of one workload, launched one kernel at a time, for the
    FETCH_SIZE / WRITE_SIZE runs. The column pass is pinned (NKREG_COL_E, before the first
    handle exists) so the autotuner never runs, and the handle never captures or replays a
    HIP graph: a counter-collection run once ended in a host segmentation fault at the
    point where the autotuner captures and event-times its column-pass graphs."""
    os.environ["NKREG_COL_E"] = os.environ.get("NKREG_COL_E") or COUNTER_COLUMN_PASS[name]
    os.environ["NKREG_NO_GRAPHS"] = "1"
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS[name]
    stokes = name == "c4"
    mT, vstar = synth.make_inputs(spec)
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, stokes, spec.beta, precision=32,
                   checkpoint_every=spec.checkpoint_every)
    G.use_graphs(False)
    mTd = torch.from_numpy(mT).to(dev).to(torch.float32)
    G.set_images(mTd, mTd)
    mR = G.forward(torch.from_numpy(vstar).to(dev))
    G.set_images(mTd, mR)
    G.objective_gradient(G.zeros_v())
    w = torch.from_numpy(synth.bandlimited_velocity(spec.shape, 52, 6, 0.05, divfree=stokes)).to(dev)
    out = G.empty_v()
    for _ in range(3):
        G.hessian_matvec(w, out)
    torch.cuda.synchronize()
    print(json.dumps({"workload": name, "matvecs": 3, "launch": G.describe()}), flush=True)
    G.close()
    return 0


def batch_section(nk, synth, torch, reps):
    """64 independent 2D pairs of uneven grid sizes (64^2..512^2), H1, beta 1e-2, nt = 16:
    one graph-captured batched matvec (items of one grid size share every kernel launch)
    versus the same items one after another (each a graph replay of its own), and the
    FP64 batch."""
    dev = torch.device("cuda:0")
    specs = synth.batch_specs()
    inputs = []
    for i, sp in enumerate(specs):
        mT, vstar = synth.make_inputs(sp)
        gen = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=64)
        gen.set_images(torch.from_numpy(mT).to(dev), torch.zeros(sp.shape, dtype=torch.float64, device=dev))
        mR = gen.forward(torch.from_numpy(vstar).to(dev)).cpu().numpy()
        gen.close()
        w = synth.bandlimited_velocity(sp.shape, 500 + i, 6, 0.05)
        inputs.append((sp, mT, mR, w))
    out = {"items": len(specs), "grids": {str(n): sum(1 for s in specs if s.shape[0] == n) for n in (64, 128, 256, 512)},
           "nt": specs[0].nt}
    pts = sum(int(np.prod(sp.shape)) for sp in specs)
    for prec in (32, 64):
        dt = torch.float32 if prec == 32 else torch.float64
        probs, ws, outs = [], [], []
        for sp, mT, mR, w in inputs:
            G = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=prec)
            G.set_images(torch.from_numpy(mT).to(dev).to(dt), torch.from_numpy(mR).to(dev).to(dt))
            G.objective_gradient(G.zeros_v())
            probs.append(G)
            ws.append(torch.from_numpy(w).to(dev))
            outs.append(G.empty_v())
        B = nk.Batch(probs)
        for _ in range(2):
            B.hessian_matvec(ws, outs)
        torch.cuda.synchronize()
        out["groups"] = [{"items": n, "form": f} for n, f in B.group_plan()]
        t0 = time.perf_counter()
        for _ in range(reps):
            B.hessian_matvec(ws, outs)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        r = {"batched_ms": 1e3 * tb, "item_matvecs_per_s": len(specs) / tb, "mpoints_per_s": pts * 1e-6 / tb}
        # the whole batch against the HBM roofline: the items' algorithmic bytes over the batch time
        nbytes = sum(G.matvec_bytes(w)[0] for G, w in zip(probs, ws))
        ach = nbytes / tb / 1e9
        r["roofline"] = {"bound": "hbm", "bytes_per_batched_matvec": nbytes, "achieved": ach, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
        if prec == 32:
            for G, w, o in zip(probs, ws, outs):
                G.hessian_matvec(w, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                for G, w, o in zip(probs, ws, outs):
                    G.hessian_matvec(w, o)
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t0) / reps
            r["sequential_ms"] = 1e3 * ts
            r["batched_speedup_vs_sequential"] = ts / tb
        # every item's objective and gradient (state and adjoint sweeps) as one graph launch
        vz = [G.zeros_v() for G in probs]
        gs = [G.empty_v() for G in probs]
        B.objective_gradient(vz, gs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.objective_gradient(vz, gs)
        torch.cuda.synchronize()
        r["batched_gradient_ms"] = 1e3 * (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for G, v, g in zip(probs, vz, gs):
            G.objective_gradient(v, g)
        torch.cuda.synchronize()
        r["sequential_gradient_ms"] = 1e3 * (time.perf_counter() - t0)
        # PCG on every item (rhs = -g at v = 0, relative tolerance 1e-2) in lockstep, one
        # batched matvec per iteration, against each item's own PCG one after another
        rhs = [-g for g in gs]
        xs = [G.empty_v() for G in probs]
        B.pcg(rhs, 1e-2, 0, xs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, _, _ = B.pcg(rhs, 1e-2, 0, xs)
        r["batched_pcg_ms"] = 1e3 * (time.perf_counter() - t0)
        r["pcg_iterations"] = [min(its), max(its), int(sum(its))]
        t0 = time.perf_counter()
        for G, b, x in zip(probs, rhs, xs):
            G.pcg(b, 1e-2, 0, x)
        torch.cuda.synchronize()
        r["sequential_pcg_ms"] = 1e3 * (time.perf_counter() - t0)
        out[f"fp{prec}"] = r
        log(f"batch FP{prec}: {r['batched_ms']:.3f} ms per batched matvec ({r['item_matvecs_per_s']:.0f} item-matvecs/s, "
            f"{ach / 1e3:.2f} TB/s)" + (f", sequential {r['sequential_ms']:.3f} ms" if prec == 32 else "")
            + f"; gradient {r['batched_gradient_ms']:.3f} ms batched, {r['sequential_gradient_ms']:.3f} ms one after another"
            + f"; PCG to 1e-2 ({r['pcg_iterations'][0]}-{r['pcg_iterations'][1]} iterations) "
              f"{r['batched_pcg_ms']:.1f} ms batched, {r['sequential_pcg_ms']:.1f} ms one after another")
        B.close()
        for G in probs:
            G.close()
    out["fp32_batched_speedup_vs_fp64_batched"] = out["fp64"]["batched_ms"] / out["fp32"]["batched_ms"]
    return out


def cube_section(nk, synth, torch, reps, kernel, precisions=(32, 64)):
    """256^3, nt = 32, H2 + Stokes, beta 1e-3, stationary divergence-free velocity at CFL 0.1,
    trajectory checkpointed every 8 steps: Hessian matvec time, FP32 and FP64."""
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS["c4"]
    shape, nt = spec.shape, spec.nt
    mT, vstar = synth.make_inputs(spec)
    w = synth.bandlimited_velocity(shape, 52, 6, 0.05, divfree=True)
    gen = nk.Problem(shape, nt, 1, spec.reg, True, spec.beta, precision=64, checkpoint_every=spec.checkpoint_every)
    gen.set_images(torch.from_numpy(mT).to(dev), torch.zeros(shape, dtype=torch.float64, device=dev))
    mR = gen.forward(torch.from_numpy(vstar).to(dev))
    gen.close()
    out = {"grid": list(shape), "nt": nt, "checkpoint_every": spec.checkpoint_every}
    for prec in precisions:
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(shape, nt, 1, spec.reg, True, spec.beta, precision=prec, checkpoint_every=spec.checkpoint_every)
        G.set_images(torch.from_numpy(mT).to(dev).to(dt), mR.to(dt))
        G.objective_gradient(G.zeros_v())
        wt = torch.from_numpy(w).to(dev)
        o = G.empty_v()
        G.hessian_matvec(wt, o)
        torch.cuda.synchronize()
        n = reps if prec == 32 else max(1, reps // 2)
        t0 = time.perf_counter()
        for _ in range(n):
            G.hessian_matvec(wt, o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / n
        out[f"fp{prec}"] = {"matvec_ms": 1e3 * t, "matvecs_per_s": 1.0 / t}
        log(f"256^3 FP{prec}: {1e3 * t:.1f} ms per matvec")
        out[f"fp{prec}"]["matvec_roofline"] = matvec_roofline(G, wt, 1e3 * t)
        if prec == 32:
            k = kernel_pass(G, kernel, wt, o, 1, torch)
            if k["launches"]:
                sym = symbol_of(kernel, G.describe())
                out["roofline"] = roofline(kernel, sym, k, measured_traffic(sym))
            ref = o.clone()
        G.close()
        if prec == 32:
            out["fp32"]["trajectory_slots"] = slots_sweep(nk, spec, mT, mR, wt, ref, reps, torch)
    if "fp64" in out:
        out["fp32_speedup"] = out["fp64"]["matvec_ms"] / out["fp32"]["matvec_ms"]
    return out


def slots_sweep(nk, spec, mT, mR, wt, ref, reps, torch, slots=(2, 4)):
    """FP32 matvec time with more K-step trajectory segments kept in memory (the default
    keeps one); every setting must reproduce the one-slot matvec bit for bit."""
    dev = torch.device("cuda:0")
    shape, nt, K = spec.shape, spec.nt, spec.checkpoint_every
    field = 4 * int(np.prod(shape))
    res = []
    for S in slots:
        G = nk.Problem(shape, nt, 1, spec.reg, True, spec.beta, precision=32, checkpoint_every=K,
                       trajectory_slots=S)
        G.set_images(torch.from_numpy(mT).to(dev).to(torch.float32), mR.to(torch.float32))
        G.objective_gradient(G.zeros_v())
        o = G.empty_v()
        G.hessian_matvec(wt, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.hessian_matvec(wt, o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        nseg = -(-nt // K)
        res.append({"slots": S, "matvec_ms": 1e3 * t, "segment_recomputes_per_matvec": 2 * max(0, nseg - S),
                    "trajectory_gib": 2 * min(S, nseg) * K * len(shape) * field / 2**30,
                    "bit_identical": bool(torch.equal(o, ref))})
        log(f"256^3 FP32, {S} trajectory slots: {1e3 * t:.1f} ms per matvec, "
            f"bit-identical {res[-1]['bit_identical']}")
        G.close()
    return res


def beta_search_section(nk, synth, torch, precisions=(32, 64)):
    """Parameter continuation in beta with a lower bound on det F_1 (decade descent from
    beta = 1, then bisection), 256^2, H1, nt = 64: time to beta*, FP32 and FP64."""
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS["c2beta"]
    shape, nt, eps = spec.shape, spec.nt, spec.extra["eps_F"]
    mT, vstar = synth.make_inputs(spec)
    gen = nk.Problem(shape, nt, 1, spec.reg, False, 1.0, precision=64)
    gen.set_images(torch.from_numpy(mT).to(dev), torch.zeros(shape, dtype=torch.float64, device=dev))
    mR = gen.forward(torch.from_numpy(vstar).to(dev))
    _, st = gen.det_grad_y(torch.from_numpy(vstar).to(dev))
    gen.close()
    out = {"grid": list(shape), "nt": nt, "reg": "H1", "eps_F": eps, "min_det_of_true_velocity": st[0]}
    for prec in precisions:
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(shape, nt, 1, spec.reg, False, 1.0, precision=prec)
        G.set_images(torch.from_numpy(mT).to(dev).to(dt), mR.to(dt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v, res = G.beta_search(eps, gtol=1e-3, max_outer=50)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out[f"fp{prec}"] = {"seconds": secs, "steps": res.steps, "beta_star": res.beta_star,
                            "min_det_star": res.min_det_star, "l2_rel_star": res.l2_rel_star,
                            "dbeta_min": res.dbeta_min, "reason": res.reason,
                            "newton_iterations": res.newton_iterations, "matvecs": res.cg_iterations,
                            "trials": [[t.beta, t.min_det, t.accepted] for t in res.trials]}
        log(f"beta search FP{prec}: {secs:.2f} s, {res.steps} solves, beta* = {res.beta_star:.5g}, "
            f"min det F_1 = {res.min_det_star:.4f}, {res.cg_iterations} matvecs")
        G.close()
    return out


def solver_section(nk, torch, spec, mT_h, mR_h, precisions=(32, 64), beta=1e-2):
    """GN-PCG against the globalised Picard iteration (preconditioned gradient descent with
    the step-scale memory) on the headline grid at one beta, from v = 0 to a relative
    gradient of 1e-3: wall time, outer iterations and hyperbolic PDE solves."""
    dev = torch.device("cuda:0")
    out = {"beta": beta, "gtol": 1e-3}
    for prec in precisions:
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, beta, precision=prec)
        G.set_images(torch.from_numpy(mT_h).to(dev).to(dt), torch.from_numpy(mR_h).to(dev).to(dt))
        r = {}
        for name, run in (("gn_pcg", lambda: G.newton_solve(G.zeros_v(), gtol=1e-3, max_outer=50)),
                          ("picard", lambda: G.picard_solve(G.zeros_v(), gtol=1e-3, max_outer=2000)),
                          ("picard_no_stagnation_stop",
                           lambda: G.picard_solve(G.zeros_v(), gtol=1e-3, max_outer=2000, stagnation=(0, 0.0)))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = run()
            torch.cuda.synchronize()
            r[name] = {"seconds": time.perf_counter() - t0, "outer_iterations": rep.iterations,
                       "matvecs": rep.cg_iterations, "n_pde": rep.n_pde, "converged": rep.converged,
                       "grad_rel": rep.gnorm_inf / rep.gnorm0_inf if rep.gnorm0_inf else 0.0}
        log(f"FP{prec} beta={beta}: GN-PCG {r['gn_pcg']['seconds']:.3f} s ({r['gn_pcg']['n_pde']} PDE solves), "
            f"Picard {r['picard']['seconds']:.3f} s ({r['picard']['n_pde']} PDE solves, "
            f"{r['picard']['outer_iterations']} iterations, stops on stagnation at |g|/|g0| = "
            f"{r['picard']['grad_rel']:.2e}); to the gradient tolerance: "
            f"{r['picard_no_stagnation_stop']['seconds']:.3f} s, {r['picard_no_stagnation_stop']['n_pde']} PDE "
            f"solves, converged {r['picard_no_stagnation_stop']['converged']}")
        out[f"fp{prec}"] = r
        G.close()
    return out


def analysis_section(nk, synth, torch, spec, mT_h, mR_h):
    """Hessian analysis: the dense 64^2 Hessian (n = 8192) by unit-vector matvecs, and a
    100-step Lanczos estimate of the extreme eigenvalues and condition number of the
    headline Hessian (FP32 transport) at v = 0."""
    dev = torch.device("cuda:0")
    out = {}
    shape, nt = (64, 64), 8
    mT = synth.smooth_image(shape, 5, 0.6 * 64 ** 2 / 16)
    vstar = synth.bandlimited_velocity(shape, 77, 4, synth.cfl_literal_linf(64, nt), norm="linf")
    G = nk.Problem(shape, nt, 1, 2, False, 1e-3, precision=64)
    G.set_images(torch.from_numpy(mT).to(dev), torch.from_numpy(mT).to(dev))
    G.objective_gradient(torch.from_numpy(vstar).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = G.hessian_matrix()
    torch.cuda.synchronize()
    out["assemble_64sq"] = {"n": int(H.shape[0]), "seconds": time.perf_counter() - t0,
                            "sweeps": G.describe().get("assembly_sweeps")}
    del H
    G.close()
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=32)
    G.set_images(torch.from_numpy(mT_h).to(dev).float(), torch.from_numpy(mR_h).to(dev).float())
    G.objective_gradient(G.zeros_v())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ritz = G.lanczos(100)
    secs = time.perf_counter() - t0
    out["lanczos_headline"] = {"steps": len(ritz), "seconds": secs, "ritz_min": ritz[0], "ritz_max": ritz[-1],
                               "condition_estimate": ritz[-1] / ritz[0] if ritz[0] > 0 else None}
    log(f"Hessian analysis: 64^2 assembly ({out['assemble_64sq']['n']} matvecs) "
        f"{out['assemble_64sq']['seconds']:.2f} s ({out['assemble_64sq']['sweeps']}); Lanczos(100) at 512^2 {secs:.2f} s, "
        f"Ritz values [{ritz[0]:.4g}, {ritz[-1]:.4g}]")
    G.close()
    return out


def reference_image(nk, torch, spec, mT, vstar, precision=64):
    """m_R = m_T transported by v* with the library's FP64 forward solve (input synthesis)."""
    dev = torch.device("cuda:0")
    G = nk.Problem(spec.shape, spec.nt, spec.nc, spec.reg, bool(spec.gamma), spec.beta, precision=64,
                   checkpoint_every=spec.checkpoint_every)
    G.set_images(torch.from_numpy(mT).to(dev), torch.zeros(spec.shape, dtype=torch.float64, device=dev))
    mR = G.forward(torch.from_numpy(vstar).to(dev))
    torch.cuda.synchronize()
    G.close()
    return mR


def timed_solve(G, torch, **kw):
    """Newton solve from v = 0; returns (seconds, report, v)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v, rep = G.newton_solve(G.zeros_v(), **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, rep, v


def solve_record(secs, rep, mis=None):
    r = {"seconds": secs, "outer_iterations": rep.iterations, "matvecs": rep.cg_iterations, "n_pde": rep.n_pde,
         "converged": rep.converged, "stop": rep.stop_reason,
         "grad_rel": rep.gnorm_inf / rep.gnorm0_inf if rep.gnorm0_inf else 0.0}
    if mis is not None:
        r["relative_mismatch"] = mis
    return r


def c0_section(nk, synth, torch, reps=20):
    """64^2 FP64, H1, beta 1e-2, nt = 16 (the paper's smooth test case at its size): GN-PCG
    time-to-solution to a relative gradient of 1e-3, and the graph-replayed matvec rate."""
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS["c0"]
    mT, vstar = synth.make_inputs(spec)
    mR = reference_image(nk, torch, spec, mT, vstar)
    G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta, precision=64)
    G.set_images(torch.from_numpy(mT).to(dev), mR)
    secs, rep, v = timed_solve(G, torch, gtol=1e-3, max_outer=50)
    mis = 2.0 * rep.J_dist / (G.hd * float(np.sum((mR.cpu().numpy() - mT) ** 2)))
    out = {"grid": list(spec.shape), "nt": spec.nt, "precision": 64, "solve": solve_record(secs, rep, mis)}
    G.objective_gradient(G.zeros_v())
    w = torch.from_numpy(synth.bandlimited_velocity(spec.shape, 31, 4, 0.3)).to(dev)
    ms = time_matvecs(G, w, reps, torch)
    out["matvec_ms"] = ms
    out["matvecs_per_s"] = 1e3 / ms
    out["matvec_roofline"] = matvec_roofline(G, w, ms)
    d = G.describe()
    out["sweeps"] = {"persistent": d.get("persistent_sweeps"), "timing": d.get("sweep_timing")}
    log(f"c0 64^2 FP64: solve {secs:.3f} s ({rep.iterations} outer / {rep.cg_iterations} matvecs), "
        f"matvec {ms:.3f} ms; sweeps: {out['sweeps']}")
    G.close()
    return out


def c1_section(nk, synth, torch, precisions=(32, 64), reps=3):
    """256^2, three Chebyshev coefficients per component, H2 + Stokes, beta 1e-3, nt = 408
    (the CFL-adapted steps of the 32-step configuration): FP32 against FP64 matvec time and
    time-to-solution (relative gradient 1e-3), and det F_1 of each solution (FP64)."""
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS["c1"]
    mT, vstar = synth.make_inputs(spec)
    mR = reference_image(nk, torch, spec, mT, vstar)
    out = {"grid": list(spec.shape), "nt": spec.nt, "nc": spec.nc, "reg": "H2", "incompressible": True,
           "beta": spec.beta}
    _, st = nk.Problem(spec.shape, spec.nt, spec.nc, spec.reg, True, spec.beta, precision=64).det_grad_y(
        torch.from_numpy(vstar).to(dev))
    out["det_F1_true_velocity"] = {"min": st[0], "max": st[1]}
    w = torch.from_numpy(synth.bandlimited_velocity(spec.shape, 30, 8, 0.1, divfree=True, nc=3)).to(dev)
    mis0 = float(np.sum((mR.cpu().numpy() - mT) ** 2))
    for prec in precisions:
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(spec.shape, spec.nt, spec.nc, spec.reg, True, spec.beta, precision=prec)
        G.set_images(torch.from_numpy(mT).to(dev).to(dt), mR.to(dt))
        G.objective_gradient(G.zeros_v())
        ms = time_matvecs(G, w, reps, torch)
        r = {"matvec_ms": ms, "matvecs_per_s": 1e3 / ms, "matvec_roofline": matvec_roofline(G, w, ms)}
        secs, rep, v = timed_solve(G, torch, gtol=1e-3, max_outer=50)
        r["solve"] = solve_record(secs, rep, 2.0 * rep.J_dist / (G.hd * mis0))
        _, st = G.det_grad_y(v)
        r["det_F1"] = {"min": st[0], "max": st[1], "mean": st[2], "std": st[3]}
        out[f"fp{prec}"] = r
        log(f"c1 256^2 nt=408 FP{prec}: matvec {ms:.2f} ms, solve {secs:.2f} s ({rep.iterations} outer / "
            f"{rep.cg_iterations} matvecs), det F_1 in [{st[0]:.4f}, {st[1]:.4f}]")
        G.close()
    if 32 in precisions and 64 in precisions:
        out["fp32_matvec_speedup"] = out["fp64"]["matvec_ms"] / out["fp32"]["matvec_ms"]
        out["fp32_solve_speedup"] = out["fp64"]["solve"]["seconds"] / out["fp32"]["solve"]["seconds"]
    return out


def c2_full_section(nk, synth, torch, precisions=(32, 64), reps=3, max_outer=5):
    """512^2, H2, nt = 1224 (the CFL-adapted steps at max|v*| = 1.5), beta continuation
    1e-1 -> 1e-4 with the paper's termination rule of its 512^2 continuation runs
    ((C1 and C2 and C3) or C4 or C5, tau_J = 1e-3; at most max_outer + 1 iterations per
    level): time-to-solution and matvec time. (The relative-gradient rule at 1e-3 is not
    reached within 50 iterations here: at 1224 FP32 steps the gradient's round-off floor
    lies above it.)"""
    dev = torch.device("cuda:0")
    spec = synth.CONFIGS["c2"]
    mT, vstar = synth.make_inputs(spec)
    mR = reference_image(nk, torch, spec, mT, vstar)
    mis0 = float(np.sum((mR.cpu().numpy() - mT) ** 2))
    out = {"grid": list(spec.shape), "nt": spec.nt, "beta_levels": list(spec.beta_levels)}
    for prec in precisions:
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(spec.shape, spec.nt, 1, spec.reg, False, spec.beta_levels[0], precision=prec)
        G.set_images(torch.from_numpy(mT).to(dev).to(dt), mR.to(dt))
        # the continuation level by level (as nkreg_continuation runs it: every level's
        # relative-gradient rule against the first level's gradient), one line per level
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v, levels = G.zeros_v(), []
        for b in spec.beta_levels:
            G.beta = b
            v, rep = G.newton_solve(v, gtol=0.0, tau_J=1e-3, max_outer=max_outer)
            levels.append(rep)
            log(f"c2 FP{prec} beta={b:g}: {rep.iterations} outer / {rep.cg_iterations} matvecs, stop "
                f"{rep.stop_reason}, {time.perf_counter() - t0:.1f} s so far")
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        G.beta = spec.beta
        G.objective_gradient(G.zeros_v())
        w = torch.from_numpy(synth.bandlimited_velocity(spec.shape, 20, 16, 0.05)).to(dev)
        ms = time_matvecs(G, w, reps, torch)
        r = {"seconds": secs, "rule": "C1-C5, tau_J = 1e-3", "stops": [x.stop_reason for x in levels],
             "outer_iterations": sum(x.iterations for x in levels),
             "matvecs": sum(x.cg_iterations for x in levels), "n_pde": sum(x.n_pde for x in levels),
             "converged": all(x.converged for x in levels),
             "relative_mismatch": 2.0 * levels[-1].J_dist / (G.hd * mis0),
             "matvec_ms": ms, "matvecs_per_s": 1e3 / ms, "matvec_roofline": matvec_roofline(G, w, ms)}
        out[f"fp{prec}"] = r
        log(f"c2 512^2 nt=1224 FP{prec}: continuation {secs:.2f} s ({r['outer_iterations']} outer / "
            f"{r['matvecs']} matvecs), matvec {ms:.1f} ms")
        G.close()
    if 32 in precisions and 64 in precisions:
        out["fp32_solve_speedup"] = out["fp64"]["seconds"] / out["fp32"]["seconds"]
    return out


def c4_full_section(nk, synth, torch, precisions=(32, 64)):
    """256^3, H2 + Stokes, nt = 408 (the CFL-adapted steps at max|v*| = 1), checkpoint
    every 8 steps (51 segments): gradient and matvec time, det F_1 of the true velocity."""
    dev = torch.device("cuda:0")
    base = synth.CONFIGS["c4"]
    shape = base.shape
    nt = synth.cfl_steps(1.0, shape[0], 0.1, 8)
    vstar = synth.bandlimited_velocity(shape, base.vel_seed, base.vel_kmax, 1.0, divfree=True)
    mT = synth.smooth_image(shape, base.image_seed, base.image_width)
    out = {"grid": list(shape), "nt": nt, "checkpoint_every": base.checkpoint_every,
           "segments": -(-nt // base.checkpoint_every)}
    G64 = nk.Problem(shape, nt, 1, base.reg, True, base.beta, precision=64, checkpoint_every=base.checkpoint_every)
    G64.set_images(torch.from_numpy(mT).to(dev), torch.zeros(shape, dtype=torch.float64, device=dev))
    mR = G64.forward(torch.from_numpy(vstar).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = G64.det_grad_y(torch.from_numpy(vstar).to(dev))
    out["det_F1_true_velocity"] = {"min": st[0], "max": st[1], "mean": st[2], "std": st[3],
                                   "seconds": time.perf_counter() - t0}
    G64.close()
    w = torch.from_numpy(synth.bandlimited_velocity(shape, 52, 6, 0.05, divfree=True)).to(dev)
    for prec in precisions:
        dt = torch.float32 if prec == 32 else torch.float64
        G = nk.Problem(shape, nt, 1, base.reg, True, base.beta, precision=prec, checkpoint_every=base.checkpoint_every)
        G.set_images(torch.from_numpy(mT).to(dev).to(dt), mR.to(dt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.objective_gradient(G.zeros_v())
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        ms = time_matvecs(G, w, 1, torch)
        out[f"fp{prec}"] = {"gradient_s": tg, "matvec_ms": ms, "matvec_roofline": matvec_roofline(G, w, ms)}
        log(f"c4 256^3 nt={nt} FP{prec}: gradient {tg:.2f} s, matvec {ms:.0f} ms")
        G.close()
    if 32 in precisions and 64 in precisions:
        out["fp32_matvec_speedup"] = out["fp64"]["matvec_ms"] / out["fp32"]["matvec_ms"]
    return out


def batch_nteff_section(nk, synth, torch, reps=2):
    """The 64-pair batch at its own amplitudes: each item with the steps its CFL bound needs
    (rounded up to a multiple of 64, 64..640): one batched matvec against the items one after
    another, FP32."""
    dev = torch.device("cuda:0")
    specs = synth.batch_specs_nteff()
    probs, ws, outs = [], [], []
    for i, sp in enumerate(specs):
        mT, vstar = synth.make_inputs(sp)
        mR = reference_image(nk, torch, sp, mT, vstar)
        G = nk.Problem(sp.shape, sp.nt, 1, sp.reg, False, sp.beta, precision=32)
        G.set_images(torch.from_numpy(mT).to(dev).float(), mR.float())
        G.objective_gradient(G.zeros_v())
        probs.append(G)
        ws.append(torch.from_numpy(synth.bandlimited_velocity(sp.shape, 500 + i, 6, 0.05)).to(dev))
        outs.append(G.empty_v())
        if i % 16 == 15:
            log(f"batch at CFL steps: {i + 1} items set up")
    steps = sorted({(sp.shape[0], sp.nt) for sp in specs})
    out = {"items": len(specs), "nt_range": [min(sp.nt for sp in specs), max(sp.nt for sp in specs)],
           "grid_steps_pairs": len(steps)}
    B = nk.Batch(probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.hessian_matvec(ws, outs)
    torch.cuda.synchronize()
    out["build_and_first_s"] = time.perf_counter() - t0
    plan = B.group_plan()
    out["groups"] = len(plan)
    out["group_forms"] = {f: sum(1 for _, g in plan if g == f) for f in nk.Batch.GROUP_FORMS}
    log(f"batch at CFL steps: graph of {out['groups']} groups built and run in {out['build_and_first_s']:.1f} s; "
        f"forms {out['group_forms']}")
    t0 = time.perf_counter()
    for _ in range(reps):
        B.hessian_matvec(ws, outs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    for G, w, o in zip(probs, ws, outs):
        G.hessian_matvec(w, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for G, w, o in zip(probs, ws, outs):
        G.hessian_matvec(w, o)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    nbytes = sum(G.matvec_bytes(w)[0] for G, w in zip(probs, ws))
    ach = nbytes / tb / 1e9
    out.update({"batched_ms": 1e3 * tb, "sequential_ms": 1e3 * ts, "batched_speedup_vs_sequential": ts / tb,
                "roofline": {"bound": "hbm", "bytes_per_batched_matvec": nbytes, "achieved": ach,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}})
    log(f"batch at CFL steps ({out['nt_range'][0]}..{out['nt_range'][1]}, {out['groups']} groups): batched "
        f"{1e3 * tb:.1f} ms, sequential {1e3 * ts:.1f} ms, {ach / 1e3:.2f} TB/s")
    B.close()
    for G in probs:
        G.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel", default="col_deriv",
                    help="kernel whose launches are timed for the roofline (see Problem.KERNELS)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the Newton time-to-solution runs")
    ap.add_argument("--cpu-matvecs", type=int, default=16, help="oracle matvecs in the CPU sample")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 runs (headline and 256^3)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-pair batched workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--no-3d", action="store_true", help="skip the 256^3 workload")
    ap.add_argument("--no-beta-search", action="store_true", help="skip the det F_1-bounded beta search")
    ap.add_argument("--no-analysis", action="store_true", help="skip the Hessian assembly and Lanczos estimate")
    ap.add_argument("--c2-fp64", action="store_true",
                    help="also time the FP64 transport on the 512^2 nt = 1224 continuation (minutes)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (64^2 solve, 256^2 n_c = 3 Stokes at nt = 408, 512^2 at "
                         "nt = 1224, 256^3 at nt = 408, the batch at its CFL steps)")
    ap.add_argument("--counter-pass", choices=("c2lit", "c4"), default=None,
                    help="only run three eager FP32 Hessian matvecs of the workload (no graphs, no timers; for "
                         "HBM counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (got --gpus {args.gpus}).",
              file=sys.stderr)
        return 2

    import torch
    import synth
    import paper_1408_6299_amd as nk

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale the counters to bytes
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n, "launches": 3}), flush=True)
        return 0
    if args.counter_pass:
        return counter_pass(nk, synth, torch, args.counter_pass)
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
    for prec in ((32,) if args.no_fp64 else (32, 64)):
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
        r["matvec_roofline"] = matvec_roofline(G, rhs, time_matvecs(G, rhs, max(20, steps // 2), torch))
        if prec == 32:
            # second timed region, same workload: HIP events stamped by every launch of the
            # dominant kernel (the library launches eagerly while its timer is armed)
            r["kernel"] = kernel_pass(G, args.kernel, rhs, G.empty_v(), 20, torch)
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
            # the same with the full-Newton Hessian (e:second-order-opt-cond)
            G.hessian = "newton"
            _, _, _, gN = G.objective_gradient(G.zeros_v())
            rhsN = (-gN).contiguous()
            nsteps = max(10, steps // 2)
            timed_pcg_steps(G, rhsN, 3, torch)
            secsN = timed_pcg_steps(G, rhsN, nsteps, torch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vN, repsN = G.continuation(spec.beta_levels, G.zeros_v(), gtol=1e-3, max_outer=50)
            torch.cuda.synchronize()
            tN = time.perf_counter() - t0
            misN = 2.0 * repsN[-1].J_dist / (G.hd * float(np.sum((mR_h - mT_h) ** 2)))
            r["full_newton"] = {"matvecs_per_s": nsteps / secsN, "ms_per_step": 1e3 * secsN / nsteps,
                                "seconds": tN, "outer_iterations": sum(x.iterations for x in repsN),
                                "matvecs": sum(x.cg_iterations for x in repsN), "relative_mismatch": misN,
                                "converged": all(x.converged for x in repsN)}
            log(f"FP{prec}: full Newton {nsteps / secsN:.1f} matvecs/s; solve {tN:.3f} s, "
                f"{r['full_newton']['outer_iterations']} outer / {r['full_newton']['matvecs']} matvecs, "
                f"mismatch {misN:.3e}")
            G.hessian = "gn"
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
    }
    out["matvec_roofline"] = results[32]["matvec_roofline"]
    # the launch-latency floor of the same number of dependent launches (plain copies of the
    # row spectrum, row and column patterns alternating), against which the matvec is bound
    fl = {k: nk.launch_floor(k, shape[0], shape[1] // 2, 200) for k in ("empty", "row_column_alternating")}
    mv = out["matvec_roofline"]
    floor_ms = mv["launches"] * fl["row_column_alternating"] * 1e-3
    out["latency_floor"] = {"empty_node_us": fl["empty"], "copy_node_us": fl["row_column_alternating"],
                            "launches_per_matvec": mv["launches"], "floor_ms": floor_ms, "matvec_ms": mv["matvec_ms"],
                            "frac": floor_ms / mv["matvec_ms"],
                            "note": "graph of dependent launches, each copying the spectrum the previous one wrote"}
    log(f"latency floor: empty node {fl['empty']:.2f} us, copy node {fl['row_column_alternating']:.2f} us; "
        f"{mv['launches']} launches -> {floor_ms:.3f} ms against the {mv['matvec_ms']:.3f} ms matvec "
        f"({100 * floor_ms / mv['matvec_ms']:.0f}%)")
    if 64 in results:
        out["fp64"] = {"matvecs_per_s": results[64]["matvecs_per_s"], "ms_per_step": results[64]["ms_per_step"],
                       "fp32_speedup": results[32]["matvecs_per_s"] / results[64]["matvecs_per_s"],
                       "matvec_roofline": results[64]["matvec_roofline"]}
    if not args.no_solve:
        for prec in results:
            out[f"newton_fp{prec}"] = results[prec]["newton"]
            out[f"full_newton_fp{prec}"] = results[prec]["full_newton"]
    k = results[32]["kernel"]
    if k["launches"] > 0 and k["avg_us"] > 0:
        sym = symbol_of(k["name"], results[32]["launch"])
        out["roofline"] = roofline(k["name"], sym, k, measured_traffic(sym))
    if not args.no_batch:
        out["batch"] = batch_section(nk, synth, torch, reps=10)
    if not args.no_solve:
        out["solvers"] = solver_section(nk, torch, spec, mT_h, mR_h, (32,) if args.no_fp64 else (32, 64))
    if not args.no_analysis:
        out["hessian_analysis"] = analysis_section(nk, synth, torch, spec, mT_h, mR_h)
    if not args.no_beta_search:
        out["beta_search"] = beta_search_section(nk, synth, torch, (32,) if args.no_fp64 else (32, 64))
    if not args.no_3d:
        out["cube_256"] = cube_section(nk, synth, torch, reps=4, kernel=args.kernel,
                                       precisions=(32,) if args.no_fp64 else (32, 64))
    if not args.no_configs:
        configs = {}
        precs = (32,) if args.no_fp64 else (32, 64)
        configs["c0_64sq_fp64"] = c0_section(nk, synth, torch)
        configs["c1_256sq_nc3_stokes_nt408"] = c1_section(nk, synth, torch, precs)
        configs["c2_512sq_nt1224"] = c2_full_section(nk, synth, torch, (32, 64) if args.c2_fp64 else (32,))
        if not args.no_3d:
            configs["c4_256cube_nt408"] = c4_full_section(nk, synth, torch, precs)
        if not args.no_batch:
            configs["batch_cfl_steps"] = batch_nteff_section(nk, synth, torch)
        out["configs"] = configs
    if not args.no_cpu:
        from oracle import reduced as ord_
        from oracle import spectral as osp
        from oracle import transport as otr
        # the oracle's own reference image (its FP64 forward solve of the same velocity)
        mR_o = otr.forward_only(mT_h, vstar_h, nt)
        P = ord_.Problem(mT_h, mR_o, nt, 1, spec.reg, 0, spec.beta)
        S = ord_.objective_gradient(P, np.zeros(P.vshape()))
        w = -S.g
        n = max(1, args.cpu_matvecs)
        t0 = time.perf_counter()
        for _ in range(n):
            hw = ord_.hessian_matvec(P, S, w)
            z = ord_.precond(P, hw)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / tc, "unit": "matvecs/s", "cores": osp.WORKERS, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"{n} oracle GN Hessian matvecs + preconditioner applications "
                                         f"(FP64 NumPy/SciPy) at the 512^2 nt=32 state, {tc:.1f} s"}
        c2 = out.get("configs", {}).get("c2_512sq_nt1224", {}).get("fp32")
        if c2:
            # a matvec is two transport solves of nt steps; the oracle's cost grows linearly in nt
            per_pde = tc / n / 2.0 * (synth.CONFIGS["c2"].nt / nt)
            out["cpu_baseline"]["c2_512sq_nt1224_solve_extrapolated_s"] = c2["n_pde"] * per_pde
        log(f"CPU oracle: {n / tc:.3f} matvecs/s on {osp.WORKERS} threads ({cpu_model()})")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
