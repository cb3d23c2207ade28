#!/usr/bin/env python3
"""Benchmark: batched airfoil solves/s on one MI355X.

One step = one pass of the panel-method hot path over the whole batch:
assembly (FP64) -> LU with partial pivoting + solve (FP64, or FP32 factors
with FP64 iterative refinement) -> surface speed / Cp / Cl reductions.
Inputs (NACA nodes from the library's geometry kernel, angles) are resident
in device memory before the timed region starts.

Prints ONE JSON line.  ``value`` is the FP64 solves/s on the GA-population
batch (2048 seeded NACA 4-digit airfoils, 256 panels, 257x257 systems);
the FP32+refinement rate, the adjoint rate, per-kernel times, the roofline
of the dominant kernel and the CPU oracle baseline ride along.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "airfoil solves/s at N=256 (FP64 vs FP32+refine) + Cl err vs FP64 oracle"
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "hbm": 8.0e12}

# FP64 operations per off-diagonal influence entry of the assembly kernel,
# counted from its compiled gfx950 code: one logarithm (27 FP64 instructions,
# 17 of them FMA), one arctangent (34, 15 FMA) and the closed-form
# combination; 39 FMA x 2 + 40 other FP64 instructions in total.
ASM_FLOPS_PER_ENTRY = 118.0

# HBM bytes moved by one launch of the FP64 LU kernel on the 2048 x N=256
# batch, from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a plain copy's
# readings (x2.0 and x1.0).  Valid only for the kernel source it was taken
# on, which is identified by the SHA-256 prefix of that source file.
LU_TRAFFIC = {("lu_wave.hip", "2e2fbcc78dbaeca4"): 10_219_450_864}   # one wavefront per airfoil


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ga2048",
                    help="seeded workload (synth.WORKLOADS; default: the GA-population batch)")
    ap.add_argument("--batch", type=int, default=None, help="truncate the batch (debugging only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="airfoils in the oracle sample (default: the whole batch)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--wave-limit", type=int, default=None,
                    help="largest system order for the one-wavefront LU (0 = workgroup LU only)")
    return ap.parse_args()


def _flops(w):
    n1 = w.n_panels.astype(np.float64) + 1
    K = np.array([len(a) for a in w.alpha], dtype=np.float64)
    lu = float(np.sum(2.0 / 3.0 * n1 ** 3))
    solve = float(np.sum(2.0 * n1 ** 2 * K))
    pairs = float(np.sum(w.n_panels.astype(np.float64) ** 2))
    return lu, solve, pairs


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import synth
    import paper_1511_02166_amd as P

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    P.load_library()   # fails loudly without the HIP library
    dev = torch.device("cuda")
    w = synth.workload(a.workload, B=a.batch)
    noff, aoff = w.node_offsets(), w.alpha_offsets()
    alpha = torch.as_tensor(w.alpha_flat(), device=dev)
    mpt = torch.as_tensor(w.mpt(), device=dev)

    s64 = P.PanelSolver(noff, aoff, P.PANEL_FP64, wave_limit=a.wave_limit)
    s32 = P.PanelSolver(noff, aoff, P.PANEL_FP32_REFINE, wave_limit=a.wave_limit)
    xy = s64.naca4(mpt, True)
    torch.cuda.synchronize()

    lu_f, solve_f, pairs = _flops(w)
    B = w.B
    n_solves = int(aoff[-1])

    def timed(solver, steps, warmup, tol=1e-10, max_iter=10):
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            solver.step(xy, alpha, refine_tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t_start.record(stream)
        for i in range(steps):
            e = ev[i]
            e[0].record(stream)
            solver.assemble(xy, alpha)
            e[1].record(stream)
            solver.factor_solve(tol, max_iter)
            e[2].record(stream)
            solver.forces(True)
            e[3].record(stream)
        t_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        total_ms = t_start.elapsed_time(t_end)
        asm = np.mean([e[0].elapsed_time(e[1]) for e in ev])
        fs = np.mean([e[1].elapsed_time(e[2]) for e in ev])
        fo = np.mean([e[2].elapsed_time(e[3]) for e in ev])
        return dict(ms_per_step=total_ms / steps, wall_ms_per_step=1e3 * wall / steps,
                    assemble_ms=float(asm), factor_solve_ms=float(fs), forces_ms=float(fo))

    r64 = timed(s64, a.steps, a.warmup)
    info64 = s64.info.cpu().numpy()
    cl64 = s64.cl.cpu().numpy()
    cp64 = s64.cp.cpu().numpy()
    r32 = timed(s32, a.steps, a.warmup)
    info32 = s32.info.cpu().numpy()
    cl32 = s32.cl.cpu().numpy()
    cp32 = s32.cp.cpu().numpy()
    iters32 = s32.refine_iterations()

    v64 = n_solves / (r64["ms_per_step"] * 1e-3)
    v32 = n_solves / (r32["ms_per_step"] * 1e-3)

    # adjoint (dCl/d nodes), timed on the FP64 factors
    adj = None
    if not a.no_adjoint:
        try:
            dcl = torch.ones(n_solves, dtype=torch.float64, device=dev)
            dxy = torch.empty_like(xy)
            s64.step(xy, alpha)
            for _ in range(a.warmup):
                s64.adjoint(xy, dcl, dxy)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(a.steps):
                s64.adjoint(xy, dcl, dxy)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / a.steps
            adj = {"gradients_per_s": B / (ms * 1e-3), "ms_per_step": ms,
                   "fwd_plus_bwd_per_s": B / ((ms + r64["ms_per_step"]) * 1e-3)}
        except P.PanelError as exc:
            adj = {"error": str(exc)}

    # roofline of the dominant kernel (FP64 path): LU+solve on the matrix
    # cores, or the transcendental-bound assembly on the vector ALUs.
    lu_ms = r64["factor_solve_ms"]
    asm_ms = r64["assemble_ms"]
    lu_ach = (lu_f + solve_f) / (lu_ms * 1e-3)
    asm_ach = pairs * ASM_FLOPS_PER_ENTRY / (asm_ms * 1e-3)
    kern = {
        "lu_solve_f64": {"bound": "mfma", "achieved": lu_ach / 1e12, "peak": PEAK["f64"] / 1e12,
                         "unit": "TFLOP/s", "frac": lu_ach / PEAK["f64"], "ms": lu_ms,
                         "work": "(2/3)n^3 + 2n^2K flops per airfoil"},
        "assemble_f64": {"bound": "alu", "achieved": asm_ach / 1e12, "peak": PEAK["f64"] / 1e12,
                         "unit": "TFLOP/s", "frac": asm_ach / PEAK["f64"], "ms": asm_ms,
                         "work": f"{ASM_FLOPS_PER_ENTRY:.0f} FP64 flops per influence entry"},
    }
    dom = "lu_solve_f64" if lu_ms >= asm_ms else "assemble_f64"
    roof = dict(kern[dom])
    traffic = None
    if dom == "lu_solve_f64" and a.workload == "ga2048" and a.batch is None and a.wave_limit is None:
        import hashlib
        src = "lu_wave.hip"
        with open(os.path.join(os.path.dirname(P.__file__), "csrc", src), "rb") as f:
            traffic = LU_TRAFFIC.get((src, hashlib.sha256(f.read()).hexdigest()[:16]))
    roof = {"kernel": dom, "bound": roof["bound"], "achieved": roof["achieved"], "peak": roof["peak"],
            "unit": roof["unit"], "frac": roof["frac"], "traffic": traffic}

    out = {
        "metric": METRIC,
        "value": v64,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {B} seeded NACA 4-digit airfoils, N={int(w.n_panels.max())} "
                               f"panels (cosine spacing, closed TE), one {int(w.n_panels.max()) + 1}-order "
                               f"system per airfoil, {n_solves} angle(s) total",
                   "airfoils": B, "panels": int(w.n_panels.max()), "angles": n_solves},
        "fp64": dict(r64, solves_per_s=v64, bad_info=int(np.sum(info64 != 0))),
        "fp32_refine": dict(r32, solves_per_s=v32, bad_info=int(np.sum(info32 != 0)),
                            refine_sweeps_max=int(iters32.max()), refine_sweeps_mean=float(iters32.mean())),
        "adjoint": adj,
        "roofline": roof,
        "roofline_kernels": kern,
    }

    if not a.no_cpu_baseline:
        import oracle
        nthr = min(os.cpu_count() or 1, 16)
        S = min(B, a.cpu_sample or B)
        idx = np.linspace(0, B - 1, S).astype(int)
        ws = w.subset(idx)
        xy_o, noff_o = oracle.workload_nodes(ws)
        w0 = ws.subset(np.arange(min(S, nthr)))          # untimed warm-up (pages, threads)
        x0, n0 = oracle.workload_nodes(w0)
        oracle.solve_batch(x0, n0, w0.alpha_flat(), w0.alpha_offsets(), nthreads=nthr)
        t0 = time.perf_counter()
        ref = oracle.solve_batch(xy_o, noff_o, ws.alpha_flat(), ws.alpha_offsets(), nthreads=nthr)
        dt = time.perf_counter() - t0
        # parity of the timed GPU results on the sampled airfoils
        aidx = np.concatenate([np.arange(aoff[i], aoff[i + 1]) for i in idx])
        so = np.concatenate([[0], np.cumsum((np.diff(noff) - 1) * np.diff(aoff))])
        cpidx = np.concatenate([np.arange(so[i], so[i + 1]) for i in idx])

        def err(cl, cp):
            ecl = np.max(np.abs(cl[aidx] - ref["cl"]) / np.maximum(1.0, np.abs(ref["cl"])))
            ecp = np.max(np.abs(cp[cpidx] - ref["cp"])) / max(1.0, np.max(np.abs(ref["cp"])))
            return float(ecl), float(ecp)

        e64, p64 = err(cl64, cp64)
        e32, p32 = err(cl32, cp32)
        out["fp64"].update(cl_err=e64, cp_err=p64)
        out["fp32_refine"].update(cl_err=e32, cp_err=p32)
        out["cpu_baseline"] = {"value": int(ref["cl"].size) / dt, "unit": "solves/s",
                               "cores": int(ref["threads"]), "kind": "oracle",
                               "sample": f"{S} of the {B} airfoils, full pipeline (nodes given; assembly, "
                                         f"LU, solve, forces in plain C FP64, OpenMP over airfoils), "
                                         f"{dt:.2f} s wall"}
        out["cl_err_vs_oracle"] = {"fp64": e64, "fp32_refine": e32}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
