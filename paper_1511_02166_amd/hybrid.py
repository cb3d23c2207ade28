"""The paper's hybrid scheme, kept as an ablation (Sec. 4: assembly on the
accelerator, LU on the host with LAPACK, the population cut into slices so
that the assembly and the device-to-host copy of one slice overlap the host
solves of the previous one).

On MI355X the all-device path (PanelSolver) supersedes it: the assembled
systems are ~1 MB per airfoil at N=256, so moving them over PCIe alone costs
more than the device's whole assemble + factor + solve step.  This module
exists to measure that, slice count by slice count, in the terms of the
paper's table (wall time W, host solve time L, unhidden overhead O = W - L,
device assembly time A); it is not a fallback of the product path.

Per slice the device assembles the slice's systems (the library's FP64
assembly kernel; for FP32 the FP32 copy it writes is what travels) and
copies them into pinned host memory on the same stream; the host waits for
that slice's event and solves its systems with LAPACK (numpy.linalg.solve,
gesv with partial pivoting) in a thread pool, then forms Cl from the
circulation.  Only the systems cross the bus; nodes, angles and chords are
inputs and are read once per step.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch
from threadpoolctl import threadpool_limits

from . import _binding as B
from .solver import PanelSolver


class HybridSolver:
    """Slices of a batch: device assembly -> D2H -> host LAPACK solve."""

    def __init__(self, node_offsets, alpha_offsets, slices: int, threads: int = 16,
                 precision: int = B.PANEL_FP64, device="cuda"):
        noff = np.ascontiguousarray(node_offsets, dtype=np.int64)
        aoff = np.ascontiguousarray(alpha_offsets, dtype=np.int64)
        self.B = noff.size - 1
        if not 1 <= slices <= self.B:
            raise ValueError("slices must be in 1..B")
        self.noff, self.aoff, self.precision = noff, aoff, int(precision)
        self.device = torch.device(device)
        self.threads = int(threads)
        cuts = np.linspace(0, self.B, slices + 1).round().astype(int)
        self.slices = []
        for s in range(slices):
            b0, b1 = int(cuts[s]), int(cuts[s + 1])
            so = PanelSolver((noff[b0:b1 + 1] - noff[b0]).astype(np.int32),
                             (aoff[b0:b1 + 1] - aoff[b0]).astype(np.int32), self.precision, device=device)
            key = "a64" if self.precision == B.PANEL_FP64 else "a32"
            esz = 8 if key == "a64" else 4
            lays = [so.plan.layout(b) for b in range(b1 - b0)]
            lo = min(d[key] for d in lays)
            hi = max(d[key] + esz * d["ld"] * (d["n1"] + d["K"]) for d in lays)
            host = torch.empty(hi - lo, dtype=torch.uint8, pin_memory=True)
            # airfoils grouped by system shape, for one batched gesv each
            groups = {}
            for i, d in enumerate(lays):
                groups.setdefault((d["n1"], d["ld"], d["K"]), []).append((i, d[key] - lo))
            self.slices.append(dict(b0=b0, b1=b1, solver=so, lo=lo, hi=hi, host=host, groups=groups,
                                    dtype=np.float64 if esz == 8 else np.float32,
                                    ev_a=torch.cuda.Event(enable_timing=True),
                                    ev_c=torch.cuda.Event(enable_timing=True),
                                    ev_0=torch.cuda.Event(enable_timing=True)))
        self.pool = ThreadPoolExecutor(max_workers=self.threads)

    def _solve_group(self, buf, dtype, n1, ld, K, items, L, scale, out_cl, a0):
        # column-major systems: rows of the view are the matrix's columns
        nb = len(items)
        M = np.empty((nb, n1 + K, n1), dtype=dtype)
        for q, (i, off) in enumerate(items):
            M[q] = np.frombuffer(buf, dtype=dtype, count=ld * (n1 + K), offset=off).reshape(n1 + K, ld)[:, :n1]
        A = np.transpose(M[:, :n1, :], (0, 2, 1))
        R = np.transpose(M[:, n1:, :], (0, 2, 1))
        X = np.linalg.solve(A, R)                     # [nb, n1, K]
        for q, (i, _) in enumerate(items):
            b = a0 + i
            g = X[q, :n1 - 1, :].astype(np.float64)   # the sheet strengths gamma_i
            out_cl[self.aoff[b]:self.aoff[b + 1]] = scale[b] * (L[b][:, None] * g).sum(0)

    def step(self, xy, alpha, chord=None, vinf: float = 1.0):
        """One pass over the batch; returns (cl [sum K] host array, timings)."""
        # the pool's workers run single-threaded LAPACK calls side by side
        with threadpool_limits(1):
            return self._step(xy, alpha, chord, vinf)

    def _step(self, xy, alpha, chord, vinf):
        stream = torch.cuda.current_stream()
        t0 = time.perf_counter()
        # inputs read once on the host: panel lengths and the lift scale
        P = xy.detach().cpu().numpy()
        ch = np.ones(self.B) if chord is None else chord.detach().cpu().numpy()
        L = []
        for b in range(self.B):
            nb = P[2 * self.noff[b]:2 * self.noff[b + 1]].reshape(-1, 2)
            L.append(np.hypot(*np.diff(nb, axis=0).T))
        scale = -2.0 / (vinf * ch)
        # device: every slice's assembly and copy enqueued up front
        for sl in self.slices:
            b0, b1 = sl["b0"], sl["b1"]
            so = sl["solver"]
            sl["ev_0"].record(stream)
            so.assemble(xy[2 * self.noff[b0]:2 * self.noff[b1]], alpha[self.aoff[b0]:self.aoff[b1]],
                        None if chord is None else chord[b0:b1], vinf)
            sl["ev_a"].record(stream)
            sl["host"].copy_(so.ws[sl["lo"]:sl["hi"]], non_blocking=True)
            sl["ev_c"].record(stream)
        cl = np.empty(int(self.aoff[-1]))
        t_solve = 0.0
        for sl in self.slices:
            sl["ev_c"].synchronize()
            ts = time.perf_counter()
            buf = sl["host"].numpy()
            futs = []
            for (n1, ld, K), items in sl["groups"].items():
                step_ = max(1, -(-len(items) // self.threads))
                for c in range(0, len(items), step_):
                    futs.append(self.pool.submit(self._solve_group, buf, sl["dtype"], n1, ld, K,
                                                 items[c:c + step_], L, scale, cl, sl["b0"]))
            for f in futs:
                f.result()
            t_solve += time.perf_counter() - ts
        W = time.perf_counter() - t0
        A = sum(sl["ev_0"].elapsed_time(sl["ev_a"]) for sl in self.slices) * 1e-3
        C = sum(sl["ev_a"].elapsed_time(sl["ev_c"]) for sl in self.slices) * 1e-3
        nbytes = sum(sl["hi"] - sl["lo"] for sl in self.slices)
        return cl, dict(W=W, L=t_solve, O=W - t_solve, A=A, copy=C, bytes=nbytes,
                        pcie_GBps=nbytes / C / 1e9 if C > 0 else None)

    def close(self):
        self.pool.shutdown()
