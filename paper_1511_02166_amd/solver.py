"""Convenience layer over the C ABI: a batch solver object and autograd hooks.

torch provides the device memory (workspace and outputs) and the stream;
all arithmetic happens in the library's HIP kernels.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import _binding as B


def _aligned_workspace(nbytes: int, device) -> tuple[torch.Tensor, torch.Tensor]:
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:off + nbytes]


class TileTable:
    """Measured tilings per batch layout (the autotuner's table), optionally
    kept in a JSON file so that later runs with the same layout (a genetic
    algorithm's generations) skip the search."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key):
        return self.entries.get(key)

    def put(self, key, entry):
        self.entries[key] = entry
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1)
            os.replace(tmp, self.path)


class PanelSolver:
    """One batch layout (node and angle offsets) with its workspace and outputs.

    Typical use (all tensors on the GPU, float64)::

        s = PanelSolver(node_offsets, alpha_offsets)
        out = s.solve(xy, alpha)          # dict of gamma, cp, cl, cl_p, info
    """

    def __init__(self, node_offsets, alpha_offsets, precision=B.PANEL_FP64, device="cuda",
                 wave_limit=None, tiling=None, formulation=B.PANEL_STREAM_FUNCTION):
        self.device = torch.device(device)
        self.plan = B.Plan(node_offsets, alpha_offsets, precision, formulation)
        self.formulation = int(formulation)
        if tiling is not None:
            B.panel_plan_set_tiling(self.plan, *tiling)
            wave_limit = tiling[0]
        elif wave_limit is not None:
            B.panel_plan_set_wave_limit(self.plan, wave_limit)
        self.wave_limit = 320 if wave_limit is None else int(wave_limit)
        self.precision = int(precision)
        p = self.plan
        self._ws_raw, self.ws = _aligned_workspace(p.workspace_size(), self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.info = torch.zeros(p.B, dtype=torch.int32, device=self.device)
        self.cl = torch.empty(p.n_alpha, **f64)
        self.cl_p = torch.empty(p.n_alpha, **f64)
        self.gamma = torch.empty(p.n_out, **f64)
        self.cp = torch.empty(p.n_out, **f64)
        self.adj_info = torch.zeros(p.B, dtype=torch.int32, device=self.device)
        self.node_off_dev = torch.as_tensor(p.node_offsets, dtype=torch.int32, device=self.device)
        B.panel_workspace_init(p, self.ws)
        # counts forward solves: the adjoint uses whatever factors the
        # workspace holds, so autograd checks that they are still its own
        self.steps = 0

    @property
    def B(self) -> int:
        return self.plan.B

    def set_wave_limit(self, max_n1: int):
        """Systems of order <= max_n1 go to the one-wavefront kernels (0..320)."""
        B.panel_plan_set_wave_limit(self.plan, max_n1)
        B.panel_workspace_init(self.plan, self.ws)
        self.wave_limit = int(max_n1)

    @property
    def tiling(self) -> dict:
        return B.panel_plan_get_tiling(self.plan)

    def set_tiling(self, wave_max_n1: int, persistent: int = 1, wg_waves: int = 0):
        """Kernel mapping of the factorisation (panel_tiling in include/panel.h)."""
        B.panel_plan_set_tiling(self.plan, wave_max_n1, persistent, wg_waves)
        B.panel_workspace_init(self.plan, self.ws)
        self.wave_limit = int(wave_max_n1)

    def tiling_candidates(self):
        """Distinct tilings for this batch: wave limits that split the systems
        differently, one launch or one per kernel family, and four or eight
        wavefronts per workgroup-factored system where some exist."""
        n1 = np.asarray(self.plan.n_panels) + 1
        out, seen = [], set()
        for wl in (320, 256, 192, 128, 0):
            big = n1 > wl
            nb = int(big.sum())
            key_part = tuple(np.flatnonzero(big)) if 0 < nb < len(n1) else nb
            wgs = (0,) if nb == 0 else ((8,) if int(n1.max()) > 768 else (4, 8))
            for pers in (1, 0):
                for wg in wgs:
                    # one launch applies only where the workgroup systems fit four wavefronts
                    eff_pers = pers if (nb == 0 or wg == 4) else 0
                    key = (key_part, eff_pers, wg)
                    if key in seen:
                        continue
                    seen.add(key)
                    out.append((wl, eff_pers, wg))
        return out

    def shape_key(self) -> str:
        """Identifies the batch layout (precision, panel and angle counts)."""
        h = hashlib.sha256()
        h.update(np.asarray([self.precision], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.plan.node_offsets, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.plan.alpha_offsets, dtype=np.int32).tobytes())
        return h.hexdigest()[:24]

    def autotune(self, xy, alpha, chord=None, vinf=1.0, refine_tol=1e-10, max_iter=10, reps=3,
                 table: "TileTable | None" = None, candidates=None):
        """Time the step (assembly -> factor/solve -> forces) on this batch for
        every candidate tiling and keep the fastest.

        With a ``table`` whose entry for this batch layout exists, that entry
        is applied without timing; otherwise the measured result is stored in
        it.  Returns {(wave_max_n1, persistent, wg_waves): ms}."""
        key = self.shape_key()
        if table is not None:
            hit = table.get(key)
            if hit is not None:
                self.set_tiling(*hit["tiling"])
                return {tuple(k): v for k, v in hit["times"]}
        times = {}
        for cand in (candidates or self.tiling_candidates()):
            self.set_tiling(*cand)
            self.step(xy, alpha, chord, vinf, refine_tol, max_iter)
            torch.cuda.synchronize(self.device)
            ms = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                self.step(xy, alpha, chord, vinf, refine_tol, max_iter)
                e1.record()
                torch.cuda.synchronize(self.device)
                ms.append(e0.elapsed_time(e1))
            times[tuple(cand)] = float(np.median(ms))
        best = min(times, key=times.get)
        self.set_tiling(*best)
        if table is not None:
            table.put(key, dict(tiling=list(best), times=[[list(k), v] for k, v in times.items()],
                                B=self.B, precision=self.precision))
        return times

    # -- steps ---------------------------------------------------------------
    def naca4(self, mpt: torch.Tensor, closed_te: bool = True, out: torch.Tensor | None = None):
        xy = out if out is not None else torch.empty(2 * self.plan.n_nodes, dtype=torch.float64,
                                                     device=self.device)
        B.panel_naca4(self.plan.B, self.node_off_dev, closed_te, mpt, xy)
        return xy

    def assemble(self, xy, alpha, chord=None, vinf=1.0):
        B.panel_assemble(self.plan, xy, alpha, chord, vinf, self.ws)

    def factor_solve(self, refine_tol=1e-10, max_iter=10):
        B.panel_factor_solve(self.plan, self.ws, refine_tol, max_iter, self.info)

    def forces(self, fields=True):
        B.panel_forces(self.plan, self.ws, self.gamma if fields else None, self.cp if fields else None,
                       self.cl, self.cl_p)

    def step(self, xy, alpha, chord=None, vinf=1.0, refine_tol=1e-10, max_iter=10, fields=True):
        """assemble -> factor_solve -> forces, enqueued on the current stream."""
        self.assemble(xy, alpha, chord, vinf)
        self.factor_solve(refine_tol, max_iter)
        self.forces(fields)
        self.steps += 1

    def solve(self, xy, alpha, chord=None, vinf=1.0, refine_tol=1e-10, max_iter=10):
        self.step(xy, alpha, chord, vinf, refine_tol, max_iter)
        return dict(gamma=self.gamma, cp=self.cp, cl=self.cl, cl_p=self.cl_p, info=self.info)

    def viscous(self, re: float):
        """Thwaites' laminar correction on the last forces' surface speeds:
        dict(cd, ld, sep) (see panel_thwaites in include/panel.h)."""
        p = self.plan
        cd = torch.empty(p.n_alpha, dtype=torch.float64, device=self.device)
        ld = torch.empty_like(cd)
        sep = torch.empty(2 * p.n_alpha, dtype=torch.int32, device=self.device)
        B.panel_thwaites(p, self.ws, self.gamma, self.cl, re, cd, ld, sep)
        return dict(cd=cd, ld=ld, sep=sep)

    def adjoint(self, xy, dcl, dcp=None, out=None):
        """d/d(nodes) of sum(dcl * cl) + sum(dcp * cp) for the last step's
        factors (per-airfoil status in ``adj_info``)."""
        dxy = out if out is not None else torch.empty(2 * self.plan.n_nodes, dtype=torch.float64,
                                                      device=self.device)
        B.panel_adjoint(self.plan, self.ws, xy, dcl, dcp, dxy, self.adj_info)
        return dxy

    def naca4_vjp(self, mpt, dxy, closed_te=True):
        dmpt = torch.empty_like(mpt)
        B.panel_naca4_vjp(self.plan.B, self.node_off_dev, closed_te, mpt, dxy, dmpt)
        return dmpt

    # -- inspection ------------------------------------------------------------
    def system(self, b: int, which: str = "a64") -> tuple[np.ndarray, np.ndarray]:
        """Airfoil b's stored system: (matrix n1 x n1, right-hand sides K x n1).

        After panel_assemble this is M and b; after panel_factor_solve the
        factored copy holds L\\U and L^{-1} P b."""
        d = self.plan.layout(b)
        n1, ld, K = d["n1"], d["ld"], d["K"]
        if which == "a64":
            t = self.ws[d["a64"]:d["a64"] + 8 * ld * (n1 + K)].view(torch.float64)
        else:
            t = self.ws[d["a32"]:d["a32"] + 4 * ld * (n1 + K)].view(torch.float32)
        cols = t.cpu().numpy().reshape(n1 + K, ld)[:, :n1]
        return cols[:n1].T.copy(), cols[n1:].copy()

    def tangential(self, b: int) -> np.ndarray:
        """Hess-Smith: airfoil b's tangential-velocity influence matrix [N, N+1]."""
        if self.formulation != B.PANEL_HESS_SMITH:
            raise ValueError("only the Hess-Smith formulation keeps a tangential matrix")
        d = self.plan.layout(b)
        n1, ld = d["n1"], d["ld"]
        t = self.ws[d["tg"]:d["tg"] + 8 * ld * n1].view(torch.float64)
        return t.cpu().numpy().reshape(n1, ld)[:, :n1 - 1].T.copy()

    def pivots(self, b: int) -> np.ndarray:
        d = self.plan.layout(b)
        return self.ws[d["piv"]:d["piv"] + 4 * d["n1"]].view(torch.int32).cpu().numpy()

    def refine_iterations(self) -> np.ndarray:
        """Refinement sweeps per airfoil of the last mixed-precision solve."""
        d = self.plan.layout(0)
        return self.ws[d["iters"]:d["iters"] + 4 * self.plan.B].view(torch.int32).cpu().numpy()


class _ClFunction(torch.autograd.Function):
    """(Cl, Cp)(xy) with the hand-written adjoint kernels as the backward."""

    @staticmethod
    def forward(ctx, xy, alpha, solver: PanelSolver, chord, vinf):
        solver.step(xy, alpha, chord, vinf, fields=True)
        ctx.solver = solver
        ctx.step_id = solver.steps
        ctx.args = (alpha, chord, vinf)
        ctx.save_for_backward(xy)
        ctx.set_materialize_grads(False)
        return solver.cl.clone(), solver.cp.clone()

    @staticmethod
    def backward(ctx, dcl, dcp):
        (xy,) = ctx.saved_tensors
        s = ctx.solver
        if dcl is None and dcp is None:
            return None, None, None, None, None
        if s.steps != ctx.step_id:
            # the solver has solved another batch since this forward: redo
            # this one so the adjoint sees its own factors (this overwrites
            # the solver's output buffers with this forward's values)
            alpha, chord, vinf = ctx.args
            s.step(xy, alpha, chord, vinf, fields=False)
            ctx.step_id = s.steps
        if dcl is None:
            dcl = torch.zeros(s.plan.n_alpha, dtype=torch.float64, device=s.device)
        dxy = s.adjoint(xy, dcl.contiguous(), None if dcp is None else dcp.contiguous())
        return dxy, None, None, None, None


def panel_cl_cp(xy, alpha, solver: PanelSolver, chord=None, vinf=1.0):
    """Lift and pressure coefficients of a batch, (cl, cp), differentiable
    with respect to the nodes."""
    return _ClFunction.apply(xy, alpha, solver, chord, vinf)


def panel_cl(xy, alpha, solver: PanelSolver, chord=None, vinf=1.0):
    """Lift coefficients of a batch, differentiable with respect to the nodes."""
    return _ClFunction.apply(xy, alpha, solver, chord, vinf)[0]


class _NacaFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mpt, solver: PanelSolver, closed_te):
        ctx.solver, ctx.closed_te = solver, closed_te
        ctx.save_for_backward(mpt)
        return solver.naca4(mpt, closed_te)

    @staticmethod
    def backward(ctx, dxy):
        (mpt,) = ctx.saved_tensors
        return ctx.solver.naca4_vjp(mpt, dxy.contiguous(), ctx.closed_te), None, None


def naca_cl(mpt, alpha, solver: PanelSolver, closed_te=True, vinf=1.0):
    """Cl of NACA sections, differentiable with respect to (m, p, t)."""
    xy = _NacaFunction.apply(mpt, solver, closed_te)
    return panel_cl(xy, alpha, solver, None, vinf)
