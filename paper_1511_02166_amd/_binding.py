"""ctypes marshalling for the C ABI in include/panel.h (same names)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libpanel.so")

PANEL_OK, PANEL_EINVAL, PANEL_ENOMEM, PANEL_EHIP, PANEL_EUNSUPPORTED = range(5)
PANEL_FP64, PANEL_FP32_REFINE = 0, 1
PANEL_STREAM_FUNCTION, PANEL_HESS_SMITH = 0, 1
PANEL_NMAX, PANEL_NMIN, PANEL_KMAX = 1024, 4, 16
PANEL_NOALLOC_MAX_BYTES = 256 << 20
PANEL_GA_MAX_GENES, PANEL_GA_MAX_CTRL, PANEL_GA_MAX_DEGREE, PANEL_GA_MAX_TOURNAMENT = 64, 64, 7, 16

_lib = None


class panel_tiling(C.Structure):
    """Mirror of the C struct panel_tiling (see include/panel.h)."""
    _fields_ = [("wave_max_n1", C.c_int32), ("persistent", C.c_int32), ("wg_waves", C.c_int32)]

    def as_dict(self):
        return dict(wave_max_n1=int(self.wave_max_n1), persistent=int(self.persistent), wg_waves=int(self.wg_waves))


class PanelError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{panel_status_str(status)}: {msg}")
        self.status = status


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libpanel.so (built in-tree by ``python -m paper_1511_02166_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_1511_02166_amd.build` (no CPU fallback exists)")
    L = C.CDLL(_LIB_PATH)
    vp, i32, f64, sz = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
    L.panel_plan_create.argtypes = [i32, vp, vp, i32, C.POINTER(vp)]
    L.panel_plan_destroy.argtypes = [vp]
    L.panel_plan_destroy.restype = None
    L.panel_plan_set_wave_limit.argtypes = [vp, i32]
    L.panel_plan_set_tiling.argtypes = [vp, C.POINTER(panel_tiling)]
    L.panel_plan_set_formulation.argtypes = [vp, i32]
    L.panel_plan_get_tiling.argtypes = [vp, C.POINTER(panel_tiling)]
    L.panel_workspace_size.argtypes = [vp, C.POINTER(sz)]
    L.panel_workspace_init.argtypes = [vp, vp, vp]
    L.panel_workspace_layout.argtypes = [vp, i32, vp]
    L.panel_assemble.argtypes = [vp, vp, vp, vp, f64, vp, vp]
    L.panel_factor_solve.argtypes = [vp, vp, f64, i32, vp, vp]
    L.panel_forces.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.panel_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.panel_naca4.argtypes = [i32, vp, i32, vp, vp, vp]
    L.panel_thwaites.argtypes = [vp, vp, vp, vp, f64, vp, vp, vp, vp]
    L.panel_naca4_vjp.argtypes = [i32, vp, i32, vp, vp, vp, vp]
    L.panel_math_eval.argtypes = [i32, vp, vp, vp, vp, vp]
    L.panel_solve_noalloc.argtypes = [vp, vp, vp, vp, f64, f64, i32, vp, vp, vp, vp, vp, vp]
    L.panel_bspline_nodes.argtypes = [i32, i32, i32, i32, vp, i32, vp, vp, vp, vp]
    L.panel_ga_init.argtypes = [i32, i32, vp, vp, vp, vp, vp]
    L.panel_ga_fitness.argtypes = [vp, vp, vp, vp, vp, vp]
    L.panel_ga_uniform_count.argtypes = [i32, i32, C.POINTER(C.c_int64)]
    L.panel_ga_step.argtypes = [i32, i32, i32, f64, f64, f64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.panel_ga_record.argtypes = [i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    L.panel_status_str.argtypes = [i32]
    L.panel_status_str.restype = C.c_char_p
    L.panel_last_error.argtypes = []
    L.panel_last_error.restype = C.c_char_p
    for name in ("panel_plan_create", "panel_plan_set_wave_limit", "panel_plan_set_tiling", "panel_plan_get_tiling",
                 "panel_plan_set_formulation",
                 "panel_workspace_size", "panel_workspace_init",
                 "panel_workspace_layout", "panel_assemble",
                 "panel_factor_solve", "panel_forces", "panel_adjoint", "panel_naca4", "panel_thwaites",
                 "panel_naca4_vjp", "panel_math_eval", "panel_solve_noalloc", "panel_bspline_nodes", "panel_ga_init",
                 "panel_ga_fitness", "panel_ga_uniform_count", "panel_ga_step", "panel_ga_record"):
        getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def panel_status_str(status: int) -> str:
    return load_library().panel_status_str(int(status)).decode()


def panel_last_error() -> str:
    return load_library().panel_last_error().decode()


def _check(status: int):
    if status != PANEL_OK:
        raise PanelError(status, panel_last_error())


def _ptr(t, dtype=None, name="array", allow_none=False):
    """Device pointer of a contiguous CUDA/HIP torch tensor (or None)."""
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU (got {t.device})")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """Owner of a ``panel_plan*`` (host metadata for one batch layout)."""

    def __init__(self, node_offsets, alpha_offsets, precision=PANEL_FP64, formulation=PANEL_STREAM_FUNCTION):
        L = load_library()
        no = np.ascontiguousarray(node_offsets, dtype=np.int32)
        ao = np.ascontiguousarray(alpha_offsets, dtype=np.int32)
        if no.ndim != 1 or ao.ndim != 1 or no.size != ao.size or no.size < 2:
            raise ValueError("node_offsets and alpha_offsets must be 1-D int arrays of length B+1")
        self.B = int(no.size - 1)
        self.node_offsets = no
        self.alpha_offsets = ao
        self.precision = int(precision)
        h = C.c_void_p()
        _check(L.panel_plan_create(self.B, no.ctypes.data_as(C.c_void_p), ao.ctypes.data_as(C.c_void_p),
                                   self.precision, C.byref(h)))
        self._h = h
        self.formulation = int(formulation)
        if self.formulation != PANEL_STREAM_FUNCTION:
            _check(L.panel_plan_set_formulation(h, self.formulation))
        self.n_nodes = int(no[-1])
        self.n_alpha = int(ao[-1])
        n = np.diff(no).astype(np.int64) - 1
        k = np.diff(ao).astype(np.int64)
        self.n_panels = n
        self.n_angles = k
        self.n_out = int(np.sum(n * k))

    @property
    def handle(self):
        return self._h

    def workspace_size(self) -> int:
        out = C.c_size_t()
        _check(load_library().panel_workspace_size(self._h, C.byref(out)))
        return int(out.value)

    def layout(self, b: int) -> dict:
        d = np.zeros(9, dtype=np.int64)
        _check(load_library().panel_workspace_layout(self._h, int(b), d.ctypes.data_as(C.c_void_p)))
        return dict(a64=int(d[0]), a32=int(d[1]), x=int(d[2]), piv=int(d[3]), n1=int(d[4]),
                    ld=int(d[5]), K=int(d[6]), iters=int(d[7]), tg=int(d[8]))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.panel_plan_destroy(h)
            self._h = None


# -- functions with the C ABI's names ---------------------------------------

def panel_plan_create(node_offsets, alpha_offsets, precision=PANEL_FP64) -> Plan:
    return Plan(node_offsets, alpha_offsets, precision)


def panel_plan_set_formulation(plan: Plan, formulation: int):
    """PANEL_STREAM_FUNCTION or PANEL_HESS_SMITH (before sizing the workspace)."""
    _check(load_library().panel_plan_set_formulation(plan.handle, int(formulation)))
    plan.formulation = int(formulation)


def panel_plan_destroy(plan: Plan):
    if plan._h is not None and plan._h.value:
        load_library().panel_plan_destroy(plan._h)
    plan._h = None


def panel_plan_set_wave_limit(plan: Plan, max_n1: int):
    """Largest system order factored by one wavefront (0..320; 0 = none)."""
    _check(load_library().panel_plan_set_wave_limit(plan.handle, int(max_n1)))


def panel_plan_set_tiling(plan: Plan, wave_max_n1: int, persistent: int, wg_waves: int):
    """Kernel mapping of the factorisation (see panel_tiling in include/panel.h)."""
    t = panel_tiling(int(wave_max_n1), int(persistent), int(wg_waves))
    _check(load_library().panel_plan_set_tiling(plan.handle, C.byref(t)))


def panel_plan_get_tiling(plan: Plan) -> dict:
    t = panel_tiling()
    _check(load_library().panel_plan_get_tiling(plan.handle, C.byref(t)))
    return t.as_dict()


def panel_workspace_size(plan: Plan) -> int:
    return plan.workspace_size()


def panel_workspace_layout(plan: Plan, b: int) -> dict:
    return plan.layout(b)


def panel_workspace_init(plan: Plan, ws, stream=None):
    import torch
    _check(load_library().panel_workspace_init(plan.handle, _ptr(ws, torch.uint8, "ws"), _stream(stream)))


def panel_assemble(plan: Plan, xy, alpha, chord, vinf, ws, stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_assemble(plan.handle, _ptr(xy, d, "xy"), _ptr(alpha, d, "alpha"),
                                         _ptr(chord, d, "chord", True), float(vinf),
                                         _ptr(ws, torch.uint8, "ws"), _stream(stream)))


def panel_factor_solve(plan: Plan, ws, refine_tol, max_iter, info, stream=None):
    import torch
    _check(load_library().panel_factor_solve(plan.handle, _ptr(ws, torch.uint8, "ws"), float(refine_tol),
                                             int(max_iter), _ptr(info, torch.int32, "info"),
                                             _stream(stream)))


def panel_forces(plan: Plan, ws, gamma, cp, cl, cl_p, stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_forces(plan.handle, _ptr(ws, torch.uint8, "ws"),
                                       _ptr(gamma, d, "gamma", True), _ptr(cp, d, "cp", True),
                                       _ptr(cl, d, "cl"), _ptr(cl_p, d, "cl_p", True), _stream(stream)))


def panel_thwaites(plan: Plan, ws, gamma, cl, re, cd, ld, sep, stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_thwaites(plan.handle, _ptr(ws, torch.uint8, "ws"), _ptr(gamma, d, "gamma"),
                                         _ptr(cl, d, "cl"), float(re), _ptr(cd, d, "cd"), _ptr(ld, d, "ld"),
                                         _ptr(sep, torch.int32, "sep"), _stream(stream)))


def panel_adjoint(plan: Plan, ws, xy, dcl, dcp, dxy, info=None, stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_adjoint(plan.handle, _ptr(ws, torch.uint8, "ws"), _ptr(xy, d, "xy"),
                                        _ptr(dcl, d, "dcl"), _ptr(dcp, d, "dcp", True), _ptr(dxy, d, "dxy"),
                                        _ptr(info, torch.int32, "info", True), _stream(stream)))


def panel_solve_noalloc(plan: Plan, xy, alpha, chord, vinf, refine_tol, max_iter, info, gamma, cp, cl, cl_p,
                        stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_solve_noalloc(plan.handle, _ptr(xy, d, "xy"), _ptr(alpha, d, "alpha"),
                                              _ptr(chord, d, "chord", True), float(vinf), float(refine_tol),
                                              int(max_iter), _ptr(info, torch.int32, "info"),
                                              _ptr(gamma, d, "gamma", True), _ptr(cp, d, "cp", True),
                                              _ptr(cl, d, "cl"), _ptr(cl_p, d, "cl_p", True), _stream(stream)))


def panel_naca4(B, node_off, closed_te, mpt, xy, stream=None):
    import torch
    _check(load_library().panel_naca4(int(B), _ptr(node_off, torch.int32, "node_off"), int(bool(closed_te)),
                                      _ptr(mpt, torch.float64, "mpt"), _ptr(xy, torch.float64, "xy"),
                                      _stream(stream)))


def panel_naca4_vjp(B, node_off, closed_te, mpt, dxy, dmpt, stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_naca4_vjp(int(B), _ptr(node_off, torch.int32, "node_off"),
                                          int(bool(closed_te)), _ptr(mpt, d, "mpt"), _ptr(dxy, d, "dxy"),
                                          _ptr(dmpt, d, "dmpt"), _stream(stream)))


def panel_math_eval(x, y, log_out, atan2_out, stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_math_eval(int(x.numel()), _ptr(x, d, "x"), _ptr(y, d, "y", True),
                                          _ptr(log_out, d, "log_out", True),
                                          _ptr(atan2_out, d, "atan2_out", True), _stream(stream)))


# ---- genetic algorithm -----------------------------------------------------------

def _host_f64(a, name):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    return a, a.ctypes.data_as(C.c_void_p)


def _host_i32(a, name):
    a = np.ascontiguousarray(a, dtype=np.int32).reshape(-1)
    return a, a.ctypes.data_as(C.c_void_p)


def panel_bspline_nodes(B, N, template, degree, gene_map, genome, xy, stream=None):
    """template: host [M, 2]; gene_map: host int [G]; genome, xy: device."""
    import torch
    t, tp = _host_f64(template, "template")
    gm, gp = _host_i32(gene_map, "gene_map")
    _check(load_library().panel_bspline_nodes(int(B), int(N), t.size // 2, int(degree), tp, gm.size, gp,
                                              _ptr(genome, torch.float64, "genome", allow_none=gm.size == 0),
                                              _ptr(xy, torch.float64, "xy"), _stream(stream)))


def panel_ga_init(B, G, lo, hi, u, genome, stream=None):
    import torch
    lo_, lp = _host_f64(lo, "lo")
    hi_, hp = _host_f64(hi, "hi")
    if lo_.size != G or hi_.size != G:
        raise ValueError("lo and hi need one value per gene")
    _check(load_library().panel_ga_init(int(B), int(G), lp, hp, _ptr(u, torch.float64, "u"),
                                        _ptr(genome, torch.float64, "genome"), _stream(stream)))


def panel_ga_fitness(plan: Plan, ws, ld, info, fitness, stream=None):
    import torch
    _check(load_library().panel_ga_fitness(plan.handle, _ptr(ws, torch.uint8, "ws"), _ptr(ld, torch.float64, "ld"),
                                           _ptr(info, torch.int32, "info"), _ptr(fitness, torch.float64, "fitness"),
                                           _stream(stream)))


def panel_ga_uniform_count(B, k) -> int:
    n = C.c_int64()
    _check(load_library().panel_ga_uniform_count(int(B), int(k), C.byref(n)))
    return int(n.value)


def panel_ga_step(B, G, k, p_sel, p_mut, sigma, lo, hi, fitness, genome_in, u, genome_out, trace=None,
                  stream=None):
    import torch
    lo_, lp = _host_f64(lo, "lo")
    hi_, hp = _host_f64(hi, "hi")
    if lo_.size != G or hi_.size != G:
        raise ValueError("lo and hi need one value per gene")
    _check(load_library().panel_ga_step(int(B), int(G), int(k), float(p_sel), float(p_mut), float(sigma), lp, hp,
                                        _ptr(fitness, torch.float64, "fitness"),
                                        _ptr(genome_in, torch.float64, "genome_in"), _ptr(u, torch.float64, "u"),
                                        _ptr(genome_out, torch.float64, "genome_out"),
                                        _ptr(trace, torch.int32, "trace", allow_none=True), _stream(stream)))


def panel_ga_record(B, G, fitness, genome, counter, max_gen, hist_fit, hist_idx, best_fit, best_genome,
                    stream=None):
    import torch
    d = torch.float64
    _check(load_library().panel_ga_record(int(B), int(G), _ptr(fitness, d, "fitness"), _ptr(genome, d, "genome"),
                                          _ptr(counter, torch.int32, "counter"), int(max_gen),
                                          _ptr(hist_fit, d, "hist_fit", allow_none=max_gen == 0),
                                          _ptr(hist_idx, torch.int32, "hist_idx", allow_none=max_gen == 0),
                                          _ptr(best_fit, d, "best_fit"), _ptr(best_genome, d, "best_genome"),
                                          _stream(stream)))
