"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every symbol include/panel.h declares, and
reject bad arguments synchronously, before any HIP call is made.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "panel.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1511_02166_amd as P
    if not os.path.exists(P.lib_path()):
        from paper_1511_02166_amd import build
        build.build()
    return P.load_library()


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(panel_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("panel_plan_create", "panel_workspace_size", "panel_assemble", "panel_factor_solve",
              "panel_forces", "panel_adjoint", "panel_naca4", "panel_status_str"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared_functions():
        assert hasattr(lib, n), n


def _plan(lib, noff, aoff, prec=0):
    noff = np.ascontiguousarray(noff, dtype=np.int32)
    aoff = np.ascontiguousarray(aoff, dtype=np.int32)
    h = C.c_void_p()
    st = lib.panel_plan_create(len(noff) - 1, noff.ctypes.data_as(C.c_void_p),
                               aoff.ctypes.data_as(C.c_void_p), prec, C.byref(h))
    return st, h


def test_plan_validation(lib):
    import paper_1511_02166_amd as P
    st, h = _plan(lib, [0, 129, 258], [0, 1, 3])
    assert st == P._binding.PANEL_OK and h.value
    size = C.c_size_t()
    assert lib.panel_workspace_size(h, C.byref(size)) == 0
    # ld = 160 for n1 = 129; two systems of 160 x (129 + K) doubles at least
    assert size.value > 8 * 160 * (130 + 132)
    lib.panel_plan_destroy(h)
    bad = [([0, 3], [0, 1]),              # too few panels
           ([0, 2000], [0, 1]),           # too many panels
           ([1, 130], [0, 1]),            # offsets not starting at 0
           ([0, 129], [0, 0]),            # no angle
           ([0, 129], [0, 40])]           # too many angles
    for noff, aoff in bad:
        st, h = _plan(lib, noff, aoff)
        assert st == P._binding.PANEL_EINVAL, (noff, aoff)
        assert lib.panel_last_error()
    st, h = _plan(lib, [0, 129], [0, 1], prec=7)
    assert st == P._binding.PANEL_EINVAL
    st, h = _plan(lib, [0, 129], [0, 1])
    assert lib.panel_plan_set_wave_limit(h, 0) == 0
    assert lib.panel_plan_set_wave_limit(h, 320) == 0
    assert lib.panel_plan_set_wave_limit(h, 321) == P._binding.PANEL_EINVAL
    assert lib.panel_plan_set_wave_limit(h, -1) == P._binding.PANEL_EINVAL
    assert lib.panel_plan_set_wave_limit(None, 0) == P._binding.PANEL_EINVAL
    lib.panel_plan_destroy(h)


def test_changed_wave_limit_requires_workspace_init(lib):
    # The airfoil order lives in the workspace: after the limit changes, the
    # factorisation and the adjoint refuse to run (before any HIP call) until
    # panel_workspace_init has copied the new order.
    import paper_1511_02166_amd as P
    EINVAL = P._binding.PANEL_EINVAL
    st, h = _plan(lib, [0, 129, 500], [0, 1, 2])
    fake = C.c_void_p(0x100000)
    assert lib.panel_plan_set_wave_limit(h, 320) == 0           # unchanged: stays valid
    assert lib.panel_plan_set_wave_limit(h, 0) == 0
    assert lib.panel_factor_solve(h, fake, C.c_double(1e-10), 10, fake, None) == EINVAL
    assert b"panel_workspace_init" in lib.panel_last_error()
    assert lib.panel_adjoint(h, fake, fake, fake, None, fake, None, None) == EINVAL
    lib.panel_plan_destroy(h)


def test_entry_points_reject_bad_arguments_before_hip(lib):
    import paper_1511_02166_amd as P
    EINVAL = P._binding.PANEL_EINVAL
    st, h = _plan(lib, [0, 129], [0, 1], prec=1)
    assert st == 0
    fake = C.c_void_p(0x100000)          # never dereferenced: checks fail first
    odd = C.c_void_p(0x100003)
    assert lib.panel_assemble(h, None, fake, None, C.c_double(1.0), fake, None) == EINVAL
    assert lib.panel_assemble(h, odd, fake, None, C.c_double(1.0), fake, None) == EINVAL
    assert lib.panel_assemble(h, fake, fake, None, C.c_double(-1.0), fake, None) == EINVAL
    assert lib.panel_assemble(h, fake, fake, None, C.c_double(float("nan")), fake, None) == EINVAL
    assert lib.panel_assemble(h, fake, fake, None, C.c_double(1.0), C.c_void_p(0x100008), None) == EINVAL
    assert lib.panel_factor_solve(h, fake, C.c_double(0.0), 10, fake, None) == EINVAL
    assert lib.panel_factor_solve(h, fake, C.c_double(1e-10), 101, fake, None) == EINVAL
    assert lib.panel_factor_solve(h, fake, C.c_double(1e-10), 3, None, None) == EINVAL
    assert lib.panel_forces(h, fake, None, None, None, None, None) == EINVAL
    assert lib.panel_adjoint(h, fake, fake, None, None, fake, None, None) == EINVAL
    assert lib.panel_adjoint(h, fake, fake, fake, odd, fake, None, None) == EINVAL
    assert lib.panel_adjoint(h, fake, fake, fake, None, fake, C.c_void_p(0x100002), None) == EINVAL
    assert lib.panel_naca4(0, fake, 1, fake, fake, None) == EINVAL
    assert lib.panel_naca4_vjp(2, fake, 1, fake, None, fake, None) == EINVAL
    lib.panel_plan_destroy(h)


def test_layout_and_status_strings(lib):
    import paper_1511_02166_amd as P
    st, h = _plan(lib, [0, 257, 514], [0, 1, 5])
    d = (C.c_int64 * 9)()
    assert lib.panel_workspace_layout(h, 1, d) == 0
    assert d[4] == 257 and d[5] == 288 and d[6] == 4
    assert d[0] % 128 == 0 and d[8] == -1
    assert lib.panel_workspace_layout(h, 2, d) == P._binding.PANEL_EINVAL
    lib.panel_plan_destroy(h)
    for s in range(5):
        assert P.panel_status_str(s).startswith("PANEL_")


def test_noalloc_entry_refuses_oversized_plans_before_hip(lib):
    # 1024 sections at N = 256 need ~600 MB of workspace, more than the
    # static scratch: refused on the host, before any HIP call.
    import paper_1511_02166_amd as P
    noff = np.arange(1025, dtype=np.int32) * 257
    aoff = np.arange(1025, dtype=np.int32)
    st, h = _plan(lib, noff, aoff)
    size = C.c_size_t()
    assert lib.panel_workspace_size(h, C.byref(size)) == 0 and size.value > P.PANEL_NOALLOC_MAX_BYTES
    fake = C.c_void_p(0x100000)
    assert lib.panel_solve_noalloc(h, fake, fake, None, C.c_double(1.0), C.c_double(1e-10), 10, fake,
                                   None, None, fake, None, None) == P._binding.PANEL_EINVAL
    assert b"static scratch" in lib.panel_last_error()
    lib.panel_plan_destroy(h)


def test_tiling_defaults_and_validation(lib):
    import paper_1511_02166_amd as P
    from paper_1511_02166_amd._binding import panel_tiling
    EINVAL = P._binding.PANEL_EINVAL
    st, h = _plan(lib, [0, 129, 500], [0, 1, 2])
    t = panel_tiling()
    assert lib.panel_plan_get_tiling(h, C.byref(t)) == 0
    assert t.as_dict() == dict(wave_max_n1=320, persistent=0, wg_waves=0)
    for bad in ((321, 1, 0), (-1, 1, 0), (320, 2, 0), (320, 1, 6)):
        assert lib.panel_plan_set_tiling(h, C.byref(panel_tiling(*bad))) == EINVAL, bad
    assert lib.panel_plan_set_tiling(h, C.byref(panel_tiling(192, 0, 8))) == 0
    assert lib.panel_plan_get_tiling(h, C.byref(t)) == 0 and t.as_dict() == dict(wave_max_n1=192, persistent=0,
                                                                                   wg_waves=8)
    # a new wave limit needs the workspace re-initialised before factoring
    fake = C.c_void_p(0x100000)
    assert lib.panel_factor_solve(h, fake, C.c_double(1e-10), 10, fake, None) == EINVAL
    lib.panel_plan_destroy(h)


def test_formulation_switch_and_workspace(lib):
    # Hess-Smith keeps the tangential-velocity matrix: one more system-sized
    # section; unknown formulations are refused
    import paper_1511_02166_amd as P
    st, h = _plan(lib, [0, 257, 514], [0, 1, 3])
    s0 = C.c_size_t()
    assert lib.panel_workspace_size(h, C.byref(s0)) == 0
    assert lib.panel_plan_set_formulation(h, 7) == P._binding.PANEL_EINVAL
    assert lib.panel_plan_set_formulation(h, P.PANEL_HESS_SMITH) == 0
    s1 = C.c_size_t()
    assert lib.panel_workspace_size(h, C.byref(s1)) == 0
    assert s1.value - s0.value > 0.99 * 8 * 288 * (258 + 260)   # one more system-sized section
    d = (C.c_int64 * 9)()
    assert lib.panel_workspace_layout(h, 1, d) == 0 and d[8] > d[0]
    lib.panel_plan_destroy(h)


def test_ga_entry_points_validate_before_any_hip_call(lib):
    # B-spline contours: closure, gene map, sizes; GA step: population,
    # tournament size, probabilities, buffers; the uniform count
    import paper_1511_02166_amd as P
    EINVAL = P._binding.PANEL_EINVAL
    fake = C.c_void_p(0x100000)
    T = np.array([[1.0, 0.0], [0.5, 0.1], [0.0, 0.0], [0.5, -0.1], [1.0, 0.0]])
    tp = T.ctypes.data_as(C.c_void_p)
    gm = np.array([3, 7], dtype=np.int32)
    gp = gm.ctypes.data_as(C.c_void_p)
    assert lib.panel_bspline_nodes(4, 64, 5, 3, tp, 2, gp, fake, C.c_void_p(0x100004), None) == EINVAL  # unaligned
    assert lib.panel_bspline_nodes(4, 63, 5, 3, tp, 2, gp, fake, fake, None) == EINVAL    # odd N
    assert lib.panel_bspline_nodes(4, 64, 5, 5, tp, 2, gp, fake, fake, None) == EINVAL    # M < degree + 1
    assert lib.panel_bspline_nodes(4, 64, 5, 8, tp, 2, gp, fake, fake, None) == EINVAL    # degree > max
    open_T = T.copy()
    open_T[-1, 1] = 1e-3
    assert lib.panel_bspline_nodes(4, 64, 5, 3, open_T.ctypes.data_as(C.c_void_p), 2, gp, fake, fake,
                                   None) == EINVAL                                     # not closed
    for bad in ([1, 7], [3, 8], [3, 3]):   # gene on the trailing edge, out of range, repeated
        b = np.array(bad, dtype=np.int32)
        assert lib.panel_bspline_nodes(4, 64, 5, 3, tp, 2, b.ctypes.data_as(C.c_void_p), fake, fake,
                                       None) == EINVAL, bad
    n = C.c_int64()
    assert lib.panel_ga_uniform_count(2048, 4, C.byref(n)) == 0 and n.value == 1024 * 15 + 3 * 2048
    assert lib.panel_ga_uniform_count(7, 4, C.byref(n)) == EINVAL
    assert lib.panel_ga_uniform_count(8, 17, C.byref(n)) == EINVAL
    lo = np.zeros(2)
    hi = np.ones(2)
    lp, hp = lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p)
    f2 = C.c_void_p(0x200000)
    ok_args = dict(B=8, G=2, k=3, p_sel=0.7, p_mut=0.1, sigma=0.1)

    def step(**kw):
        a = dict(ok_args, **kw)
        gin = kw.get("gin", fake)
        return lib.panel_ga_step(a["B"], a["G"], a["k"], C.c_double(a["p_sel"]), C.c_double(a["p_mut"]),
                                 C.c_double(a["sigma"]), lp, hp, fake, gin, fake, f2, None, None)
    assert step(B=7) == EINVAL and step(B=0) == EINVAL
    assert step(G=1) == EINVAL and step(G=65) == EINVAL
    assert step(k=0) == EINVAL and step(k=17) == EINVAL
    assert step(p_sel=0.0) == EINVAL and step(p_sel=1.5) == EINVAL
    assert step(p_mut=-0.1) == EINVAL and step(sigma=float("nan")) == EINVAL
    assert step(gin=f2) == EINVAL   # in place
    hi_bad = np.array([1.0, -1.0])
    assert lib.panel_ga_step(8, 2, 3, C.c_double(0.7), C.c_double(0.1), C.c_double(0.1), lp,
                             hi_bad.ctypes.data_as(C.c_void_p), fake, fake, fake, f2, None, None) == EINVAL
    assert lib.panel_ga_init(8, 2, lp, hi_bad.ctypes.data_as(C.c_void_p), fake, f2, None) == EINVAL
    assert lib.panel_ga_record(8, 2, fake, fake, fake, 5, None, None, fake, fake, None) == EINVAL
