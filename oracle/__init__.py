"""CPU FP64 oracle for the batched 2-D panel method (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The product library never imports, links or calls it, and it
shares no code with the GPU path.  The arithmetic lives in plain C in
``panel_oracle.c`` (each function cites the passage of the paper it follows);
this module compiles it with gcc and marshals numpy arrays through ctypes.

Parity status per function (see the pins under ``tests/``):
  oracle_naca4          pinned (standard NACA 4-digit values, symmetry, LE/TE)
  oracle_g_entry        pinned (adaptive quadrature of the defining integral)
  oracle_assemble       pinned (entry-wise vs quadrature; Kutta row vs the
                        Kutta-substituted system of Sec. 2)
  oracle_lu / _solve    pinned (LAPACK getrf/getrs; hand-checked 3x3)
  oracle_lu_solve_t     pinned (LAPACK transposed solve)
  oracle_forces         pinned (cylinder Cp = 1 - 4 sin^2, lifting cylinder
                        Cl = 4 pi sin alpha, Joukowski circulation, symmetric
                        sections at zero incidence, the paper's C_L tables)
  oracle_cl_gradient    pinned (central differences, exact discrete
                        invariants: translation, scaling, rotation)
  oracle_force_gradient pinned (central differences of the oracle's Cp and
                        Cl; translation, scaling and rotation invariants of
                        Cp; equals oracle_cl_gradient without cp weights)
  oracle_hs_*           Hess-Smith formulation (panel_oracle_hs.c): pinned
                        (velocity integrals by quadrature, cylinder and lifting
                        cylinder, Joukowski circulation, symmetric sections,
                        invariances, convergence to the stream-function
                        scheme's limit)
  oracle_thwaites*      viscous correction (panel_oracle_bl.c): pinned
                        (stagnation flow exact, power-law edge flows at second
                        order, the circular cylinder's closed-form drag and
                        separation angle, symmetry, Reynolds scaling)
  oracle_bspline_*      B-spline contour of the genome (panel_oracle_ga.c):
                        pinned (SciPy's BSpline, a different algorithm; the
                        polyline at degree 1; linear precision at the
                        Greville abscissae; endpoint interpolation, mirror
                        symmetry)
  oracle_ga_*           genetic-algorithm operators (panel_oracle_ga.c):
                        pinned (tournament rank frequencies p(1-p)^r, the
                        special cases k = 1 and p = 1 by brute force,
                        crossover conservation, mutation bounds and rate,
                        convergence on a quadratic fitness)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "panel_oracle.c"), os.path.join(_HERE, "panel_oracle_grad.c"),
        os.path.join(_HERE, "panel_oracle_hs.c"), os.path.join(_HERE, "panel_oracle_bl.c"),
        os.path.join(_HERE, "panel_oracle_ga.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    srcs = [s for s in _SRC if os.path.exists(s)]
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or any(os.path.getmtime(s) > os.path.getmtime(_LIB)
                                           for s in _SRC if os.path.exists(s)):
            build()
        L = C.CDLL(_LIB)
        L.oracle_naca4.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, _dp]
        L.oracle_naca4.restype = None
        L.oracle_naca4_spaced.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                          C.c_int, _dp]
        L.oracle_naca4_spaced.restype = None
        L.oracle_g_entry.argtypes = [_dp, C.c_int, C.c_int]
        L.oracle_g_entry.restype = C.c_double
        L.oracle_assemble.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_double, _dp, _dp]
        L.oracle_assemble.restype = None
        L.oracle_lu.argtypes = [C.c_int, _dp, _ip]
        L.oracle_lu.restype = C.c_int
        L.oracle_lu_solve.argtypes = [C.c_int, _dp, _ip, C.c_int, _dp]
        L.oracle_lu_solve.restype = None
        L.oracle_lu_solve_t.argtypes = [C.c_int, _dp, _ip, _dp]
        L.oracle_lu_solve_t.restype = None
        L.oracle_forces.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                    _dp, _dp, _dp, _dp]
        L.oracle_forces.restype = None
        L.oracle_solve_airfoil.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_double, C.c_double,
                                           _dp, _dp, _dp, _dp]
        L.oracle_solve_airfoil.restype = C.c_int
        L.oracle_solve_batch.argtypes = [C.c_int, _ip, _dp, _ip, _dp, C.c_void_p, C.c_double,
                                         _dp, _dp, _dp, _dp, _ip, C.c_int]
        L.oracle_solve_batch.restype = C.c_int
        if hasattr(L, "oracle_cl_gradient"):
            L.oracle_cl_gradient.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_double,
                                             _dp, _dp]
            L.oracle_cl_gradient.restype = C.c_int
            L.oracle_naca4_jacobian.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int,
                                                C.c_int, _dp]
            L.oracle_naca4_jacobian.restype = None
            L.oracle_force_gradient.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_double,
                                                C.c_double, C.c_void_p, _dp]
            L.oracle_force_gradient.restype = C.c_int
        L.oracle_hs_influence.argtypes = [_dp, C.c_int, C.c_double, C.c_double, C.c_int] + \
            [C.POINTER(C.c_double)] * 4
        L.oracle_hs_influence.restype = None
        L.oracle_hs_assemble.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_double, _dp, _dp, _dp]
        L.oracle_hs_assemble.restype = None
        L.oracle_hs_forces.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, _dp, C.c_double, C.c_double,
                                       _dp, _dp, _dp, _dp]
        L.oracle_hs_forces.restype = None
        L.oracle_hs_solve_airfoil.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_double, C.c_double,
                                              _dp, _dp, _dp, _dp]
        L.oracle_hs_solve_airfoil.restype = C.c_int
        L.oracle_hs_solve_batch.argtypes = [C.c_int, _ip, _dp, _ip, _dp, C.c_void_p, C.c_double,
                                            _dp, _dp, _dp, _dp, _ip, C.c_int]
        L.oracle_hs_solve_batch.restype = C.c_int
        L.oracle_hs_force_gradient.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_double,
                                                C.c_double, C.c_void_p, _dp]
        L.oracle_hs_force_gradient.restype = C.c_int
        L.oracle_thwaites_surface.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp, _dp]
        L.oracle_thwaites_surface.restype = C.c_int
        L.oracle_thwaites.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, _dp, C.c_double, C.c_double,
                                      C.c_double, _dp, _dp, _ip]
        L.oracle_thwaites.restype = None
        L.oracle_bspline_point.argtypes = [C.c_int, C.c_int, _dp, C.c_double, _dp]
        L.oracle_bspline_point.restype = None
        L.oracle_bspline_param.argtypes = [C.c_int, C.c_int]
        L.oracle_bspline_param.restype = C.c_double
        L.oracle_bspline_nodes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _ip, _dp, _dp]
        L.oracle_bspline_nodes.restype = None
        L.oracle_ga_init.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.oracle_ga_init.restype = None
        L.oracle_ga_fitness.argtypes = [C.c_int, _ip, _dp, _ip, _dp]
        L.oracle_ga_fitness.restype = None
        L.oracle_ga_step.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                     _dp, _dp, _dp, _dp, _ip]
        L.oracle_ga_step.restype = None
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Single-airfoil helpers
# ---------------------------------------------------------------------------

def naca4(m, p, t, N, closed_te=True, uniform=False) -> np.ndarray:
    """Nodes [N+1, 2] of a NACA 4-digit section, cosine (or uniform-x) spacing."""
    if N % 2:
        raise ValueError("N must be even")
    xy = np.zeros(2 * (N + 1))
    lib().oracle_naca4_spaced(float(m), float(p), float(t), int(N), int(bool(closed_te)),
                              int(bool(uniform)), xy)
    return xy.reshape(N + 1, 2)


def g_entry(xy, j, i) -> float:
    return lib().oracle_g_entry(_f64(xy).reshape(-1), int(j), int(i))


def assemble(xy, alpha, vinf=1.0):
    """Bordered matrix M [(N+1),(N+1)] and right-hand sides R [K, N+1]."""
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    alpha = _f64(np.atleast_1d(alpha))
    K = alpha.size
    M = np.zeros((N + 1) * (N + 1))
    R = np.zeros((N + 1) * K)
    lib().oracle_assemble(N, xy, K, alpha, float(vinf), M, R)
    return M.reshape(N + 1, N + 1), R.reshape(K, N + 1)


def lu(A):
    """(LU, piv, info) of a square matrix with partial pivoting."""
    A = _f64(A).copy()
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib().oracle_lu(n, A.reshape(-1), piv)
    return A, piv, info


def lu_solve(LU, piv, Bm):
    """Solve with K right-hand sides given as rows of Bm [K, n]."""
    LU = _f64(LU)
    X = _f64(np.atleast_2d(Bm)).copy()
    n = LU.shape[0]
    lib().oracle_lu_solve(n, LU.reshape(-1), np.ascontiguousarray(piv, dtype=np.int32),
                          X.shape[0], X.reshape(-1))
    return X


def lu_solve_t(LU, piv, w):
    LU = _f64(LU)
    y = _f64(w).copy()
    lib().oracle_lu_solve_t(LU.shape[0], LU.reshape(-1), np.ascontiguousarray(piv, dtype=np.int32), y)
    return y


def forces(xy, alpha, X, vinf=1.0, chord=1.0):
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    alpha = _f64(np.atleast_1d(alpha))
    K = alpha.size
    X = _f64(np.atleast_2d(X))
    gamma = np.zeros(K * N)
    cp = np.zeros(K * N)
    cl = np.zeros(K)
    clp = np.zeros(K)
    lib().oracle_forces(N, xy, K, alpha, X.reshape(-1), float(vinf), float(chord), gamma, cp, cl, clp)
    return gamma.reshape(K, N), cp.reshape(K, N), cl, clp


FORMULATIONS = ("stream", "hess_smith")


def solve_airfoil(xy, alpha, vinf=1.0, chord=1.0, formulation="stream"):
    """Whole pipeline for one airfoil: dict(gamma[K,N], cp[K,N], cl[K], cl_p[K], info).

    ``gamma`` is the tangential surface speed at the panel midpoints (for the
    stream-function scheme it equals the sheet strength)."""
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    alpha = _f64(np.atleast_1d(alpha))
    K = alpha.size
    gamma = np.zeros(K * N)
    cp = np.zeros(K * N)
    cl = np.zeros(K)
    clp = np.zeros(K)
    fn = {"stream": lib().oracle_solve_airfoil, "hess_smith": lib().oracle_hs_solve_airfoil}[formulation]
    info = fn(N, xy, K, alpha, float(vinf), float(chord), gamma, cp, cl, clp)
    return dict(gamma=gamma.reshape(K, N), cp=cp.reshape(K, N), cl=cl, cl_p=clp, info=info)


def solve_batch(xy_flat, node_off, alpha_flat, alpha_off, chord=None, vinf=1.0, nthreads=0,
                formulation="stream"):
    """Batch in the packed layout of the GPU library (see panel_oracle.c)."""
    node_off = np.ascontiguousarray(node_off, dtype=np.int32)
    alpha_off = np.ascontiguousarray(alpha_off, dtype=np.int32)
    B = node_off.size - 1
    Ns = np.diff(node_off) - 1
    Ks = np.diff(alpha_off)
    tot = int(np.sum(Ns.astype(np.int64) * Ks))
    gamma = np.zeros(tot)
    cp = np.zeros(tot)
    cl = np.zeros(int(alpha_off[-1]))
    clp = np.zeros(int(alpha_off[-1]))
    info = np.zeros(B, dtype=np.int32)
    ch = None
    if chord is not None:
        chord = _f64(chord)
        ch = chord.ctypes.data_as(C.c_void_p)
    fn = {"stream": lib().oracle_solve_batch, "hess_smith": lib().oracle_hs_solve_batch}[formulation]
    used = fn(B, node_off, _f64(xy_flat).reshape(-1), alpha_off, _f64(alpha_flat), ch, float(vinf), gamma, cp, cl,
              clp, info, int(nthreads))
    return dict(gamma=gamma, cp=cp, cl=cl, cl_p=clp, info=info, threads=used)


def hs_influence(xy, i, x, y, self_point=False):
    """Hess-Smith velocities at (x, y) of panel i: unit source (sx, sy), unit
    counter-clockwise vortex (wx, wy)."""
    out = [C.c_double() for _ in range(4)]
    lib().oracle_hs_influence(_f64(xy).reshape(-1), int(i), float(x), float(y), int(bool(self_point)),
                              *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def hs_assemble(xy, alpha, vinf=1.0):
    """Hess-Smith system: M [(N+1),(N+1)], right-hand sides R [K, N+1] and the
    tangential-velocity matrix Mt [N, N+1]."""
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    alpha = _f64(np.atleast_1d(alpha))
    K = alpha.size
    M = np.zeros((N + 1) * (N + 1))
    R = np.zeros((N + 1) * K)
    Mt = np.zeros((N + 1) * (N + 1))
    lib().oracle_hs_assemble(N, xy, K, alpha, float(vinf), M, R, Mt)
    return M.reshape(N + 1, N + 1), R.reshape(K, N + 1), Mt.reshape(N + 1, N + 1)[:N]


def thwaites_surface(ds, U, nu):
    """One boundary-layer surface: (theta, lambda, index of the first
    separated station or len(U))."""
    ds, U = _f64(ds), _f64(U)
    th = np.zeros(U.size)
    lm = np.zeros(U.size)
    sep = lib().oracle_thwaites_surface(int(U.size), ds, U, float(nu), th, lm)
    return th, lm, int(sep)


def thwaites(xy, alpha, u, cl, re, vinf=1.0, chord=1.0):
    """Viscous correction of one airfoil from its surface speeds u [K, N] and
    lift cl [K]: dict(cd[K], ld[K], sep[K, 2]) (separation panel of the upper
    and lower layer, -1 if attached to the trailing edge)."""
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    alpha = _f64(np.atleast_1d(alpha))
    K = alpha.size
    cd = np.zeros(K)
    ld = np.zeros(K)
    sep = np.zeros(2 * K, dtype=np.int32)
    lib().oracle_thwaites(N, xy, K, alpha, _f64(u).reshape(-1), _f64(np.atleast_1d(cl)), float(vinf),
                          float(chord), float(re), cd, ld, sep)
    return dict(cd=cd, ld=ld, sep=sep.reshape(K, 2))


def cl_gradient(xy, alpha, vinf=1.0, chord=1.0, with_alpha=False):
    """dCl/dP for all N+1 nodes (Cl by circulation, chord held fixed): [N+1, 2].

    With ``with_alpha`` also returns dCl/dalpha."""
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    g = np.zeros(2 * (N + 1))
    da = np.zeros(1)
    info = lib().oracle_cl_gradient(N, xy, float(alpha), float(vinf), float(chord), g, da)
    if info != 0:
        raise RuntimeError(f"oracle gradient failed, info={info}")
    if with_alpha:
        return g.reshape(N + 1, 2), float(da[0])
    return g.reshape(N + 1, 2)


def force_gradient(xy, alpha, dcl=1.0, dcp=None, vinf=1.0, chord=1.0, formulation="stream"):
    """d/dP of dcl * Cl + sum_i dcp[i] Cp_i for one angle: [N+1, 2]."""
    xy = _f64(xy).reshape(-1)
    N = xy.size // 2 - 1
    g = np.zeros(2 * (N + 1))
    w = None
    if dcp is not None:
        w = _f64(dcp).reshape(-1)
        if w.size != N:
            raise ValueError("dcp must hold one value per panel")
    fn = {"stream": lib().oracle_force_gradient, "hess_smith": lib().oracle_hs_force_gradient}[formulation]
    info = fn(N, xy, float(alpha), float(vinf), float(chord), float(dcl),
              None if w is None else w.ctypes.data_as(C.c_void_p), g)
    if info != 0:
        raise RuntimeError(f"oracle gradient failed, info={info}")
    return g.reshape(N + 1, 2)


def naca4_jacobian(m, p, t, N, closed_te=True) -> np.ndarray:
    """d(node coordinates)/d(m, p, t): [N+1, 2, 3]."""
    J = np.zeros(2 * (N + 1) * 3)
    lib().oracle_naca4_jacobian(float(m), float(p), float(t), int(N), int(bool(closed_te)), J)
    return J.reshape(N + 1, 2, 3)


def workload_nodes(w):
    """Oracle-side NACA nodes for a synth.Workload: (xy_flat, node_offsets)."""
    parts = [naca4(w.m[b], w.p[b], w.t[b], int(w.n_panels[b]), w.closed_te) for b in range(w.B)]
    xy = np.concatenate([q.reshape(-1) for q in parts])
    return xy, w.node_offsets()


# ---------------------------------------------------------------------------
# Genetic algorithm (Sec. 2): B-spline genome and the generation operators
# ---------------------------------------------------------------------------

def bspline_point(Q, degree, u):
    """Point of the clamped uniform B-spline with control points Q [M, 2] at u."""
    Q = _f64(Q).reshape(-1)
    out = np.zeros(2)
    lib().oracle_bspline_point(Q.size // 2, int(degree), Q, float(u), out)
    return out


def bspline_param(k, N):
    return lib().oracle_bspline_param(int(k), int(N))


def bspline_nodes(template, gene_map, genome, degree, N):
    """Contour nodes [B, N+1, 2] of the genomes [B, G]."""
    template = _f64(template).reshape(-1)
    genome = _f64(np.atleast_2d(genome))
    B, G = genome.shape
    gm = np.ascontiguousarray(gene_map, dtype=np.int32)
    xy = np.zeros(B * 2 * (N + 1))
    lib().oracle_bspline_nodes(B, int(N), template.size // 2, int(degree), G, template, gm, genome.reshape(-1), xy)
    return xy.reshape(B, N + 1, 2)


def ga_uniforms_per_generation(B, k):
    """Uniforms one generation consumes: (B/2)(4k - 1) for the pairs, 3 per child."""
    return (B // 2) * (4 * k - 1) + 3 * B


def ga_init(lo, hi, u):
    lo, hi = _f64(lo), _f64(hi)
    u = _f64(np.atleast_2d(u))
    B, G = u.shape
    out = np.zeros(B * G)
    lib().oracle_ga_init(B, G, lo, hi, u.reshape(-1), out)
    return out.reshape(B, G)


def ga_fitness(alpha_off, ld, info):
    alpha_off = np.ascontiguousarray(alpha_off, dtype=np.int32)
    B = alpha_off.size - 1
    out = np.zeros(B)
    lib().oracle_ga_fitness(B, alpha_off, _f64(ld), np.ascontiguousarray(info, dtype=np.int32), out)
    return out


def ga_step(genome, fitness, u, k, p_sel, p_mut, sigma, lo, hi):
    """Next generation [B, G] and its trace [B, 4] (parents, cut, mutated gene)."""
    genome = _f64(genome)
    B, G = genome.shape
    u = _f64(u).reshape(-1)
    if u.size < ga_uniforms_per_generation(B, k):
        raise ValueError("too few uniforms for one generation")
    out = np.zeros(B * G)
    trace = np.zeros(4 * B, dtype=np.int32)
    lib().oracle_ga_step(B, G, int(k), float(p_sel), float(p_mut), float(sigma), _f64(lo), _f64(hi),
                         _f64(fitness), genome.reshape(-1), u, out, trace)
    return out.reshape(B, G), trace.reshape(B, 4)
