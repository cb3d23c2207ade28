"""Pins for the CPU FP64 oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to something fixed outside it:
adaptive quadrature of the defining integral, LAPACK, closed-form potential
flows (circular cylinder, lifting cylinder, Joukowski section), exact
symmetries and invariances of the discrete system, textbook NACA ordinates,
and the lift values printed in the paper (Sec. 2, Fig. 2 tables).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DEG = math.pi / 180.0


# ---------------------------------------------------------------------------
# NACA section helper
# ---------------------------------------------------------------------------

def test_naca_textbook_thickness_ordinates():
    # NACA 0012 half-thickness (classic open trailing edge), percent chord,
    # from the standard tabulated ordinates: x=0.25 -> 5.941, x=0.5 -> 5.294,
    # x=1.0 -> 0.126.
    N = 48  # cosine stations s=16 -> x=0.25, s=12 -> x=0.5, s=0 -> x=1
    xy = oracle.naca4(0.0, 0.4, 0.12, N, closed_te=False)
    assert abs(xy[16, 0] - 0.25) < 1e-14 and abs(xy[12, 0] - 0.5) < 1e-14
    assert abs(xy[16, 1] - 0.05941) < 6e-6
    assert abs(xy[12, 1] - 0.05294) < 6e-6
    assert abs(xy[0, 1] - 0.00126) < 6e-6
    # lower surface mirrors
    assert abs(xy[N - 16, 1] + 0.05941) < 6e-6


def test_naca_structure_closed_symmetric():
    N = 64
    xy = oracle.naca4(0.0, 0.4, 0.12, N, closed_te=True)
    assert np.all(xy[N // 2] == 0.0)              # leading edge at the origin
    assert np.all(xy[N] == xy[0])                 # P_N = P_0 bitwise
    assert abs(xy[0, 0] - 1.0) < 1e-15 and abs(xy[0, 1]) < 1e-15
    k = np.arange(1, N // 2)
    assert np.all(xy[k, 0] == xy[N - k, 0])       # exact mirror
    assert np.all(xy[k, 1] == -xy[N - k, 1])
    assert np.all(xy[1:N // 2, 1] > 0)            # upper surface first (CCW)


def test_naca_camber_line_values():
    # Upper/lower pairs straddle the camber line: their mean is (x, y_c(x)).
    # For p = 0.5, y_c(0.5) = m and, worked by hand, y_c(0.25) = y_c(0.75) = 0.75 m.
    N, m, p, t = 48, 0.05, 0.5, 0.12
    xy = oracle.naca4(m, p, t, N, closed_te=False)
    for s, x, yc in ((12, 0.5, m), (16, 0.25, 0.75 * m), (8, 0.75, 0.75 * m)):
        up, lo = xy[s], xy[N - s]
        assert abs(0.5 * (up[0] + lo[0]) - x) < 1e-14
        assert abs(0.5 * (up[1] + lo[1]) - yc) < 1e-14
    # at x = p the camber slope vanishes, so the thickness is vertical: 2 y_t
    assert abs((xy[12, 1] - xy[N - 12, 1]) - 2 * 0.05294) < 1.2e-5
    assert abs(xy[12, 0] - xy[N - 12, 0]) < 1e-15


def test_naca_jacobian_vs_central_differences():
    N, h = 32, 1e-6
    th = np.array([0.04, 0.35, 0.13])
    J = oracle.naca4_jacobian(*th, N)
    for q in range(3):
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd = (oracle.naca4(*tp, N) - oracle.naca4(*tm, N)) / (2 * h)
        assert np.max(np.abs(J[:, :, q] - fd)) < 1e-8


# ---------------------------------------------------------------------------
# Influence coefficients against the defining integral
# ---------------------------------------------------------------------------

def _quad_g(xy, j, i):
    p0, p1 = xy[i], xy[i + 1]
    m = 0.5 * (xy[j] + xy[j + 1])
    L = np.hypot(*(p1 - p0))

    def f(tau):
        s = p0 + tau * (p1 - p0)
        return -1.0 / (2 * np.pi) * np.log(np.hypot(*(m - s))) * L

    pts = [0.5] if i == j else None
    val, _ = scipy.integrate.quad(f, 0.0, 1.0, points=pts, epsabs=1e-15, epsrel=1e-13, limit=200)
    return val


@pytest.mark.parametrize("geom", ["naca", "joukowski", "random"])
def test_g_entries_match_quadrature(geom):
    N = 16
    if geom == "naca":
        xy = oracle.naca4(0.03, 0.4, 0.15, N)
    elif geom == "joukowski":
        xy = synth.joukowski_nodes(N)
    else:
        rng = np.random.default_rng(5)
        th = np.sort(rng.uniform(0, 2 * np.pi, N))
        r = 0.5 + 0.1 * rng.uniform(size=N)
        xy = np.stack([r * np.cos(th), 0.3 * r * np.sin(th)], 1)
        xy = np.vstack([xy, xy[:1]])
    M, _ = oracle.assemble(xy, [0.0])
    for j in range(N):
        for i in range(N):
            q = _quad_g(xy, j, i)
            assert abs(M[j, i] - q) <= 1e-12 * max(1.0, abs(q)) + 1e-14, (j, i, M[j, i], q)


def test_g_endpoint_swap_and_translation_invariance():
    # The integral does not depend on which end the panel starts from, nor on
    # a rigid translation of the whole contour.
    xy = oracle.naca4(0.02, 0.4, 0.12, 24)
    M, _ = oracle.assemble(xy, [0.0])
    M2, _ = oracle.assemble(xy + np.array([3.25, -1.5]), [0.0])
    assert np.max(np.abs(M - M2)) < 1e-13
    rev = xy[::-1].copy()  # reversed node order: panel i becomes panel N-1-i
    Mr, _ = oracle.assemble(rev, [0.0])
    N = 24
    Mr_back = Mr[:N, :N][::-1, ::-1]
    assert np.max(np.abs(M[:N, :N] - Mr_back)) < 1e-14


def test_system_structure_and_rhs():
    N = 20
    xy = oracle.naca4(0.02, 0.4, 0.12, N)
    al = np.array([0.1, -0.05])
    M, R = oracle.assemble(xy, al, vinf=2.0)
    assert np.all(M[:N, N] == -1.0)
    kutta = np.zeros(N + 1)
    kutta[0] = kutta[N - 1] = 1.0
    assert np.all(M[N] == kutta)
    mid = 0.5 * (xy[:-1] + xy[1:])
    for k, a in enumerate(al):
        expect = -2.0 * (mid[:, 1] * np.cos(a) - mid[:, 0] * np.sin(a))
        assert np.max(np.abs(R[k, :N] - expect)) < 1e-15
        assert R[k, N] == 0.0


# ---------------------------------------------------------------------------
# LU against LAPACK, the Kutta-substituted system of the paper
# ---------------------------------------------------------------------------

def test_lu_hand_example():
    A = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 10.0]])
    LU, piv, info = oracle.lu(A)
    assert info == 0 and list(piv) == [2, 2, 2]
    # worked by hand: P A = L U with rows (7 8 10), (1 2 3), (4 5 6)
    Lm = np.array([[1, 0, 0], [1 / 7, 1, 0], [4 / 7, 0.5, 1]])
    Um = np.array([[7, 8, 10], [0, 2 - 8 / 7, 3 - 10 / 7], [0, 0, 6 - 40 / 7 - 0.5 * (3 - 10 / 7)]])
    assert np.allclose(np.tril(LU, -1) + np.eye(3), Lm, atol=1e-15)
    assert np.allclose(np.triu(LU), Um, atol=1e-14)


def test_lu_zero_pivot_info():
    A = np.array([[0.0, 1.0], [0.0, 2.0]])
    _, _, info = oracle.lu(A)
    assert info == 1


@pytest.mark.parametrize("N", [32, 128])
def test_lu_matches_lapack(N):
    xy = oracle.naca4(0.04, 0.3, 0.1, N)
    M, R = oracle.assemble(xy, [0.07, 0.2])
    LU, piv, info = oracle.lu(M)
    assert info == 0
    lu_s, piv_s = scipy.linalg.lu_factor(M)
    assert np.array_equal(piv, piv_s.astype(np.int32))
    assert np.max(np.abs(LU - lu_s)) < 1e-12 * np.max(np.abs(lu_s))
    X = oracle.lu_solve(LU, piv, R)
    for k in range(2):
        xs = scipy.linalg.lu_solve((lu_s, piv_s), R[k])
        assert np.max(np.abs(X[k] - xs)) <= 1e-10 * np.max(np.abs(xs))
        res = np.max(np.abs(M @ X[k] - R[k])) / (np.max(np.abs(M).sum(1)) * np.max(np.abs(X[k])))
        assert res < 1e-15 * (N + 1)
    w = np.random.default_rng(0).standard_normal(N + 1)
    y = oracle.lu_solve_t(LU, piv, w)
    ys = scipy.linalg.lu_solve((lu_s, piv_s), w, trans=1)
    assert np.max(np.abs(y - ys)) <= 1e-10 * np.max(np.abs(ys))


def test_bordered_equals_kutta_substituted_system():
    # The paper's form (Sec. 2): n unknowns gamma_0..gamma_{n-2}, C with
    # gamma_{n-1} = -gamma_0 substituted.  Solved with LAPACK independently.
    N = 64
    xy = oracle.naca4(0.03, 0.45, 0.14, N)
    a = 5 * DEG
    M, R = oracle.assemble(xy, [a])
    G = M[:N, :N]
    A = np.zeros((N, N))
    A[:, 0] = G[:, 0] - G[:, N - 1]
    A[:, 1:N - 1] = G[:, 1:N - 1]
    A[:, N - 1] = -1.0
    z = np.linalg.solve(A, R[0, :N])
    gam = np.concatenate([z[:N - 1], [-z[0]]])
    res = oracle.solve_airfoil(xy, [a])
    assert np.max(np.abs(res["gamma"][0] - gam)) < 1e-11 * np.max(np.abs(gam))


# ---------------------------------------------------------------------------
# Closed-form flows
# ---------------------------------------------------------------------------

def test_cylinder_cp_second_order():
    # Non-lifting circular cylinder: Cp = 1 - 4 sin^2(theta) on the surface.
    errs = []
    for N in (64, 128, 256):
        xy = synth.circle_nodes(N, R=0.5)
        r = oracle.solve_airfoil(xy, [0.0], chord=1.0)
        thm = 2 * np.pi * (np.arange(N) + 0.5) / N
        errs.append(np.max(np.abs(r["cp"][0] - (1 - 4 * np.sin(thm) ** 2))))
        assert abs(r["cl"][0]) < 1e-12
    assert errs[0] < 4e-3 and errs[2] < 3e-4
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5   # O(N^-2)


def test_lifting_cylinder_kutta_point():
    # Kutta point at theta = 0: u = -2 vinf [sin(theta - a) + sin a],
    # Cl = 4 pi sin a with chord 2R.
    a = 5 * DEG
    errs = []
    for N in (64, 256):
        xy = synth.circle_nodes(N, R=0.5)
        r = oracle.solve_airfoil(xy, [a], chord=1.0)
        errs.append(abs(r["cl"][0] - 4 * np.pi * np.sin(a)))
        thm = 2 * np.pi * (np.arange(N) + 0.5) / N
        u = -2 * (np.sin(thm - a) + np.sin(a))
        assert np.max(np.abs(r["gamma"][0] - u)) < 40.0 / N ** 2 + 1e-3 * (N == 64)
    assert errs[1] < 3e-4 and errs[0] / errs[1] > 8


def test_joukowski_circulation_converges():
    # Joukowski section: Gamma = -4 pi a vinf sin(alpha + beta), CCW-positive,
    # beta = -arg(b - mu).
    b, mu = 0.25, complex(-0.02, 0.03)
    a_rad = abs(b - mu)
    beta = -np.angle(b - mu)
    alpha = 4 * DEG
    gam_exact = -4 * np.pi * a_rad * np.sin(alpha + beta)
    errs = []
    for N in (64, 128, 256):
        xy = synth.joukowski_nodes(N, b, mu)
        r = oracle.solve_airfoil(xy, [alpha], chord=1.0)
        gam = -0.5 * r["cl"][0]        # Cl = -2 Gamma / (vinf c), c = 1
        errs.append(abs(gam - gam_exact) / abs(gam_exact))
    assert errs[0] < 1.5e-2 and errs[2] < 1e-3
    assert errs[0] / errs[2] > 8


def test_symmetric_section_zero_lift_and_odd_in_alpha():
    xy = oracle.naca4(0.0, 0.4, 0.12, 256)
    r0 = oracle.solve_airfoil(xy, [0.0])
    assert abs(r0["cl"][0]) < 1e-13
    r = oracle.solve_airfoil(xy, [3 * DEG, -3 * DEG])
    assert abs(r["cl"][0] + r["cl"][1]) < 1e-12
    assert r["cl"][0] > 0


def test_thin_section_limit():
    a = 4 * DEG
    ratios = []
    for t in (0.04, 0.02, 0.01):
        xy = oracle.naca4(0.0, 0.4, t, 256)
        r = oracle.solve_airfoil(xy, [a])
        ratios.append(r["cl"][0] / (2 * np.pi * np.sin(a)))
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] - 1.0 < 0.015


def test_scale_translation_rotation_invariance():
    N = 96
    xy = oracle.naca4(0.03, 0.35, 0.11, N)
    a = 6 * DEG
    base = oracle.solve_airfoil(xy, [a])
    # uniform scaling with the chord scaled along: same gamma, same Cl
    s = 2.7
    r = oracle.solve_airfoil(xy * s + np.array([0.3, -0.8]), [a], chord=s)
    assert np.max(np.abs(r["gamma"] - base["gamma"])) < 1e-10
    assert abs(r["cl"][0] - base["cl"][0]) < 1e-12
    assert abs(r["cl_p"][0] - base["cl_p"][0]) < 1e-11
    # rotating the section by beta (CCW) equals reducing the incidence by beta
    beta = 2.5 * DEG
    Rm = np.array([[np.cos(beta), -np.sin(beta)], [np.sin(beta), np.cos(beta)]])
    r = oracle.solve_airfoil(xy @ Rm.T, [a + beta])
    assert abs(r["cl"][0] - base["cl"][0]) < 1e-12
    assert abs(r["cl_p"][0] - base["cl_p"][0]) < 1e-11


def test_lifting_cylinder_pressure_lift():
    # The pressure integral of the lifting cylinder (Kutta point at theta = 0,
    # chord 2R = 1) tends to the Kutta-Joukowski value 4 pi sin a at second
    # order: pins the sign, the outward normal and e_L in Cl_p.
    a = 5 * DEG
    errs = []
    for N in (64, 128, 256):
        r = oracle.solve_airfoil(synth.circle_nodes(N, R=0.5), [a], chord=1.0)
        errs.append(abs(r["cl_p"][0] - 4 * np.pi * np.sin(a)))
    assert errs[2] < 2e-4
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_freestream_speed_and_chord_scaling():
    # The system is linear in vinf (right-hand side only): gamma scales with
    # vinf, while Cp = 1 - (gamma/vinf)^2, Cl and Cl_p do not change.  The
    # chord c only normalises the two lift coefficients (both ~ 1/c).
    xy = oracle.naca4(0.03, 0.35, 0.11, 96)
    a = [6 * DEG, -2 * DEG]
    base = oracle.solve_airfoil(xy, a)
    v = 2.5
    r = oracle.solve_airfoil(xy, a, vinf=v)
    assert np.max(np.abs(r["gamma"] - v * base["gamma"])) < 1e-12 * v * np.max(np.abs(base["gamma"])) * 10
    assert np.max(np.abs(r["cp"] - base["cp"])) < 1e-12
    assert np.max(np.abs(r["cl"] - base["cl"])) < 1e-13
    assert np.max(np.abs(r["cl_p"] - base["cl_p"])) < 1e-13
    c = 0.37
    r = oracle.solve_airfoil(xy, a, vinf=v, chord=c)
    assert np.max(np.abs(c * r["cl"] - base["cl"])) < 1e-13
    assert np.max(np.abs(c * r["cl_p"] - base["cl_p"])) < 1e-13
    assert np.max(np.abs(r["gamma"] - v * base["gamma"])) < 1e-11


def test_batch_packing_matches_single_airfoil_calls():
    # The batch entry point packs every airfoil's outputs at offsets derived
    # from (N_b, K_b); per-airfoil chords and a common vinf.  Each slice must
    # equal the one-airfoil call bit for bit (same arithmetic, same order),
    # with the offsets recomputed here from the panel and angle counts.
    rng = np.random.default_rng(41)
    Ns = [16, 40, 6, 64, 30]
    Ks = [1, 3, 4, 2, 1]
    nodes = [oracle.naca4(rng.uniform(0, 0.06), rng.uniform(0.2, 0.6), rng.uniform(0.08, 0.18), n)
             for n in Ns]
    xy, noff = synth.pack_nodes(nodes)
    alphas = [rng.uniform(-4, 12, k) * DEG for k in Ks]
    aoff = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int32)
    chord = rng.uniform(0.5, 2.0, len(Ns))
    vinf = 1.7
    r = oracle.solve_batch(xy, noff, np.concatenate(alphas), aoff, chord=chord, vinf=vinf, nthreads=2)
    assert np.all(r["info"] == 0)
    so = 0
    for b, (N, K) in enumerate(zip(Ns, Ks)):
        assert noff[b + 1] - noff[b] == N + 1
        one = oracle.solve_airfoil(nodes[b], alphas[b], vinf=vinf, chord=chord[b])
        assert np.array_equal(r["gamma"][so:so + N * K], one["gamma"].reshape(-1))
        assert np.array_equal(r["cp"][so:so + N * K], one["cp"].reshape(-1))
        assert np.array_equal(r["cl"][aoff[b]:aoff[b + 1]], one["cl"])
        assert np.array_equal(r["cl_p"][aoff[b]:aoff[b + 1]], one["cl_p"])
        so += N * K
    assert so == r["gamma"].size


def test_panel_refinement_cauchy_and_pressure_lift_agree():
    cls, clps = [], []
    for N in (128, 256, 512):
        xy = oracle.naca4(0.02, 0.4, 0.12, N)
        r = oracle.solve_airfoil(xy, [4 * DEG])
        cls.append(r["cl"][0])
        clps.append(r["cl_p"][0])
    d1, d2 = abs(cls[1] - cls[0]), abs(cls[2] - cls[1])
    assert d2 < d1
    assert abs(cls[2] - clps[2]) < abs(cls[0] - clps[0])
    assert abs(cls[2] - clps[2]) < 2e-3


def test_paper_lift_tables():
    g = json.load(open(os.path.join(GOLDEN, "paper_cl_tables.json")))
    t1 = g["lift_vs_alpha"]
    xy = oracle.naca4(0.02, 0.4, 0.12, t1["panels"], closed_te=False, uniform=True)
    r = oracle.solve_airfoil(xy, np.deg2rad(t1["alpha_deg"]))
    assert np.max(np.abs(r["cl"] - np.array(t1["cl"]))) < 1e-3
    t3 = g["lift_vs_panels"]
    got = []
    for N in t3["panels"]:
        if N > 1000:
            continue  # the 2000-panel point runs in the slow suite
        xy = oracle.naca4(0.02, 0.4, 0.12, N, closed_te=False, uniform=True)
        got.append(oracle.solve_airfoil(xy, [0.0])["cl"][0])
    ref = [c for N, c in zip(t3["panels"], t3["cl"]) if N <= 1000]
    assert np.max(np.abs(np.array(got) - np.array(ref))) < 5e-4


# ---------------------------------------------------------------------------
# Gradient pins
# ---------------------------------------------------------------------------

def _cl(xy, a, chord=1.0):
    return oracle.solve_airfoil(xy, [a], chord=chord)["cl"][0]


def test_gradient_vs_central_differences():
    N, a, h = 32, 6 * DEG, 1e-6
    xy = oracle.naca4(0.03, 0.4, 0.12, N)
    g, dcla = oracle.cl_gradient(xy, a, with_alpha=True)
    fd = np.zeros_like(xy)
    for k in range(N + 1):
        for c in range(2):
            p, m = xy.copy(), xy.copy()
            p[k, c] += h
            m[k, c] -= h
            fd[k, c] = (_cl(p, a) - _cl(m, a)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd))
    fda = (_cl(xy, a + h) - _cl(xy, a - h)) / (2 * h)
    assert abs(dcla - fda) < 1e-7


def test_gradient_discrete_invariants():
    N, a = 128, 4 * DEG
    xy = oracle.naca4(0.02, 0.45, 0.15, N)
    g, dcla = oracle.cl_gradient(xy, a, with_alpha=True)
    cl = _cl(xy, a)
    scale = np.max(np.abs(g))
    assert np.max(np.abs(g.sum(0))) < 1e-9 * scale                  # translation
    assert abs((xy * g).sum() - cl) < 1e-9 * max(1, abs(cl))       # scaling, chord fixed
    perp = np.stack([-xy[:, 1], xy[:, 0]], 1)
    assert abs((perp * g).sum() + dcla) < 1e-9 * abs(dcla)          # rotation


@pytest.mark.slow
def test_paper_lift_table_2000_panels():
    g = json.load(open(os.path.join(GOLDEN, "paper_cl_tables.json")))["lift_vs_panels"]
    i = g["panels"].index(2000)
    xy = oracle.naca4(0.02, 0.4, 0.12, 2000, closed_te=False, uniform=True)
    assert abs(oracle.solve_airfoil(xy, [0.0])["cl"][0] - g["cl"][i]) < 5e-4


def _weighted_forces(xy, a, dcl, dcp, vinf=1.0, chord=1.0):
    r = oracle.solve_airfoil(xy, [a], vinf=vinf, chord=chord)
    return dcl * r["cl"][0] + float(np.dot(dcp, r["cp"][0]))


def test_force_gradient_vs_central_differences():
    # d/dP of dcl Cl + sum_i dcp_i Cp_i against central differences of the
    # oracle's own forward solve (vinf and chord away from 1).
    N, a, h, vinf, chord = 24, 5 * DEG, 1e-6, 1.6, 0.8
    xy = oracle.naca4(0.04, 0.35, 0.13, N)
    rng = np.random.default_rng(5)
    dcp = rng.standard_normal(N)
    dcl = 0.7
    g = oracle.force_gradient(xy, a, dcl, dcp, vinf=vinf, chord=chord)
    fd = np.zeros_like(xy)
    for k in range(N + 1):
        for c in range(2):
            p, m = xy.copy(), xy.copy()
            p[k, c] += h
            m[k, c] -= h
            fd[k, c] = (_weighted_forces(p, a, dcl, dcp, vinf, chord) -
                        _weighted_forces(m, a, dcl, dcp, vinf, chord)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd))
    # without pressure weights it is the lift gradient
    assert np.max(np.abs(oracle.force_gradient(xy, a, 1.0, None, vinf, chord) -
                         oracle.cl_gradient(xy, a, vinf, chord))) == 0.0


def test_force_gradient_pressure_invariants():
    # Cp_i is invariant under translation and uniform scaling of the nodes
    # (gamma is), so its node gradient sums to zero and is orthogonal to P;
    # a rotation by beta equals an incidence change of -beta.
    N, a = 96, 3 * DEG
    xy = oracle.naca4(0.02, 0.45, 0.14, N)
    dcp = np.random.default_rng(6).standard_normal(N)
    g = oracle.force_gradient(xy, a, 0.0, dcp)
    scale = np.max(np.abs(g))
    assert np.max(np.abs(g.sum(0))) < 1e-9 * scale
    assert abs((xy * g).sum()) < 1e-9 * scale * np.max(np.abs(xy))
    h = 1e-6
    dfa = (_weighted_forces(xy, a + h, 0.0, dcp) - _weighted_forces(xy, a - h, 0.0, dcp)) / (2 * h)
    perp = np.stack([-xy[:, 1], xy[:, 0]], 1)
    assert abs((perp * g).sum() + dfa) < 1e-6 * max(1.0, abs(dfa))
