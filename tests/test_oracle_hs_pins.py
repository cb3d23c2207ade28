"""Pins for the Hess-Smith branch of the CPU oracle (oracle/panel_oracle_hs.c).

The influence velocities are checked against adaptive quadrature of their
defining integrals, the whole method against closed-form potential flows
(circular cylinder with and without circulation, Joukowski section), exact
symmetries and invariances, the Kutta condition, and against the paper's own
stream-function scheme, whose lift it must approach as the panels shrink.
"""
import math

import numpy as np
import pytest
import scipy.integrate

import oracle
import synth

DEG = math.pi / 180.0
HS = "hess_smith"


def _quad_velocity(P0, P1, x):
    """(1/2pi) int_panel (x - s)/|x - s|^2 ds and its +90 degree turn."""
    h = np.asarray(P1) - np.asarray(P0)
    L = np.hypot(*h)

    def f(s, c):
        p = np.asarray(P0) + h * (s / L)
        d = np.asarray(x) - p
        return d[c] / (2 * np.pi * (d @ d))

    kw = dict(epsabs=1e-14, epsrel=1e-13, limit=400)
    sx = scipy.integrate.quad(f, 0.0, L, args=(0,), **kw)[0]
    sy = scipy.integrate.quad(f, 0.0, L, args=(1,), **kw)[0]
    return sx, sy, -sy, sx


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hs_influence_matches_quadrature(seed):
    rng = np.random.default_rng(seed)
    xy = oracle.naca4(0.04, 0.4, 0.12, 32)
    for _ in range(40):
        i = int(rng.integers(32))
        x = rng.uniform(-0.5, 1.5, 2)
        got = oracle.hs_influence(xy, i, x[0], x[1])
        ref = _quad_velocity(xy[i], xy[i + 1], x)
        assert np.max(np.abs(np.array(got) - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_hs_self_influence_is_the_fluid_side_limit():
    # at a panel's own midpoint: log(r1/r2) = 0 and the subtended angle pi,
    # the limit of the off-panel values as the point approaches from outside
    xy = oracle.naca4(0.02, 0.4, 0.12, 24)
    for i in (0, 5, 12, 23):
        m = 0.5 * (xy[i] + xy[i + 1])
        h = xy[i + 1] - xy[i]
        n = np.array([h[1], -h[0]]) / np.hypot(*h)   # outward normal
        self_v = np.array(oracle.hs_influence(xy, i, m[0], m[1], True))
        near = np.array(oracle.hs_influence(xy, i, *(m + 1e-9 * n)))
        assert np.max(np.abs(self_v - near)) < 1e-7
        assert abs(self_v[0] * n[0] + self_v[1] * n[1] - 0.5) < 1e-15   # half the source goes outward


def test_hs_cylinder_pressure():
    # Non-lifting circular cylinder: Cp = 1 - 4 sin^2(theta).  On a regular
    # polygon the constant-source panels reproduce it at the midpoints to
    # rounding.
    for N in (32, 64, 256):
        r = oracle.solve_airfoil(synth.circle_nodes(N, R=0.5), [0.0], formulation=HS)
        thm = 2 * np.pi * (np.arange(N) + 0.5) / N
        assert np.max(np.abs(r["cp"][0] - (1 - 4 * np.sin(thm) ** 2))) < 1e-9
        assert abs(r["cl"][0]) < 1e-12


def test_hs_lifting_cylinder():
    # Kutta point at theta = 0: u = -2 vinf [sin(theta - a) + sin a],
    # Cl = 4 pi sin a (chord 2R = 1); second-order convergence.
    a = 5 * DEG
    errs = []
    for N in (64, 128, 256):
        r = oracle.solve_airfoil(synth.circle_nodes(N, R=0.5), [a], formulation=HS)
        thm = 2 * np.pi * (np.arange(N) + 0.5) / N
        u = -2 * (np.sin(thm - a) + np.sin(a))
        assert np.max(np.abs(r["gamma"][0] - u)) < 20.0 / N ** 2
        errs.append(abs(r["cl"][0] - 4 * np.pi * np.sin(a)))
        assert abs(r["cl_p"][0] - 4 * np.pi * np.sin(a)) < 20.0 / N ** 2
    assert errs[2] < 2e-4 and errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_hs_joukowski_circulation():
    # Gamma = -4 pi a vinf sin(alpha + beta), Cl = -2 Gamma (c = 1 here).
    # The cusped trailing edge puts the two Kutta panels on top of each
    # other; constant-source panels converge there, but slowly (about
    # N^-0.8: 17% at N = 64, 2.2% at 1024), unlike the vortex-sheet scheme.
    b, mu = 0.25, complex(-0.02, 0.03)
    a_rad = abs(b - mu)
    beta = -np.angle(b - mu)
    alpha = 4 * DEG
    gam_exact = -4 * np.pi * a_rad * np.sin(alpha + beta)
    errs = []
    for N in (128, 256, 512):
        r = oracle.solve_airfoil(synth.joukowski_nodes(N, b, mu), [alpha], formulation=HS)
        errs.append(abs(-0.5 * r["cl"][0] - gam_exact) / abs(gam_exact))
    assert errs[2] < 0.05 and errs[0] > 1.5 * errs[1] > 2.25 * errs[2]


def test_hs_kutta_condition_and_symmetry():
    xy = oracle.naca4(0.0, 0.4, 0.12, 128)
    r0 = oracle.solve_airfoil(xy, [0.0], formulation=HS)
    assert abs(r0["cl"][0]) < 1e-13
    r = oracle.solve_airfoil(xy, [3 * DEG, -3 * DEG], formulation=HS)
    assert abs(r["cl"][0] + r["cl"][1]) < 1e-12 and r["cl"][0] > 0
    xy = oracle.naca4(0.04, 0.3, 0.1, 96)
    r = oracle.solve_airfoil(xy, [6 * DEG], formulation=HS)
    u = r["gamma"][0]
    assert abs(u[0] + u[-1]) < 1e-12 * np.max(np.abs(u))


def test_hs_invariances():
    N, a = 80, 5 * DEG
    xy = oracle.naca4(0.03, 0.35, 0.11, N)
    base = oracle.solve_airfoil(xy, [a], formulation=HS)
    s = 1.9
    r = oracle.solve_airfoil(xy * s + np.array([-0.4, 0.7]), [a], chord=s, formulation=HS)
    assert abs(r["cl"][0] - base["cl"][0]) < 1e-12 and abs(r["cl_p"][0] - base["cl_p"][0]) < 1e-12
    beta = 3 * DEG
    Rm = np.array([[np.cos(beta), -np.sin(beta)], [np.sin(beta), np.cos(beta)]])
    r = oracle.solve_airfoil(xy @ Rm.T, [a + beta], formulation=HS)
    assert abs(r["cl"][0] - base["cl"][0]) < 1e-12
    v = 2.2
    r = oracle.solve_airfoil(xy, [a], vinf=v, formulation=HS)
    assert np.max(np.abs(r["gamma"] - v * base["gamma"])) < 1e-12 * v * 10
    assert abs(r["cl"][0] - base["cl"][0]) < 1e-13


def test_hs_approaches_the_stream_function_scheme():
    # Two discretisations of the same potential flow: their lift coefficients
    # move together (first order in 1/N) as the panels shrink.
    d = []
    for N in (100, 200, 400):
        xy = oracle.naca4(0.02, 0.4, 0.12, N)
        a = oracle.solve_airfoil(xy, [4 * DEG], formulation=HS)["cl"][0]
        b = oracle.solve_airfoil(xy, [4 * DEG])["cl"][0]
        d.append(abs(a - b))
    assert d[0] > 1.7 * d[1] > 2.9 * d[2] and d[2] < 2e-3


def test_hs_batch_packing_matches_single_calls():
    rng = np.random.default_rng(8)
    Ns, Ks = [16, 40, 30], [2, 1, 3]
    nodes = [oracle.naca4(0.03, 0.4, 0.12, n) for n in Ns]
    xy, noff = synth.pack_nodes(nodes)
    alphas = [rng.uniform(-4, 12, k) * DEG for k in Ks]
    aoff = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int32)
    chord = np.array([0.8, 1.0, 1.3])
    r = oracle.solve_batch(xy, noff, np.concatenate(alphas), aoff, chord=chord, vinf=1.4, formulation=HS,
                           nthreads=2)
    so = 0
    for b in range(3):
        one = oracle.solve_airfoil(nodes[b], alphas[b], vinf=1.4, chord=chord[b], formulation=HS)
        assert np.array_equal(r["gamma"][so:so + Ns[b] * Ks[b]], one["gamma"].reshape(-1))
        assert np.array_equal(r["cl"][aoff[b]:aoff[b + 1]], one["cl"])
        so += Ns[b] * Ks[b]


def _hs_weighted(xy, a, dcl, dcp, vinf=1.0, chord=1.0):
    r = oracle.solve_airfoil(xy, [a], vinf=vinf, chord=chord, formulation=HS)
    return dcl * r["cl"][0] + float(np.dot(dcp, r["cp"][0]))


def test_hs_gradient_vs_central_differences():
    # d/dP of dcl Cl + sum dcp_j Cp_j (complex-step tangent-linear) against
    # central differences of the Hess-Smith forward solve
    N, a, h, vinf, chord = 20, 5 * DEG, 1e-6, 1.6, 0.8
    xy = oracle.naca4(0.04, 0.35, 0.13, N)
    dcp = np.random.default_rng(5).standard_normal(N)
    g = oracle.force_gradient(xy, a, 0.7, dcp, vinf, chord, formulation=HS)
    fd = np.zeros_like(xy)
    for k in range(N + 1):
        for c in range(2):
            p, m = xy.copy(), xy.copy()
            p[k, c] += h
            m[k, c] -= h
            fd[k, c] = (_hs_weighted(p, a, 0.7, dcp, vinf, chord) - _hs_weighted(m, a, 0.7, dcp, vinf, chord)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd))


def test_hs_gradient_invariants():
    # translation: gradients sum to zero; scaling with the chord fixed:
    # sum_k P_k . grad Cl = Cl and sum_k P_k . grad Cp_j = 0 (the surface speed
    # is scale invariant); rotation: sum_k P_k^perp . grad F = -dF/dalpha
    N, a = 40, 4 * DEG
    xy = oracle.naca4(0.02, 0.45, 0.14, N)
    dcp = np.random.default_rng(6).standard_normal(N)
    gl = oracle.force_gradient(xy, a, 1.0, None, formulation=HS)
    gp = oracle.force_gradient(xy, a, 0.0, dcp, formulation=HS)
    cl = oracle.solve_airfoil(xy, [a], formulation=HS)["cl"][0]
    for g in (gl, gp):
        assert np.max(np.abs(g.sum(0))) < 1e-9 * np.max(np.abs(g))
    assert abs((xy * gl).sum() - cl) < 1e-9
    assert abs((xy * gp).sum()) < 1e-9 * np.max(np.abs(gp))
    h = 1e-6
    dfa = (_hs_weighted(xy, a + h, 0.3, dcp) - _hs_weighted(xy, a - h, 0.3, dcp)) / (2 * h)
    g = 0.3 * gl + gp
    perp = np.stack([-xy[:, 1], xy[:, 0]], 1)
    assert abs((perp * g).sum() + dfa) < 1e-6 * max(1.0, abs(dfa))
