"""Pins for the viscous correction of the CPU oracle (oracle/panel_oracle_bl.c):
Thwaites' method on prescribed edge-speed profiles with closed-form answers,
the circular cylinder's closed-form drag and separation angle, symmetry and
the exact Reynolds-number scaling.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize

import oracle
import synth

DEG = math.pi / 180.0


def test_stagnation_flow_is_exact():
    # U = a s: theta^2 = 0.075 nu / a and lambda = 0.075 at every station
    a, nu = 3.0, 1e-5
    s = np.cumsum(np.random.default_rng(1).uniform(0.01, 0.03, 40))
    ds = np.diff(np.concatenate([[0.0], s]))
    th, lm, sep = oracle.thwaites_surface(ds, a * s, nu)
    assert sep == 40
    assert np.max(np.abs(th ** 2 / (0.075 * nu / a) - 1)) < 1e-12
    assert np.max(np.abs(lm - 0.075)) < 1e-12


@pytest.mark.parametrize("m", [0.5, 2.0])
def test_power_law_edge_flow_converges(m):
    # U = s^m: theta^2 = 0.45 nu s^(1-m) / (5m + 1), lambda = 0.45 m / (5m + 1)
    nu = 1e-4
    errs = []
    for n in (200, 400, 800):
        s = np.linspace(0, 1, n + 1)[1:]
        ds = np.full(n, 1.0 / n)
        th, lm, _ = oracle.thwaites_surface(ds, s ** m, nu)
        ref = 0.45 * nu * s ** (1 - m) / (5 * m + 1)
        sel = slice(n // 4, n - 1)   # away from the start and the one-sided end
        errs.append(max(np.max(np.abs(th[sel] ** 2 / ref[sel] - 1)),
                        np.max(np.abs(lm[sel] - 0.45 * m / (5 * m + 1)))))
    assert errs[2] < 1e-4 and errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def _cylinder_closed_form():
    def I5(p):
        if p < 0.5:
            return scipy.integrate.quad(lambda t: np.sin(t) ** 5, 0, p, epsrel=1e-14)[0]
        c = np.cos(p)
        return 8 / 15 - c + 2 / 3 * c ** 3 - c ** 5 / 5

    def lam(p):
        return 0.45 * np.cos(p) * I5(p) / np.sin(p) ** 6

    def ell(x):
        return 0.22 + 1.57 * x - 1.8 * x * x if x >= 0 else 0.22 + 1.402 * x + 0.018 * x / (x + 0.107)

    ps = scipy.optimize.brentq(lambda p: lam(p) + 0.09, 1.0, 2.5, xtol=1e-14)
    val = scipy.integrate.quad(lambda p: 4 * np.sin(p) ** 5 * ell(lam(p)) / np.sqrt(0.225 * I5(p)), 0, ps,
                               limit=400)[0]
    return ps, np.sqrt(2) * val


def test_cylinder_drag_and_separation_closed_form():
    # Edge speed U = 2 vinf sin(phi) from the front stagnation point: Thwaites'
    # integral in closed form gives separation at phi_s (lambda = -0.09) and
    # Cd sqrt(Re_D) as a quadrature of the closed-form shear (both sides).
    # Fed with the Hess-Smith surface speed (exact at a regular polygon's
    # midpoints) the discrete correction converges to both.
    ps, cdre = _cylinder_closed_form()
    assert abs(np.degrees(ps) - 103.11) < 0.01
    re = 1e5
    errs = []
    for N in (128, 256, 512):
        xy = synth.circle_nodes(N, R=0.5)
        r = oracle.solve_airfoil(xy, [0.0], formulation="hess_smith")
        bl = oracle.thwaites(xy, [0.0], r["gamma"], r["cl"], re)
        errs.append(abs(bl["cd"][0] * np.sqrt(re) / cdre - 1))
        ju, jl = bl["sep"][0]
        th_mid = 2 * np.pi * (np.arange(N) + 0.5) / N
        phi_u = np.pi - th_mid[ju]            # front stagnation point at theta = pi
        assert abs(phi_u - ps) < 1.5 * 2 * np.pi / N
        assert ju + jl == N - 1                # mirror-symmetric separation
    assert errs[2] < 1e-3 and errs[0] > errs[2]


def test_symmetry_and_reynolds_scaling():
    xy = oracle.naca4(0.0, 0.4, 0.12, 200)
    r = oracle.solve_airfoil(xy, [3 * DEG, -3 * DEG, 0.0])
    bl = oracle.thwaites(xy, [3 * DEG, -3 * DEG, 0.0], r["gamma"], r["cl"], 1e6)
    assert abs(bl["cd"][0] - bl["cd"][1]) < 1e-12 * bl["cd"][0]
    assert bl["sep"][0][0] == 199 - bl["sep"][1][1] if bl["sep"][0][0] >= 0 else bl["sep"][1][1] == -1
    assert bl["cd"][2] > 0 and abs(bl["ld"][2]) < 1e-9
    bl2 = oracle.thwaites(xy, [3 * DEG, -3 * DEG, 0.0], r["gamma"], r["cl"], 4e6)
    assert np.max(np.abs(bl2["cd"] * 2 - bl["cd"]) / bl["cd"]) < 1e-13   # cd ~ Re^-1/2
    assert np.array_equal(bl2["sep"], bl["sep"])
    assert np.allclose(bl["ld"][:2], r["cl"][:2] / bl["cd"][:2], rtol=1e-15)
