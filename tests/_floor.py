"""Measured FP64 parity floor of one airfoil's system (CPU test helper).

Two correct FP64 solutions of the same panel system differ by an amount set
by the system's conditioning, not by any mistake.  This helper measures that
spread for one airfoil, from the oracle alone:

  (a) the oracle's own LU against LAPACK's getrf/getrs on the same matrix
      (a different, equally stable, elimination order);
  (b) the oracle's LU on the matrix with every influence entry moved by one
      unit in the last place (seeded random direction), which stands for a
      different but correctly rounded evaluation of the entries' logarithms
      and arctangents;
  (c) the oracle's LU on the matrix whose influence entries come from a
      second, equivalent closed form of the same panel integral, written
      here in numpy with the host's log and atan2: global coordinates, the
      difference of the two arctangents folded into the angle the panel
      subtends, log|m - P|^2 per node.  Where a far-field entry is a small
      difference of large terms, two correct evaluations differ by a few
      ulp of those terms, not of the entry, and (b) misses that.

Each solution is reduced to (gamma, Cp, Cl, Cl_p) by the oracle's forces and
compared with the oracle's reference through the relative metrics the parity
tests use; the floor of a quantity is the largest of the three spreads.  The GPU
evaluates its entries to within a few ulp of the oracle's and factors in yet
another order, so its distance to the oracle is expected within a small
multiple of this floor (FLOOR_FACTOR).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

import oracle

# The GPU's entries are within about 4 ulp of the oracle's (library log to
# 2 ulp, atan2 to 3 ulp, a different but equivalent closed form), i.e. up to
# four times the one-ulp perturbation of (b); a further factor 2 covers the
# different elimination order on top of it.
FLOOR_FACTOR = 8.0


def metrics(gamma, cp, cl, cl_p, ref):
    """Relative errors with the parity tests' normalisation (quantities that
    cross zero are measured against max(1, |reference|))."""
    rg, rcp, rcl, rclp = ref
    return dict(
        gamma=float(np.max(np.abs(gamma - rg)) / max(1.0, np.max(np.abs(rg)))),
        cp=float(np.max(np.abs(cp - rcp)) / max(1.0, np.max(np.abs(rcp)))),
        cl=float(np.max(np.abs(cl - rcl) / np.maximum(1.0, np.abs(rcl)))),
        cl_p=float(np.max(np.abs(cl_p - rclp) / np.maximum(1.0, np.abs(rclp)))),
    )


def second_closed_form(P):
    """Influence block G [N, N] of the panel integral, evaluated as
    -(1/(4 pi L)) [(d1.h) log|d1|^2 - (d2.h) log|d2|^2 - 2 L^2 + 2 (d1 x d2) theta]
    with d1 = m_j - P_i, d2 = m_j - P_{i+1}, h = P_{i+1} - P_i and theta the
    angle the panel subtends at m_j; diagonal (L/2pi)(1 - log(L/2))."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 2)
    N = P.shape[0] - 1
    m = 0.5 * (P[:-1] + P[1:])
    h = P[1:] - P[:-1]
    L2 = (h ** 2).sum(1)
    L = np.sqrt(L2)
    d1 = m[:, None, :] - P[None, :-1, :]
    d2 = m[:, None, :] - P[None, 1:, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        l1 = np.log((d1 ** 2).sum(-1))
        l2 = np.log((d2 ** 2).sum(-1))
        dot1 = (d1 * h[None]).sum(-1)
        cr = d1[..., 0] * d2[..., 1] - d1[..., 1] * d2[..., 0]
        th = np.arctan2(cr, (d1 * d2).sum(-1))
        G = -(1.0 / (4.0 * np.pi)) / L[None, :] * (dot1 * l1 - (dot1 - L2[None, :]) * l2 - 2.0 * L2[None, :]
                                                   + 2.0 * cr * th)
    d = np.arange(N)
    G[d, d] = L / (2.0 * np.pi) * (1.0 - np.log(0.5 * L))
    return G


def measured_floor(xy, alpha, vinf=1.0, chord=1.0, seed=0) -> dict:
    """Floor of e_gamma, e_Cp, e_Cl, e_Cl_p for one airfoil (nodes [N+1, 2])."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    M, R = oracle.assemble(xy, alpha, vinf)
    LU, piv, info = oracle.lu(M)
    if info != 0:
        raise RuntimeError(f"oracle LU failed (info {info})")
    X0 = oracle.lu_solve(LU, piv, R)
    ref = oracle.forces(xy, alpha, X0, vinf, chord)

    # (a) LAPACK on the same matrix
    X1 = scipy.linalg.lu_solve(scipy.linalg.lu_factor(M), R.T).T
    # (b) one-ulp perturbation of every influence entry
    rng = np.random.default_rng(seed)
    Mp = M.copy()
    G = Mp[:-1, :-1]
    up = rng.random(G.shape) < 0.5
    Mp[:-1, :-1] = np.where(up, np.nextafter(G, np.inf), np.nextafter(G, -np.inf))
    LUp, pivp, infop = oracle.lu(Mp)
    if infop != 0:
        raise RuntimeError(f"oracle LU of the perturbed matrix failed (info {infop})")
    X2 = oracle.lu_solve(LUp, pivp, R)
    # (c) the second closed form of the influence entries
    Mc = M.copy()
    Mc[:-1, :-1] = second_closed_form(xy)
    LUc, pivc, infoc = oracle.lu(Mc)
    if infoc != 0:
        raise RuntimeError(f"oracle LU of the second-form matrix failed (info {infoc})")
    X3 = oracle.lu_solve(LUc, pivc, R)

    floor = {}
    for X in (X1, X2, X3):
        e = metrics(*oracle.forces(xy, alpha, X, vinf, chord), ref)
        for k, v in e.items():
            floor[k] = max(floor.get(k, 0.0), v)
    return floor
