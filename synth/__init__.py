"""Seeded synthetic inputs for the batched panel-method workloads.

This module only draws random numbers and lays out closed-form test
geometries.  It holds none of the panel method's arithmetic (no influence
coefficients, no solve, no forces, no NACA section formula), so both the
CPU oracle and the GPU path may consume what it produces.

The workloads stand in for the genetic-algorithm population of the paper
(Sec. 2, GA steps 1-2; Sec. 3, Table 2 uses 4000 individuals of about 200
points): each individual is a NACA 4-digit section described by
(m, p, t), evaluated at one or more angles of attack.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEG = math.pi / 180.0


@dataclass
class Workload:
    """A batch of airfoils: NACA parameters, panel counts and angles."""

    name: str
    m: np.ndarray          # max camber, fraction of chord   [B]
    p: np.ndarray          # camber position, fraction       [B]
    t: np.ndarray          # thickness, fraction of chord    [B]
    n_panels: np.ndarray   # panels per airfoil (even)       [B] int32
    alpha: list            # angles of attack in rad, one array per airfoil
    closed_te: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return int(self.m.shape[0])

    def node_offsets(self) -> np.ndarray:
        """Offsets into the packed node array: airfoil b owns N_b + 1 nodes."""
        off = np.zeros(self.B + 1, dtype=np.int32)
        off[1:] = np.cumsum(self.n_panels.astype(np.int64) + 1)
        return off

    def alpha_offsets(self) -> np.ndarray:
        off = np.zeros(self.B + 1, dtype=np.int32)
        off[1:] = np.cumsum([len(a) for a in self.alpha])
        return off

    def alpha_flat(self) -> np.ndarray:
        return np.concatenate([np.asarray(a, dtype=np.float64) for a in self.alpha])

    def mpt(self) -> np.ndarray:
        """Packed [B, 3] array of (m, p, t)."""
        return np.stack([self.m, self.p, self.t], axis=1).astype(np.float64)

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return Workload(self.name + "[sub]", self.m[idx].copy(), self.p[idx].copy(),
                        self.t[idx].copy(), self.n_panels[idx].copy(),
                        [self.alpha[i] for i in idx], self.closed_te, dict(self.meta))


def _naca_draws(rng, B):
    # Fixed draw order: camber, camber position, thickness.
    m = rng.uniform(0.0, 0.06, B)
    p = rng.uniform(0.2, 0.6, B)
    t = rng.uniform(0.08, 0.18, B)
    return m, p, t


# The seeded workloads: name -> (seed, airfoils).  Draws per workload, in a
# fixed order: camber, camber position, thickness, then the angles, then the
# panel counts.
WORKLOADS = {
    "naca128": (1, 32),        # 32 airfoils, N = 128, alpha = 4 deg
    "ga2048": (2, 2048),       # GA population: 2048 airfoils, N = 256, alpha ~ U[-4, 12] deg
    "uneven4096": (3, 4096),   # 4096 airfoils, N = 16 U{6..32}, alpha in {0, 4, 8, 12} deg
    "adjoint1024": (4, 1024),  # 1024 airfoils, N = 256, alpha = 6 deg
    "large256": (5, 256),      # 256 airfoils, N = 1024, alpha = -2, 0, ..., 12 deg
}


def workload(name: str, B: int | None = None) -> Workload:
    """One of the seeded workloads in WORKLOADS (NACA 4-digit sections,
    cosine spacing, closed trailing edge).  ``B`` truncates the batch to its
    first B airfoils (same draws)."""
    if name not in WORKLOADS:
        raise ValueError(f"unknown workload {name!r} (known: {', '.join(WORKLOADS)})")
    seed, full = WORKLOADS[name]
    rng = np.random.default_rng(seed)
    m, p, t = _naca_draws(rng, full)
    if name == "naca128":
        n = np.full(full, 128, np.int32)
        alpha = [np.array([4.0 * DEG]) for _ in range(full)]
    elif name == "ga2048":
        a = rng.uniform(-4.0, 12.0, full) * DEG
        n = np.full(full, 256, np.int32)
        alpha = [np.array([x]) for x in a]
    elif name == "uneven4096":
        n = (16 * rng.integers(6, 33, full)).astype(np.int32)
        alpha = [np.array([0.0, 4.0, 8.0, 12.0]) * DEG for _ in range(full)]
    elif name == "adjoint1024":
        n = np.full(full, 256, np.int32)
        alpha = [np.array([6.0 * DEG]) for _ in range(full)]
    else:   # large256
        n = np.full(full, 1024, np.int32)
        alpha = [np.arange(-2.0, 12.01, 2.0) * DEG for _ in range(full)]
    w = Workload(name, m, p, t, n, alpha, True, {"seed": seed})
    if B is not None and B < full:
        w = w.subset(np.arange(B))
        w.name = f"{name}[:{B}]"
    return w


def random_workload(seed: int, B: int, n_choices=(16, 32, 48, 64), k_max=3) -> Workload:
    """Small mixed batch for parity tests: uneven N and K, seeded."""
    rng = np.random.default_rng(seed)
    m, p, t = _naca_draws(rng, B)
    n = rng.choice(np.asarray(n_choices, dtype=np.int32), B).astype(np.int32)
    ks = rng.integers(1, k_max + 1, B)
    alpha = [rng.uniform(-4.0, 12.0, int(k)) * DEG for k in ks]
    return Workload(f"rand{seed}", m, p, t, n, alpha, True, {"seed": seed})


# ---------------------------------------------------------------------------
# Closed-form test geometries (node lists only; counter-clockwise, starting
# at the trailing-edge node, last node equal to the first).
# ---------------------------------------------------------------------------

def circle_nodes(N: int, R: float = 0.5, cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """Nodes R(cos th_k, sin th_k), th_k = 2 pi k / N, k = 0..N (node N = node 0)."""
    k = np.arange(N + 1)
    th = 2.0 * np.pi * k / N
    xy = np.stack([cx + R * np.cos(th), cy + R * np.sin(th)], axis=1)
    xy[N] = xy[0]
    return xy


def joukowski_nodes(N: int, b: float = 0.25, mu: complex = complex(-0.02, 0.03)) -> np.ndarray:
    """Nodes z = zeta + b^2/zeta on the circle through zeta = b centred at mu.

    Node k sits at zeta_k = mu + a exp(i(delta + 2 pi k / N)), delta = arg(b - mu),
    so node 0 is the cusped trailing edge z = 2b.
    """
    a = abs(b - mu)
    delta = np.angle(b - mu)
    k = np.arange(N + 1)
    zeta = mu + a * np.exp(1j * (delta + 2.0 * np.pi * k / N))
    zeta[0] = b
    z = zeta + b * b / zeta
    xy = np.stack([z.real, z.imag], axis=1)
    xy[N] = xy[0]
    return xy


def pack_nodes(node_lists) -> tuple[np.ndarray, np.ndarray]:
    """Pack a list of [N_b+1, 2] node arrays into (xy_flat, node_offsets)."""
    off = np.zeros(len(node_lists) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(x) for x in node_lists])
    xy = np.concatenate([np.asarray(x, dtype=np.float64).reshape(-1, 2) for x in node_lists])
    return np.ascontiguousarray(xy.reshape(-1)), off


def joukowski_batch(seed: int, B: int, n_panels) -> tuple[np.ndarray, np.ndarray]:
    """B cambered Joukowski sections with seeded circle centres (airfoil-like,
    cusped trailing edge), packed as (xy_flat, node_offsets).  ``n_panels`` is
    an int or a sequence of B even ints."""
    rng = np.random.default_rng(seed)
    ns = np.broadcast_to(np.asarray(n_panels), (B,))
    nodes = []
    for b in range(B):
        mu = complex(-rng.uniform(0.01, 0.06), rng.uniform(0.0, 0.06))
        nodes.append(joukowski_nodes(int(ns[b]), 0.25, mu))
    return pack_nodes(nodes)


# ---------------------------------------------------------------------------
# Genetic-algorithm inputs: the genome's control-point template and bounds,
# and the uniform random numbers each generation consumes.
# ---------------------------------------------------------------------------

@dataclass
class GaProblem:
    """Control-point template [M, 2] of a closed contour (first = last = the
    trailing edge (1, 0)), the coordinates the genes set (indices into the
    flattened template) and per-gene bounds."""

    template: np.ndarray
    gene_map: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    degree: int = 3

    @property
    def G(self) -> int:
        return int(self.gene_map.size)


def ga_problem(m: int = 6, degree: int = 3) -> GaProblem:
    """m control points per surface at fixed cosine-spaced abscissae (the last
    of each at x = 0, so the leading edge has a vertical tangent); the genes
    are their ordinates: upper surface in [0.01, 0.16], lower in
    [-0.10, -0.01]."""
    X = 0.5 * (1.0 + np.cos(np.pi * np.arange(1, m + 1) / m))
    X[-1] = 0.0
    M = 2 * m + 2
    T = np.zeros((M, 2))
    T[0] = T[-1] = (1.0, 0.0)
    T[1:m + 1, 0] = X
    T[m + 1:2 * m + 1, 0] = X[::-1]
    gene_map = np.array([2 * i + 1 for i in range(1, 2 * m + 1)], dtype=np.int32)
    lo = np.concatenate([np.full(m, 0.01), np.full(m, -0.10)])
    hi = np.concatenate([np.full(m, 0.16), np.full(m, -0.01)])
    return GaProblem(T, gene_map, lo, hi, degree)


def ga_uniforms(seed: int, count: int, rows: int = 1) -> np.ndarray:
    """Uniform [0, 1) draws, [rows, count]."""
    return np.random.default_rng(seed).random((rows, count))
