"""Pins of the genetic-algorithm oracle (oracle/panel_oracle_ga.c) against
what the paper and the mathematics fix, independently of the oracle's own
code (Sec. 2: B-spline genome, tournament selection with probabilities
p, p(1-p), ..., one-point crossover, mutation).
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle
import synth


def _knots(M, d):
    # clamped, uniform interior knots
    inner = np.arange(1, M - d) / (M - d)
    return np.concatenate([np.zeros(d + 1), inner, np.ones(d + 1)])


# ---- B-spline contour ------------------------------------------------------------


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_bspline_point_matches_scipy(d):
    # SciPy evaluates the same clamped B-spline from its basis functions
    # (a different algorithm from de Boor's point recursion)
    rng = np.random.default_rng(d)
    M = 11
    Q = rng.standard_normal((M, 2))
    spl = BSpline(_knots(M, d), Q, d)
    for u in np.concatenate([rng.random(50), [0.0, 0.5, 1.0 - 1e-15]]):
        got = oracle.bspline_point(Q, d, u)
        assert np.max(np.abs(got - spl(u))) < 1e-14, (u, got, spl(u))
    # u = 1 (SciPy extrapolates the last span there): the last control point
    assert np.array_equal(oracle.bspline_point(Q, d, 1.0), Q[-1])
    assert np.array_equal(oracle.bspline_point(Q, d, 0.0), Q[0])


def test_bspline_degree_one_is_the_control_polygon():
    rng = np.random.default_rng(3)
    M = 7
    Q = rng.standard_normal((M, 2))
    for i in range(M - 1):
        for f in (0.0, 0.25, 0.5, 0.75):
            u = (i + f) / (M - 1)
            want = (1 - f) * Q[i] + f * Q[i + 1]
            assert np.max(np.abs(oracle.bspline_point(Q, 1, u) - want)) < 1e-15 * np.max(np.abs(Q))


@pytest.mark.parametrize("d", [2, 3, 4])
def test_bspline_linear_precision(d):
    # control points on a line at the Greville abscissae reproduce the line
    # with x(u) = u (partition of unity and linear reproduction)
    M = 12
    t = _knots(M, d)
    xi = np.array([t[i + 1:i + d + 1].mean() for i in range(M)])
    Q = np.stack([xi, 0.3 * xi - 0.7], axis=1)
    for u in np.linspace(0, 1, 37):
        p = oracle.bspline_point(Q, d, u)
        assert abs(p[0] - u) < 1e-15 and abs(p[1] - (0.3 * u - 0.7)) < 1e-15


def test_bspline_contour_parameters_and_symmetry():
    # nodes: u_0 = 0, u_{N/2} = 1/2, u_N = 1, clustered at both ends and the
    # middle; node N is node 0; mirrored genes give a mirrored contour
    N = 64
    u = np.array([oracle.bspline_param(k, N) for k in range(N + 1)])
    assert u[0] == 0.0 and u[N // 2] == 0.5 and u[N] == 1.0
    assert np.all(np.diff(u) > 0)
    du = np.diff(u)
    assert du[0] < du[N // 4] / 10 and du[N // 2] < du[N // 4] / 10
    assert np.allclose(u + u[::-1], 1.0, atol=1e-16)
    prob = synth.ga_problem(6)
    up = np.array([0.02, 0.05, 0.08, 0.09, 0.07, 0.04])
    g = np.concatenate([up, -up[::-1]])   # lower surface listed from the leading edge
    P = oracle.bspline_nodes(prob.template, prob.gene_map, g, 3, N)[0]
    assert np.array_equal(P[N], P[0]) and np.array_equal(P[0], [1.0, 0.0])
    assert np.max(np.abs(P[::-1, 0] - P[:, 0])) < 1e-15
    assert np.max(np.abs(P[::-1, 1] + P[:, 1])) < 1e-15
    # the middle node is the leading edge (leftmost, on the chord line for a
    # mirrored genome), and the contour runs counter-clockwise
    assert np.argmin(P[:, 0]) == N // 2 and abs(P[N // 2, 1]) < 1e-16
    area = 0.5 * np.sum(P[:-1, 0] * P[1:, 1] - P[1:, 0] * P[:-1, 1])
    assert area > 0


# ---- generation operators ------------------------------------------------------


def test_ga_init_within_bounds():
    prob = synth.ga_problem(6)
    u = synth.ga_uniforms(1, prob.G, rows=50)
    u[0] = 0.0
    u[1] = 0.5
    g = oracle.ga_init(prob.lo, prob.hi, u)
    assert np.all(g >= prob.lo) and np.all(g < prob.hi)
    assert np.array_equal(g[0], prob.lo)
    assert np.allclose(g[1], 0.5 * (prob.lo + prob.hi), rtol=0, atol=1e-16)


def test_ga_fitness_mean_and_lethal_cases():
    aoff = np.array([0, 1, 3, 4, 6], dtype=np.int32)
    ld = np.array([20.0, 10.0, 30.0, np.nan, 5.0, np.inf])
    info = np.array([0, 0, 0, 0], dtype=np.int32)
    f = oracle.ga_fitness(aoff, ld, info)
    assert f[0] == 20.0 and f[1] == 20.0 and f[2] == -np.inf and f[3] == -np.inf
    info[0] = 3
    assert oracle.ga_fitness(aoff, ld, info)[0] == -np.inf


def _draws(u, B):
    return np.minimum(np.floor(u * B).astype(int), B - 1)


def test_tournament_rank_frequencies():
    # P(selected = r-th best of the k drawn) = p (1-p)^r, the worst the rest
    B, G, k, p = 4096, 4, 4, 0.6
    rng = np.random.default_rng(5)
    fit = rng.permutation(B).astype(float)
    genome = np.tile(np.arange(B, dtype=float)[:, None], (1, G))   # genes name their individual
    per = oracle.ga_uniforms_per_generation(B, k)
    counts = np.zeros(k)
    for gen in range(6):
        u = synth.ga_uniforms(100 + gen, per)[0]
        _, tr = oracle.ga_step(genome, fit, u, k, p, 0.0, 0.0, np.zeros(G), np.ones(G))
        for q in range(B // 2):
            uq = u[q * (4 * k - 1):(q + 1) * (4 * k - 1)]
            for t, parent in ((0, tr[2 * q, 0]), (1, tr[2 * q, 1])):
                drawn = _draws(uq[t * (2 * k - 1):t * (2 * k - 1) + k], B)
                if len(set(drawn)) < k:
                    continue   # repeated draw: rank ambiguous
                assert parent in drawn
                counts[int(np.sum(fit[drawn] > fit[parent]))] += 1
    n = counts.sum()
    want = np.array([p * (1 - p) ** r for r in range(k - 1)] + [(1 - p) ** (k - 1)])
    sd = np.sqrt(n * want * (1 - want))
    assert np.all(np.abs(counts - n * want) < 5 * sd), (counts / n, want)


def test_tournament_special_cases():
    # k = 1: the drawn individual; p = 1: the best drawn (brute force)
    B, G = 50, 3
    rng = np.random.default_rng(6)
    fit = rng.standard_normal(B)
    genome = rng.standard_normal((B, G))
    lo, hi = np.full(G, -5.0), np.full(G, 5.0)
    for k, p in ((1, 0.7), (3, 1.0), (5, 1.0)):
        u = synth.ga_uniforms(7 + k, oracle.ga_uniforms_per_generation(B, k))[0]
        _, tr = oracle.ga_step(genome, fit, u, k, p, 0.0, 0.0, lo, hi)
        for q in range(B // 2):
            uq = u[q * (4 * k - 1):(q + 1) * (4 * k - 1)]
            for t in range(2):
                drawn = _draws(uq[t * (2 * k - 1):t * (2 * k - 1) + k], B)
                want = drawn[0] if k == 1 else drawn[np.argmax(fit[drawn])]
                assert tr[2 * q, t] == want and tr[2 * q + 1, 1 - t] == want


def test_crossover_and_mutation():
    B, G, k = 200, 12, 3
    prob = synth.ga_problem(6)
    genome = oracle.ga_init(prob.lo, prob.hi, synth.ga_uniforms(8, G, rows=B))
    fit = np.random.default_rng(9).standard_normal(B)
    u = synth.ga_uniforms(10, oracle.ga_uniforms_per_generation(B, k))[0]
    # no mutation: children are the two one-point crossovers of their parents
    out, tr = oracle.ga_step(genome, fit, u, k, 0.7, 0.0, 0.1, prob.lo, prob.hi)
    cuts = []
    for q in range(B // 2):
        a, b, c, m = tr[2 * q]
        assert tuple(tr[2 * q + 1]) == (b, a, c, -1) and m == -1 and 1 <= c <= G - 1
        assert np.array_equal(out[2 * q], np.concatenate([genome[a, :c], genome[b, c:]]))
        assert np.array_equal(out[2 * q + 1], np.concatenate([genome[b, :c], genome[a, c:]]))
        cuts.append(c)
    assert set(cuts) == set(range(1, G))
    # certain mutation: exactly one gene moves, by at most sigma (hi - lo),
    # and stays in bounds
    sigma = 0.1
    out1, tr1 = oracle.ga_step(genome, fit, u, k, 0.7, 1.0, sigma, prob.lo, prob.hi)
    assert np.array_equal(tr1[:, :3], tr[:, :3])
    for i in range(B):
        d = np.nonzero(out1[i] != out[i])[0]
        j = tr1[i, 3]
        assert 0 <= j < G and set(d) <= {j}
        assert abs(out1[i, j] - out[i, j]) <= sigma * (prob.hi[j] - prob.lo[j]) * (1 + 1e-15)
    assert np.all(out1 >= prob.lo) and np.all(out1 <= prob.hi)
    # mutation rate
    hits = 0
    for s in range(10):
        u = synth.ga_uniforms(20 + s, oracle.ga_uniforms_per_generation(B, k))[0]
        _, trm = oracle.ga_step(genome, fit, u, k, 0.7, 0.3, sigma, prob.lo, prob.hi)
        hits += np.sum(trm[:, 3] >= 0)
    n = 10 * B
    assert abs(hits - 0.3 * n) < 5 * np.sqrt(n * 0.21)


def test_ga_climbs_a_quadratic_fitness():
    # selection pressure: on f(g) = -sum ((g - g*) / (hi - lo))^2 the
    # population's best and mean improve well beyond random search
    B, k = 64, 4
    prob = synth.ga_problem(6)
    target = prob.lo + 0.37 * (prob.hi - prob.lo)
    rng_rows = synth.ga_uniforms(30, oracle.ga_uniforms_per_generation(B, k), rows=80)
    g = oracle.ga_init(prob.lo, prob.hi, synth.ga_uniforms(31, prob.G, rows=B))

    def f(x):
        return -np.sum(((x - target) / (prob.hi - prob.lo)) ** 2, axis=1)
    f0 = f(g)
    for gen in range(80):
        g, _ = oracle.ga_step(g, f(g), rng_rows[gen], k, 0.75, 0.3, 0.1, prob.lo, prob.hi)
    f1 = f(g)
    assert f1.max() > -0.02 and f1.mean() > 0.2 * f0.mean() and f1.max() > 5 * f0.max()
