"""GPU parity of the genetic algorithm (Sec. 2) against its CPU oracle
(oracle/panel_oracle_ga.c), through the C ABI.

Index work (tournament picks, crossover positions, mutated genes, history
slots) must agree exactly; so must the genomes, whose only arithmetic
(lo + (hi - lo) u, and the mutation step) is evaluated in the same order
without contraction on both sides.  Contour nodes differ only by the
rounding of cos and of the basis recurrence (a few ulp); fitness by the
panel solve's own tolerance.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
DEG = math.pi / 180.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda") if dtype is None else \
        torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("N,degree,m", [(64, 3, 6), (256, 3, 6), (1024, 2, 9), (130, 5, 12)])
def test_bspline_nodes_match_oracle(N, degree, m):
    import torch
    import paper_1511_02166_amd as P
    _say(f"B-spline contours N={N}, degree={degree}, {2 * m} genes")
    prob = synth.ga_problem(m, degree)
    B = 64
    genome = oracle.ga_init(prob.lo, prob.hi, synth.ga_uniforms(N + degree, prob.G, rows=B))
    xy = torch.empty(2 * B * (N + 1), dtype=torch.float64, device="cuda")
    P.panel_bspline_nodes(B, N, prob.template, degree, prob.gene_map, _dev(genome), xy)
    torch.cuda.synchronize()
    got = xy.cpu().numpy().reshape(B, N + 1, 2)
    ref = oracle.bspline_nodes(prob.template, prob.gene_map, genome, degree, N)
    e = np.max(np.abs(got - ref))
    _say(f"  max |node difference| {e:.2e}")
    assert e < 1e-14
    assert np.array_equal(got[:, N], got[:, 0]) and np.array_equal(got[:, 0], np.tile([1.0, 0.0], (B, 1)))


def test_bspline_nodes_general_template():
    # free control points, genes on both coordinates, degree 4
    import torch
    import paper_1511_02166_amd as P
    _say("B-spline contours, general template")
    rng = np.random.default_rng(44)
    M, d, N, B = 20, 4, 200, 16
    T = rng.standard_normal((M, 2))
    T[-1] = T[0]
    gene_map = rng.choice(np.arange(2, 2 * M - 2), size=24, replace=False).astype(np.int32)
    genome = rng.standard_normal((B, 24))
    xy = torch.empty(2 * B * (N + 1), dtype=torch.float64, device="cuda")
    P.panel_bspline_nodes(B, N, T, d, gene_map, _dev(genome), xy)
    torch.cuda.synchronize()
    got = xy.cpu().numpy().reshape(B, N + 1, 2)
    ref = oracle.bspline_nodes(T, gene_map, genome, d, N)
    assert np.max(np.abs(got - ref)) < 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_ga_init_and_fitness_match_oracle():
    import torch
    import paper_1511_02166_amd as P
    _say("GA init and fitness")
    prob = synth.ga_problem(6)
    B = 500
    u = synth.ga_uniforms(3, prob.G, rows=B)
    g = torch.empty(B, prob.G, dtype=torch.float64, device="cuda")
    P.panel_ga_init(B, prob.G, prob.lo, prob.hi, _dev(u), g)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), oracle.ga_init(prob.lo, prob.hi, u))
    # fitness over uneven angle counts with lethal cases
    Ks = np.array([1, 3, 2, 1, 4, 2])
    aoff = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int32)
    noff = (np.arange(Ks.size + 1) * 65).astype(np.int32)
    s = P.PanelSolver(noff, aoff, 0)
    rng = np.random.default_rng(4)
    ld = rng.uniform(-20, 80, aoff[-1])
    ld[aoff[2] + 1] = np.nan
    ld[aoff[4] + 3] = np.inf
    info = np.array([0, 0, 0, 5, 0, -1], dtype=np.int32)
    fit = torch.empty(Ks.size, dtype=torch.float64, device="cuda")
    P.panel_ga_fitness(s.plan, s.ws, _dev(ld), _dev(info), fit)
    torch.cuda.synchronize()
    f = fit.cpu().numpy()
    ref = oracle.ga_fitness(aoff, ld, info)
    assert np.array_equal(f, ref)
    assert np.isneginf(f[[2, 3, 4, 5]]).all() and np.isfinite(f[:2]).all()


@pytest.mark.parametrize("B,G,k,p_sel,p_mut", [(2048, 12, 4, 0.75, 0.2), (2, 2, 1, 0.5, 1.0), (64, 7, 16, 1.0, 0.0),
                                               (1000, 64, 3, 0.3, 0.5)])
def test_ga_step_matches_oracle(B, G, k, p_sel, p_mut):
    import torch
    import paper_1511_02166_amd as P
    _say(f"GA step B={B}, G={G}, k={k}, p_sel={p_sel}, p_mut={p_mut}")
    rng = np.random.default_rng(B + G + k)
    lo = rng.uniform(-1, 0, G)
    hi = lo + rng.uniform(0.1, 2, G)
    genome = lo + (hi - lo) * rng.random((B, G))
    # fitness with ties and unusable individuals
    fit = np.round(rng.standard_normal(B), 1)
    fit[rng.random(B) < 0.05] = -np.inf
    u = synth.ga_uniforms(B * k, P.panel_ga_uniform_count(B, k))[0]
    out = torch.empty(B, G, dtype=torch.float64, device="cuda")
    trace = torch.empty(4 * B, dtype=torch.int32, device="cuda")
    P.panel_ga_step(B, G, k, p_sel, p_mut, 0.15, lo, hi, _dev(fit), _dev(genome), _dev(u), out, trace)
    torch.cuda.synchronize()
    ref, rtr = oracle.ga_step(genome, fit, u, k, p_sel, p_mut, 0.15, lo, hi)
    tr = trace.cpu().numpy().reshape(B, 4)
    assert np.array_equal(tr, rtr)
    assert np.array_equal(out.cpu().numpy(), ref)
    _say(f"  mutated {np.mean(tr[:, 3] >= 0):.2f}, distinct parents {len(set(tr[:, 0]))}")


def test_ga_record_history_and_best():
    import torch
    import paper_1511_02166_amd as P
    _say("GA history")
    B, G = 300, 5
    rng = np.random.default_rng(12)
    counter = torch.zeros(1, dtype=torch.int32, device="cuda")
    hist = torch.zeros(2, dtype=torch.float64, device="cuda")
    hidx = torch.zeros(2, dtype=torch.int32, device="cuda")
    best = torch.full((1,), -np.inf, dtype=torch.float64, device="cuda")
    bg = torch.zeros(G, dtype=torch.float64, device="cuda")
    want_best, want_g = -np.inf, None
    fits = [np.full(B, -np.inf), np.round(rng.standard_normal(B), 1), np.round(rng.standard_normal(B), 1) - 5]
    fits[1][[17, 200]] = 9.0   # a tie: the lower index wins
    for c, f in enumerate(fits):
        g = rng.standard_normal((B, G))
        P.panel_ga_record(B, G, _dev(f), _dev(g), counter, 2, hist, hidx, best, bg)
        torch.cuda.synchronize()
        i = int(np.argmax(f))
        if c < 2:
            assert hist[c].item() == f[i] and hidx[c].item() == i
        if f[i] > want_best:
            want_best, want_g = f[i], g[i].copy()
    assert counter.item() == 3 and hidx[1].item() == 17
    assert best.item() == want_best and np.array_equal(bg.cpu().numpy(), want_g)


def _optimizer(pop=64, N=128, alpha=(0.0, 4 * DEG), seed=5, **kw):
    import paper_1511_02166_amd as P
    prob = synth.ga_problem(6)
    return P.GeneticOptimizer(pop, N, prob.template, prob.gene_map, prob.lo, prob.hi, prob.degree, alpha=alpha,
                              seed=seed, **kw), prob


@pytest.mark.parametrize("formulation,precision", [(0, 0), (1, 0), (0, 1)], ids=["stream-fp64", "hs-fp64", "stream-fp32"])
def test_ga_generation_matches_the_oracle_chain(formulation, precision):
    # contours -> solve -> viscous correction -> fitness on the GPU against
    # the oracle's chain on the same genomes; then the same uniforms breed
    # the same next generation
    import torch
    _say(f"GA generation vs oracle chain, formulation {formulation}, precision {precision}")
    opt, prob = _optimizer(re=1e6, formulation=formulation, precision=precision)
    opt.initialize(_dev(synth.ga_uniforms(6, opt.pop * prob.G)))
    fit = opt.evaluate().cpu().numpy()
    genome = opt.genome.cpu().numpy()
    nodes = oracle.bspline_nodes(prob.template, prob.gene_map, genome, prob.degree, opt.N)
    K = 2
    alpha = np.tile([0.0, 4 * DEG], opt.pop)
    noff = (np.arange(opt.pop + 1) * (opt.N + 1)).astype(np.int32)
    aoff = (np.arange(opt.pop + 1) * K).astype(np.int32)
    xy = nodes.reshape(-1)
    ref = oracle.solve_batch(xy, noff, alpha, aoff, formulation=("stream", "hess_smith")[formulation])
    ld = np.concatenate([oracle.thwaites(nodes[b], alpha[K * b:K * b + K], ref["gamma"][b * K * opt.N:(b + 1) * K * opt.N],
                                         ref["cl"][K * b:K * b + K], 1e6)["ld"] for b in range(opt.pop)])
    rfit = oracle.ga_fitness(aoff, ld, ref["info"])
    ok = np.isfinite(rfit)
    assert np.array_equal(ok, np.isfinite(fit))
    e = np.max(np.abs(fit[ok] - rfit[ok]) / np.abs(rfit[ok]))
    _say(f"  fitness {np.min(rfit[ok]):.1f}..{np.max(rfit[ok]):.1f} (usable {ok.mean():.2f}), rel err {e:.1e}")
    assert e < (1e-9 if precision == 0 else 1e-7)
    assert np.array_equal(np.argsort(fit, kind="stable"), np.argsort(rfit, kind="stable"))
    u = synth.ga_uniforms(7, opt.u_gen.numel())[0]
    opt.record()
    opt.breed(_dev(u))
    torch.cuda.synchronize()
    nxt, tr = oracle.ga_step(genome, rfit, u, opt.k, opt.p_sel, opt.p_mut, opt.sigma, prob.lo, prob.hi)
    assert np.array_equal(opt.trace.cpu().numpy().reshape(-1, 4), tr)
    assert np.array_equal(opt.genome.cpu().numpy(), nxt)


def test_ga_graph_replay_matches_eager():
    # one captured generation replayed; an eager twin fed the replay's
    # uniforms must hold bit-identical genomes, fitness and history
    import torch
    _say("GA graph replay vs eager")
    a, prob = _optimizer(pop=128, N=96, seed=11)
    b, _ = _optimizer(pop=128, N=96, seed=99)
    u0 = _dev(synth.ga_uniforms(8, a.pop * prob.G))
    a.initialize(u0)
    b.initialize(u0)
    a.generation()   # eager generation on a's own generator
    b.generation(a.u_gen.clone())
    torch.cuda.synchronize()
    assert torch.equal(a.genome, b.genome)
    a.capture()      # capture runs one more eager generation first
    b.generation(a.u_gen.clone())
    for r in range(4):
        a._graph.replay()
        torch.cuda.synchronize()
        b.generation(a.u_gen.clone())
        torch.cuda.synchronize()
        assert torch.equal(a.genome, b.genome), r
        assert torch.equal(a.fitness, b.fitness), r
    assert a.counter.item() == b.counter.item() == 6
    assert np.array_equal(a.history(), b.history())
    assert a.best()[0] == b.best()[0]


def test_ga_run_improves_the_population():
    # a short run: the population's mean fitness rises under selection, the
    # history holds each generation's best and the best contour is closed
    import torch
    _say("GA run, 12 generations of 256")
    opt, prob = _optimizer(pop=256, N=128, alpha=(0.0,), seed=3)
    opt.initialize()
    f0 = opt.evaluate().clone()
    opt.run(12)
    torch.cuda.synchronize()
    f1 = opt.evaluate()
    ok0, ok1 = torch.isfinite(f0), torch.isfinite(f1)
    m0, m1 = f0[ok0].mean().item(), f1[ok1].mean().item()
    h = opt.history()
    best, g, xy = opt.best()
    _say(f"  mean L/D {m0:.1f} -> {m1:.1f}; best per generation {np.round(h, 1)}; best {best:.1f}")
    assert h.size == 12 and best == h.max()
    assert m1 > m0
    assert np.array_equal(xy[0], xy[-1]) and np.all(g >= prob.lo) and np.all(g <= prob.hi)
