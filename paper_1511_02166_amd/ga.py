"""On-device genetic algorithm over B-spline airfoils (Sec. 2 of the paper:
the shape optimisation that the batched panel solver serves).

Each generation runs entirely on the GPU, on the current stream:

    genomes --panel_bspline_nodes--> contours --PanelSolver.step--> surface
    speeds, Cl --panel_thwaites--> L/D --panel_ga_fitness--> fitness
    --panel_ga_record--> history --panel_ga_step (uniforms)--> next genomes

and can be captured once as a HIP graph and replayed per generation.  The
uniform random numbers each generation consumes are drawn with torch's
device generator into a fixed buffer (or supplied by the caller); the
selection, crossover and mutation themselves run in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B
from .solver import PanelSolver


class GeneticOptimizer:
    """Population of ``pop`` B-spline airfoils with ``N`` panels each.

    template [M, 2]: control points (first = last = the trailing edge);
    gene_map [G]: the template coordinates (flattened index) the genes set;
    lo, hi [G]: gene bounds; alpha: the angles every individual is scored
    at (fitness = mean L/D over them); re: chord Reynolds number of the
    viscous correction; k, p_sel: tournament size and the probability of
    taking the best; p_mut, sigma: mutation probability and relative size.
    """

    def __init__(self, pop: int, N: int, template, gene_map, lo, hi, degree: int = 3, alpha=(0.0,),
                 re: float = 1e6, k: int = 4, p_sel: float = 0.75, p_mut: float = 0.2, sigma: float = 0.1,
                 precision: int = B.PANEL_FP64, formulation: int = B.PANEL_STREAM_FUNCTION, seed: int = 0,
                 max_gen: int = 10000, device="cuda"):
        if pop < 2 or pop % 2:
            raise ValueError("the population size must be even and >= 2")
        self.pop, self.N, self.degree = int(pop), int(N), int(degree)
        self.template = np.ascontiguousarray(template, dtype=np.float64).reshape(-1, 2)
        self.gene_map = np.ascontiguousarray(gene_map, dtype=np.int32).reshape(-1)
        self.lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(-1)
        self.hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(-1)
        self.G = int(self.gene_map.size)
        if self.lo.size != self.G or self.hi.size != self.G:
            raise ValueError("lo and hi need one value per gene")
        self.re, self.k, self.p_sel, self.p_mut, self.sigma = float(re), int(k), float(p_sel), float(p_mut), float(sigma)
        self.device = torch.device(device)
        alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
        K = alpha.size
        node_off = (np.arange(pop + 1) * (N + 1)).astype(np.int32)
        alpha_off = (np.arange(pop + 1) * K).astype(np.int32)
        self.solver = PanelSolver(node_off, alpha_off, precision, formulation=formulation)
        dev, f64, i32 = self.device, torch.float64, torch.int32
        self.alpha = torch.as_tensor(np.tile(alpha, pop), device=dev)
        self.genome = torch.zeros(pop, self.G, dtype=f64, device=dev)
        self._next = torch.zeros_like(self.genome)
        self.xy = torch.zeros(2 * pop * (N + 1), dtype=f64, device=dev)
        self.cd = torch.zeros(pop * K, dtype=f64, device=dev)
        self.ld = torch.zeros_like(self.cd)
        self.sep = torch.zeros(2 * pop * K, dtype=i32, device=dev)
        self.fitness = torch.zeros(pop, dtype=f64, device=dev)
        self.trace = torch.zeros(4 * pop, dtype=i32, device=dev)
        self.u_gen = torch.zeros(B.panel_ga_uniform_count(pop, k), dtype=f64, device=dev)
        self.u_init = torch.zeros(pop * self.G, dtype=f64, device=dev)
        self.max_gen = int(max_gen)
        self.counter = torch.zeros(1, dtype=i32, device=dev)
        self.hist_fit = torch.zeros(max(1, self.max_gen), dtype=f64, device=dev)
        self.hist_idx = torch.zeros(max(1, self.max_gen), dtype=i32, device=dev)
        self.best_fit = torch.full((1,), -float("inf"), dtype=f64, device=dev)
        self.best_genome = torch.zeros(self.G, dtype=f64, device=dev)
        self.rng = torch.Generator(device=dev)
        self.rng.manual_seed(int(seed))
        self._graph = None

    # -- the steps of one generation -------------------------------------------------
    def initialize(self, uniforms=None):
        """Random genomes within the bounds (step 1); clears the history."""
        if uniforms is None:
            torch.rand(self.u_init.shape, generator=self.rng, dtype=torch.float64, device=self.device,
                       out=self.u_init)
        else:
            self.u_init.copy_(uniforms.reshape(-1))
        B.panel_ga_init(self.pop, self.G, self.lo, self.hi, self.u_init, self.genome)
        self.counter.zero_()
        self.best_fit.fill_(-float("inf"))

    def contours(self, genome=None, out=None):
        """Contour nodes of the genomes: [pop * (N+1) * 2] (or of ``genome``)."""
        g = self.genome if genome is None else genome
        xy = self.xy if out is None else out
        B.panel_bspline_nodes(g.shape[0], self.N, self.template, self.degree, self.gene_map, g, xy)
        return xy

    def evaluate(self):
        """Fitness of the current genomes (step 2): contours, panel solve,
        viscous correction, mean L/D."""
        s = self.solver
        self.contours()
        s.step(self.xy, self.alpha)
        B.panel_thwaites(s.plan, s.ws, s.gamma, s.cl, self.re, self.cd, self.ld, self.sep)
        B.panel_ga_fitness(s.plan, s.ws, self.ld, s.info, self.fitness)
        return self.fitness

    def record(self):
        B.panel_ga_record(self.pop, self.G, self.fitness, self.genome, self.counter, self.max_gen,
                          self.hist_fit, self.hist_idx, self.best_fit, self.best_genome)

    def breed(self, uniforms=None):
        """Selection, crossover and mutation (steps 3-5) into the next
        generation; the new genomes replace the current ones in place."""
        if uniforms is None:
            torch.rand(self.u_gen.shape, generator=self.rng, dtype=torch.float64, device=self.device,
                       out=self.u_gen)
        else:
            self.u_gen.copy_(uniforms.reshape(-1))
        B.panel_ga_step(self.pop, self.G, self.k, self.p_sel, self.p_mut, self.sigma, self.lo, self.hi,
                        self.fitness, self.genome, self.u_gen, self._next, self.trace)
        self.genome.copy_(self._next)

    def generation(self, uniforms=None):
        self.evaluate()
        self.record()
        self.breed(uniforms)

    # -- graph replay ------------------------------------------------------------------
    def capture(self):
        """Capture one generation (with its random draws) as a HIP graph."""
        self.generation()   # warm-up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        if hasattr(g, "register_generator_state"):
            g.register_generator_state(self.rng)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                self.generation()
        torch.cuda.current_stream().wait_stream(side)
        self._graph = g
        return g

    def run(self, generations: int, graph: bool = True):
        """Run generations (graph replays unless graph=False); the warm-up
        generation of the first capture counts as one of them."""
        done = 0
        if graph and self._graph is None:
            self.capture()
            done = 1   # the warm-up generation ran; the capture only records
        for _ in range(max(0, generations - done)):
            if graph:
                self._graph.replay()
            else:
                self.generation()
        return self

    # -- results -------------------------------------------------------------------------
    def history(self) -> np.ndarray:
        n = min(int(self.counter.item()), self.max_gen)
        return self.hist_fit[:n].cpu().numpy()

    def best(self):
        """(best fitness, its genome [G], its contour [N+1, 2])."""
        xy = torch.zeros(2 * (self.N + 1), dtype=torch.float64, device=self.device)
        self.contours(self.best_genome.reshape(1, -1), out=xy)
        return (float(self.best_fit.item()), self.best_genome.cpu().numpy(),
                xy.cpu().numpy().reshape(self.N + 1, 2))
