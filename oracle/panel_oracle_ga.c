/*
 * panel_oracle_ga.c -- plain FP64 CPU oracle of the genetic algorithm that
 * drives the shape optimisation (TEST INFRASTRUCTURE ONLY; nothing in the
 * product links it).
 *
 * Sec. 2 of the paper (the optimisation): the genome is the list of B-spline
 * coefficients of the airfoil contour, ordered from the trailing edge over
 * the upper surface to the trailing edge on the lower surface.  One
 * generation:
 *   1. (first generation only) random genomes within bounds;
 *   2. fitness of every individual from the panel method (lift-to-drag ratio
 *      with the viscous correction);
 *   3. selection by tournament: k individuals drawn at random, the best of
 *      them taken with probability p, the second best with p(1-p), and so on;
 *   4. one-point crossover of two selected parents: genes before a random
 *      position from the first parent, from that position on from the
 *      second; swapping the parents gives the second child; repeated until
 *      the new generation is full;
 *   5. mutation: with some probability an individual gets one of its
 *      coefficients perturbed.
 * The paper leaves the spline degree, knots, bounds, k, p, the mutation rate
 * and size unstated; the readings taken here:
 *   - contour: clamped B-spline of degree d on M control points, uniform
 *     interior knots t_j = (j - d)/(M - d); the first and last control points
 *     coincide (the trailing edge), so the contour is closed;
 *   - genes set chosen coordinates of the control points (a gene map); the
 *     other coordinates are fixed by a template;
 *   - nodes at parameters u_k = (1 - cos(2 pi k / N)) / 4 for k <= N/2 and
 *     u_k = 1 - u_{N-k} above (clustered at the trailing edge, u = 0 and 1,
 *     and at the middle of the parameter range); node N is node 0;
 *   - tournament draws are with replacement: index floor(U B) (at most B-1);
 *     the drawn individuals are ranked by fitness, best first, equal fitness
 *     in draw order; the rank taken is the first r < k-1 with V_r < p, else
 *     k-1 (so the worst gets the remaining probability (1-p)^(k-1));
 *   - crossover position c = 1 + floor(W (G-1)) (at most G-1), so both
 *     parents contribute;
 *   - mutation of each child: if X < p_mut, gene j = floor(Y G) (at most G-1)
 *     moves by sigma (hi_j - lo_j)(2 Z - 1) and is clamped to [lo_j, hi_j];
 *   - no elitism (the paper names none);
 *   - fitness: the mean over the individual's angles of L/D, or -infinity
 *     when the solve failed (info != 0) or an L/D is not finite.
 * Random numbers are inputs (uniform in [0, 1)), laid out per generation as:
 * for each child pair q (B/2 of them), 4k - 1 values [tournament 1: k draws,
 * k - 1 rank trials; tournament 2: the same; crossover: 1]; then for each
 * child i, 3 values [X, Y, Z].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- B-spline contour ---------------------------------------------------- */

static double knot(int j, int M, int d)
{
    if (j <= d)
        return 0.0;
    if (j >= M)
        return 1.0;
    return (double)(j - d) / (double)(M - d);
}

/* Knot span s with t_s <= u < t_{s+1} (s = M-1 at u = 1). */
static int span(double u, int M, int d)
{
    if (u >= 1.0)
        return M - 1;
    int s = d;
    while (s + 1 < M && knot(s + 1, M, d) <= u)
        ++s;
    return s;
}

/* Point of the curve at u by de Boor's algorithm: repeated convex
 * combination of the d+1 control points that act on the span. */
void oracle_bspline_point(int M, int d, const double *Q, double u, double *out)
{
    double px[8], py[8];
    const int s = span(u, M, d);
    for (int i = 0; i <= d; ++i) {
        px[i] = Q[2 * (s - d + i)];
        py[i] = Q[2 * (s - d + i) + 1];
    }
    for (int r = 1; r <= d; ++r) {
        for (int i = d; i >= r; --i) {
            const double lo = knot(s - d + i, M, d), hi = knot(s + 1 + i - r, M, d);
            const double a = (u - lo) / (hi - lo);
            px[i] = (1.0 - a) * px[i - 1] + a * px[i];
            py[i] = (1.0 - a) * py[i - 1] + a * py[i];
        }
    }
    out[0] = px[d];
    out[1] = py[d];
}

double oracle_bspline_param(int k, int N)
{
    const double two_pi = 6.283185307179586;
    if (2 * k <= N)
        return (1.0 - cos(two_pi * (double)k / (double)N)) / 4.0;
    return 1.0 - (1.0 - cos(two_pi * (double)(N - k) / (double)N)) / 4.0;
}

/* Nodes of B contours: control points from the template (2M values) with
 * genome[b*G + g] written to coordinate gene_map[g]; N+1 nodes each. */
void oracle_bspline_nodes(int B, int N, int M, int d, int G, const double *tmpl, const int *gene_map,
                          const double *genome, double *xy)
{
    double *Q = malloc(sizeof(double) * 2 * (size_t)M);
    for (int b = 0; b < B; ++b) {
        memcpy(Q, tmpl, sizeof(double) * 2 * (size_t)M);
        for (int g = 0; g < G; ++g)
            Q[gene_map[g]] = genome[(size_t)b * G + g];
        double *P = xy + (size_t)b * 2 * (N + 1);
        for (int k = 0; k < N; ++k)
            oracle_bspline_point(M, d, Q, oracle_bspline_param(k, N), P + 2 * k);
        P[2 * N] = P[0];
        P[2 * N + 1] = P[1];
    }
    free(Q);
}

/* ---- genetic algorithm ----------------------------------------------------- */

void oracle_ga_init(int B, int G, const double *lo, const double *hi, const double *u, double *genome)
{
    for (int b = 0; b < B; ++b)
        for (int g = 0; g < G; ++g)
            genome[(size_t)b * G + g] = lo[g] + (hi[g] - lo[g]) * u[(size_t)b * G + g];
}

void oracle_ga_fitness(int B, const int *alpha_off, const double *ld, const int *info, double *fitness)
{
    for (int b = 0; b < B; ++b) {
        const int K = alpha_off[b + 1] - alpha_off[b];
        double s = 0.0;
        int ok = info[b] == 0;
        for (int k = 0; k < K; ++k) {
            const double v = ld[alpha_off[b] + k];
            if (!isfinite(v))
                ok = 0;
            s += v;
        }
        fitness[b] = ok ? s / (double)K : -INFINITY;
    }
}

static int draw(double u, int n)
{
    int i = (int)floor(u * (double)n);
    return i < n - 1 ? i : n - 1;
}

/* One tournament from u[0 .. 2k-2]. */
static int tournament(int B, int k, double p, const double *fitness, const double *u)
{
    int cand[64];
    for (int r = 0; r < k; ++r)
        cand[r] = draw(u[r], B);
    /* rank by fitness, best first; equal fitness keeps draw order */
    for (int a = 1; a < k; ++a) {
        const int c = cand[a];
        int q = a;
        while (q > 0 && fitness[cand[q - 1]] < fitness[c]) {
            cand[q] = cand[q - 1];
            --q;
        }
        cand[q] = c;
    }
    int rank = k - 1;
    for (int r = 0; r < k - 1; ++r)
        if (u[k + r] < p) {
            rank = r;
            break;
        }
    return cand[rank];
}

/* One generation of selection, crossover and mutation.  trace (or NULL):
 * 4 int per child: first parent, second parent, crossover position, mutated
 * gene (-1 if none). */
void oracle_ga_step(int B, int G, int k, double p_sel, double p_mut, double sigma, const double *lo,
                    const double *hi, const double *fitness, const double *genome_in, const double *u,
                    double *genome_out, int *trace)
{
    const int per_pair = 4 * k - 1;
    const double *um = u + (size_t)(B / 2) * per_pair;
    for (int q = 0; q < B / 2; ++q) {
        const double *uq = u + (size_t)q * per_pair;
        const int a = tournament(B, k, p_sel, fitness, uq);
        const int b = tournament(B, k, p_sel, fitness, uq + (2 * k - 1));
        const int c = 1 + draw(uq[4 * k - 2], G - 1);
        const int par[2][2] = {{a, b}, {b, a}};
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * q + h;
            double *child = genome_out + (size_t)i * G;
            for (int g = 0; g < G; ++g)
                child[g] = genome_in[(size_t)(g < c ? par[h][0] : par[h][1]) * G + g];
            int mj = -1;
            const double *x = um + 3 * (size_t)i;
            if (x[0] < p_mut) {
                mj = draw(x[1], G);
                double v = child[mj] + sigma * (hi[mj] - lo[mj]) * (2.0 * x[2] - 1.0);
                if (v < lo[mj])
                    v = lo[mj];
                if (v > hi[mj])
                    v = hi[mj];
                child[mj] = v;
            }
            if (trace) {
                trace[4 * i] = par[h][0];
                trace[4 * i + 1] = par[h][1];
                trace[4 * i + 2] = c;
                trace[4 * i + 3] = mj;
            }
        }
    }
}
