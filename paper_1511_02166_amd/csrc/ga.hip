// ga.hip -- the genetic algorithm that drives the shape optimisation (Sec. 2)
// on gfx950: B-spline contours from the genomes, random initial genomes,
// fitness from the viscous L/D, and one generation of tournament selection,
// one-point crossover and mutation.  Random numbers are inputs (uniform in
// [0, 1)); their layout per generation is fixed by panel_ga_step.
//
// All of this is O(B (N + G k)) work against the O(B N^3) panel solve of the
// same generation: the kernels are small, latency-bound launches whose only
// job is to keep the whole generation on the device (one graph replay per
// generation, no host round trip).
#include <algorithm>

#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr int NODE_TPB = 128;

// ---- B-spline contour --------------------------------------------------------
// Clamped B-spline of degree d on M control points with uniform interior
// knots t_j = (j - d)/(M - d); node k sits at u_k = (1 - cos(2 pi k/N))/4 for
// k <= N/2 and 1 - u_{N-k} above.  The point is the sum of the d+1 non-zero
// basis functions of the span times their control points, the basis built
// by the triangular Cox-de Boor recurrence.  u = 0 and u = 1 return the end
// control points exactly (node N copies node 0: the template's end points
// coincide).
__device__ __forceinline__ double knot_at(int j, int M, int d) {
    if (j <= d) return 0.0;
    if (j >= M) return 1.0;
    return (double)(j - d) / (double)(M - d);
}

__global__ __launch_bounds__(NODE_TPB) void bspline_nodes_kernel(GaContour c, int32_t N,
                                                                 const double *__restrict__ genome,
                                                                 double *__restrict__ xy) {
    const int b = blockIdx.x;
    const int M = c.M, d = c.degree, G = c.G;
    __shared__ double Q[2 * PANEL_GA_MAX_CTRL];
    for (int i = threadIdx.x; i < 2 * M; i += NODE_TPB) Q[i] = c.tmpl[i];
    __syncthreads();
    for (int g = threadIdx.x; g < G; g += NODE_TPB) Q[c.gene_map[g]] = genome[(size_t)b * G + g];
    __syncthreads();
    const int k = blockIdx.y * NODE_TPB + threadIdx.x;
    if (k > N) return;
    double *P = xy + (size_t)b * 2 * (N + 1) + 2 * k;
    if (k == 0 || k == N) {
        P[0] = Q[0];
        P[1] = Q[1];
        return;
    }
    const double two_pi = 6.283185307179586;
    const int kk = 2 * k <= N ? k : N - k;
    const double h = (1.0 - cos(two_pi * (double)kk / (double)N)) / 4.0;
    const double u = 2 * k <= N ? h : 1.0 - h;
    int s = d;
    while (s + 1 < M && knot_at(s + 1, M, d) <= u) ++s;
    double Nb[PANEL_GA_MAX_DEGREE + 1], left[PANEL_GA_MAX_DEGREE + 1], right[PANEL_GA_MAX_DEGREE + 1];
    Nb[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= PANEL_GA_MAX_DEGREE; ++j) {
        if (j <= d) {
            left[j] = u - knot_at(s + 1 - j, M, d);
            right[j] = knot_at(s + j, M, d) - u;
            double saved = 0.0;
#pragma unroll
            for (int r = 0; r < PANEL_GA_MAX_DEGREE; ++r) {
                if (r < j) {
                    const double tmp = Nb[r] / (right[r + 1] + left[j - r]);
                    Nb[r] = saved + right[r + 1] * tmp;
                    saved = left[j - r] * tmp;
                }
            }
            Nb[j] = saved;
        }
    }
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int r = 0; r <= PANEL_GA_MAX_DEGREE; ++r) {
        if (r <= d) {
            x += Nb[r] * Q[2 * (s - d + r)];
            y += Nb[r] * Q[2 * (s - d + r) + 1];
        }
    }
    P[0] = x;
    P[1] = y;
}

// ---- initial population and fitness -------------------------------------------
__global__ void ga_init_kernel(GaOps o, int32_t B, const double *__restrict__ u, double *__restrict__ genome) {
#pragma clang fp contract(off)
    const size_t n = (size_t)B * o.G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(e % o.G);
        genome[e] = o.lo[g] + (o.hi[g] - o.lo[g]) * u[e];
    }
}

// fitness_b = mean over the airfoil's angles of L/D; -inf when its solve
// failed (info != 0) or an L/D is not finite.
__global__ void ga_fitness_kernel(WsView v, int32_t B, const double *__restrict__ ld,
                                  const int32_t *__restrict__ info, double *__restrict__ fitness) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const AirfoilMeta mt = v.meta[b];
    bool ok = info[b] == 0;
    double s = 0.0;
    for (int k = 0; k < mt.K; ++k) {
        const double x = ld[mt.alpha_off + k];
        ok = ok && isfinite(x);
        s += x;
    }
    fitness[b] = ok ? s / (double)mt.K : -__builtin_inf();
}

// ---- one generation ------------------------------------------------------------
// floor(u n), at most n - 1; inputs outside [0, 1) (NaN included) are held
// to 0 .. n-1 so that every index stays in bounds.
__device__ __forceinline__ int draw(double u, int n) {
    const double x = u * (double)n;
    if (!(x >= 1.0)) return 0;
    if (x >= (double)(n - 1)) return n - 1;
    return (int)x;
}

// Tournament from u[0 .. 2k-2]: k draws with replacement, then rank trials.
// The drawn individual of rank r (fitness descending, equal fitness in draw
// order) is the one with exactly r drawn individuals ahead of it.  cand and
// f are this thread's k-entry slices in LDS.
__device__ int tournament(int B, int k, double p, const double *__restrict__ fitness, const double *u, int *cand,
                          double *f) {
    for (int r = 0; r < k; ++r) {
        cand[r] = draw(u[r], B);
        f[r] = fitness[cand[r]];
    }
    int rank = k - 1;
    for (int r = k - 2; r >= 0; --r)
        if (u[k + r] < p) rank = r;
    int pick = cand[0];
    for (int a = 0; a < k; ++a) {
        int ahead = 0;
        for (int b2 = 0; b2 < k; ++b2) ahead += (f[b2] > f[a] || (b2 < a && f[b2] == f[a])) ? 1 : 0;
        if (ahead == rank) pick = cand[a];
    }
    return pick;
}

constexpr int STEP_TPB = 64;

// A thread per child pair: two tournaments, the crossover position, both
// children written gene by gene, then each child's mutation trial.
__global__ __launch_bounds__(STEP_TPB) void ga_step_kernel(GaOps o, int32_t B, const double *__restrict__ fitness,
                               const double *__restrict__ gin, const double *__restrict__ u,
                               double *__restrict__ gout, int32_t *__restrict__ trace) {
#pragma clang fp contract(off)
    __shared__ int scand[STEP_TPB][PANEL_GA_MAX_TOURNAMENT];
    __shared__ double sfit[STEP_TPB][PANEL_GA_MAX_TOURNAMENT];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= B / 2) return;
    const int G = o.G, k = o.k, per_pair = 4 * k - 1;
    const double *uq = u + (size_t)q * per_pair;
    int *cand = scand[threadIdx.x];
    double *f = sfit[threadIdx.x];
    const int a = tournament(B, k, o.p_sel, fitness, uq, cand, f);
    const int b = tournament(B, k, o.p_sel, fitness, uq + (2 * k - 1), cand, f);
    const int cut = 1 + draw(uq[4 * k - 2], G - 1);
    const double *um = u + (size_t)(B / 2) * per_pair;
    for (int h = 0; h < 2; ++h) {
        const int i = 2 * q + h;
        const int p0 = h == 0 ? a : b, p1 = h == 0 ? b : a;
        double *child = gout + (size_t)i * G;
        for (int g = 0; g < G; ++g) child[g] = gin[(size_t)(g < cut ? p0 : p1) * G + g];
        const double *x = um + 3 * (size_t)i;
        int mj = -1;
        if (x[0] < o.p_mut) {
            mj = draw(x[1], G);
            const double lo = o.lo[mj], hi = o.hi[mj];
            double val = child[mj] + o.sigma * (hi - lo) * (2.0 * x[2] - 1.0);
            val = val < lo ? lo : val;
            val = val > hi ? hi : val;
            child[mj] = val;
        }
        if (trace) {
            trace[4 * i] = p0;
            trace[4 * i + 1] = p1;
            trace[4 * i + 2] = cut;
            trace[4 * i + 3] = mj;
        }
    }
}

// ---- history --------------------------------------------------------------------
// One workgroup: the generation's best (highest fitness, lowest index on
// ties) goes to history slot *counter (if below max_gen); a new overall best
// also copies its genome; then *counter advances.
constexpr int REC_TPB = 256;

__global__ __launch_bounds__(REC_TPB) void ga_record_kernel(int32_t B, int32_t G, const double *__restrict__ fitness,
                                                            const double *__restrict__ genome,
                                                            int32_t *__restrict__ counter, int32_t max_gen,
                                                            double *__restrict__ hist_fit,
                                                            int32_t *__restrict__ hist_idx,
                                                            double *__restrict__ best_fit,
                                                            double *__restrict__ best_genome) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double bf = -__builtin_inf();
    int bi = B;
    for (int b = tid; b < B; b += REC_TPB) {
        const double f = fitness[b];
        if (bi == B || f > bf) {
            bf = f;
            bi = b;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double of = __shfl_xor(bf, off);
        const int oi = __shfl_xor(bi, off);
        if (oi < B && (bi == B || of > bf || (of == bf && oi < bi))) {
            bf = of;
            bi = oi;
        }
    }
    __shared__ double sf[REC_TPB / 64];
    __shared__ int si[REC_TPB / 64];
    __shared__ int take;
    if (lane == 0) {
        sf[wave] = bf;
        si[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < REC_TPB / 64; ++w)
            if (si[w] < B && (bi == B || sf[w] > bf || (sf[w] == bf && si[w] < bi))) {
                bf = sf[w];
                bi = si[w];
            }
        const int c = counter[0];
        if (c < max_gen) {
            hist_fit[c] = bf;
            hist_idx[c] = bi;
        }
        take = bf > best_fit[0] ? bi : -1;
        if (take >= 0) best_fit[0] = bf;
        counter[0] = c + 1;
    }
    __syncthreads();
    if (take >= 0)
        for (int g = tid; g < G; g += REC_TPB) best_genome[g] = genome[(size_t)take * G + g];
}

}  // namespace

hipError_t launch_bspline_nodes(const GaContour &c, int32_t B, int32_t N, const double *genome, double *xy,
                                hipStream_t stream) {
    dim3 grid(B, (N + 1 + NODE_TPB - 1) / NODE_TPB);
    bspline_nodes_kernel<<<grid, NODE_TPB, 0, stream>>>(c, N, genome, xy);
    return hipGetLastError();
}

hipError_t launch_ga_init(const GaOps &o, int32_t B, const double *u, double *genome, hipStream_t stream) {
    const size_t n = (size_t)B * o.G;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    ga_init_kernel<<<grid, 256, 0, stream>>>(o, B, u, genome);
    return hipGetLastError();
}

hipError_t launch_ga_fitness(const WsView &v, int32_t B, const double *ld, const int32_t *info, double *fitness,
                             hipStream_t stream) {
    ga_fitness_kernel<<<(B + 255) / 256, 256, 0, stream>>>(v, B, ld, info, fitness);
    return hipGetLastError();
}

hipError_t launch_ga_step(const GaOps &o, int32_t B, const double *fitness, const double *gin, const double *u,
                          double *gout, int32_t *trace, hipStream_t stream) {
    const int pairs = B / 2;
    ga_step_kernel<<<(pairs + STEP_TPB - 1) / STEP_TPB, STEP_TPB, 0, stream>>>(o, B, fitness, gin, u, gout, trace);
    return hipGetLastError();
}

hipError_t launch_ga_record(int32_t B, int32_t G, const double *fitness, const double *genome, int32_t *counter,
                            int32_t max_gen, double *hist_fit, int32_t *hist_idx, double *best_fit,
                            double *best_genome, hipStream_t stream) {
    ga_record_kernel<<<1, REC_TPB, 0, stream>>>(B, G, fitness, genome, counter, max_gen, hist_fit, hist_idx,
                                                best_fit, best_genome);
    return hipGetLastError();
}

}  // namespace panel
