// lu.hip -- batched LU factorisation with partial pivoting, triangular
// solves and mixed-precision iterative refinement on gfx950.
//
// Sec. 3 of the paper: each airfoil needs an LU decomposition of its dense
// system ((2/3)n^3 operations), and many small systems are solved at once.
// One workgroup (four wavefronts, or eight when the batch leaves at most one
// airfoil per CU) factors one airfoil's augmented matrix [M | rhs] in place,
// right-looking and blocked by NB columns:
//   1. the n - k0 rows of the NB-column panel are held in registers, one row
//      per thread; each column step finds the pivot with a wavefront
//      shuffle reduction plus an LDS reduction over the wavefronts (largest
//      |a|, lowest row index on ties), exchanges the two rows through LDS,
//      scales and applies the rank-1 update to the thread's own rows;
//   2. the row exchanges are applied to every other column (each thread
//      owns whole columns, so the exchanges of one panel run sequentially
//      per column without synchronisation);
//   3. U12 = L11^{-1} A12 (one thread per column, L11 broadcast from LDS);
//   4. A22 -= L21 U12 on the matrix cores (v_mfma 16x16x4 in FP64 or FP32),
//      U12 staged in LDS, C tiles streamed from global memory.
// The right-hand-side columns ride along as extra columns, so after the
// factorisation they hold L^{-1} P b; the same workgroup then finishes with
// the back substitution (blocked: one wavefront solves each 64-row diagonal
// block with shuffles, all of them update the rows above).
#include <algorithm>
#include <climits>

#include "lu_wave_impl.hpp"
#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr int TPB = 256;   // threads per workgroup by default (4 wavefronts)
constexpr int CH = 256;    // trailing columns per U12 chunk
constexpr int SB = 64;     // rows per diagonal block in the triangular solves
constexpr int SP = 64;     // super-panel width (rank of the big trailing update)
// columns per LDS chunk of the rank-SP update: each chunk re-reads the
// super-panel's L block, so a chunk is as wide as the LDS allows (one
// 512-thread workgroup per CU: 256 columns, 130 KB of FP64 U band; two
// 256-thread workgroups per CU: 128 columns)
template <int TB> struct CtOf { static constexpr int v = TB >= 512 ? 256 : 128; };
constexpr int JR = 16;     // columns per round trip in the refinement residual

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// D = A(16x4) B(4x16) + C.  Lane l supplies A[l%16][l/16] and B[l/16][l%16].
// Element v of lane l holds D[row(l, v)][l%16]; the row map differs between
// the two instructions (measured on gfx950): FP64 interleaves the four row
// groups, FP32 keeps each lane's four rows consecutive.
template <typename T> struct Acc;
template <> struct Acc<double> {
    typedef d4_t type;
    static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Acc<float> {
    typedef f4_t type;
    static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
__device__ inline d4_t mfma16(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4_t mfma16(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ inline T* sys_base(const WsView &v, const AirfoilMeta &mt);
template <> __device__ inline double *sys_base<double>(const WsView &v, const AirfoilMeta &mt) {
    return v.a64 + mt.a_off;
}
template <> __device__ inline float *sys_base<float>(const WsView &v, const AirfoilMeta &mt) {
    return v.a32 + mt.a_off;
}

// Hide a value from loop-invariant code motion, so that address offsets
// derived from it are formed where they are used instead of being hoisted
// to the start of the kernel and kept (or spilled) across every phase.
__device__ __forceinline__ int opaque_s(int v) {
    v = __builtin_amdgcn_readfirstlane(v);   // uniform by contract (free if already scalar)
    asm volatile("" : "+s"(v));
    return v;
}

// Pivot candidate order: larger magnitude wins, lower row index on ties.
__device__ inline bool better(double va, int ia, double vb, int ib) {
    return va > vb || (va == vb && ia < ib);
}

// ---- triangular solves on one vector held in LDS -----------------------------
// The matrix stays in global memory; each 64x64 diagonal block is staged in
// LDS (sblk, column-major, 64 x 64) and solved by one wavefront (lane = row)
// with reciprocals of the diagonal computed up front and the solved entry
// broadcast through a scalar register; the other rows are then updated by
// the whole workgroup.

// s - sum_{j < SB} p[j ld] yb[j] for one row of a full 64-column block:
// loads in groups of 16 issued before their products (left to itself the
// compiler waited after every load).
template <typename T, typename V>
__device__ __forceinline__ V block_dot(const T *p, int ld, const V *yb, V s) {
    V s1 = V(0);
#pragma unroll
    for (int j0 = 0; j0 < SB; j0 += 16) {
        T a[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) a[jj] = p[(size_t)(j0 + jj) * ld];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int jj = 0; jj < 16; jj += 2) {
            s -= V(a[jj]) * yb[j0 + jj];
            s1 -= V(a[jj + 1]) * yb[j0 + jj + 1];
        }
    }
    return s + s1;
}

// Back substitution U x = y (U upper, column-major in global memory), y in LDS.
template <typename T, typename V, int TB = TPB>
__device__ __forceinline__ void trsv_upper(const T *U, int ld, int n, V *y, T *sblk) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + SB - 1) / SB;
    for (int blk = nblk - 1; blk >= 0; --blk) {
        const int rb = blk * SB, w = min(SB, n - rb);
        for (int idx = tid; idx < SB * SB; idx += TB) {
            const int c = idx >> 6, r = idx & 63;
            sblk[idx] = (c < w && r <= c) ? U[(size_t)(rb + c) * ld + rb + r] : T(0);
        }
        __syncthreads();
        if (wave == 0) {
            V yi = (lane < w) ? y[rb + lane] : V(0);
            const V dinv = (lane < w) ? V(1) / V(sblk[lane * SB + lane]) : V(0);
            for (int j = w - 1; j >= 0; --j) {
                if (lane == j) yi *= dinv;
                const V xj = readlane_t(yi, j);
                if (lane < j) yi -= V(sblk[j * SB + lane]) * xj;
            }
            if (lane < w) y[rb + lane] = yi;
        }
        __syncthreads();
        for (int r = tid; r < rb; r += TB) {
            const T *up = U + (size_t)rb * ld + r;
            if (w == SB) {   // every block but the last, partial one
                y[r] = block_dot<T, V>(up, ld, y + rb, y[r]);
            } else {
                V s = y[r];
                for (int j = 0; j < w; ++j) s -= V(up[(size_t)j * ld]) * y[rb + j];
                y[r] = s;
            }
        }
        __syncthreads();
    }
}

// Forward substitution L y = b (unit lower), y in LDS.
template <typename T, typename V, int TB = TPB>
__device__ __forceinline__ void trsv_lower_unit(const T *L, int ld, int n, V *y, T *sblk) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + SB - 1) / SB;
    for (int blk = 0; blk < nblk; ++blk) {
        const int rb = blk * SB, w = min(SB, n - rb);
        for (int idx = tid; idx < SB * SB; idx += TB) {
            const int c = idx >> 6, r = idx & 63;
            sblk[idx] = (c < w && r < w && r > c) ? L[(size_t)(rb + c) * ld + rb + r] : T(0);
        }
        __syncthreads();
        if (wave == 0) {
            V yi = (lane < w) ? y[rb + lane] : V(0);
            for (int j = 0; j < w; ++j) {
                const V xj = readlane_t(yi, j);
                if (lane > j) yi -= V(sblk[j * SB + lane]) * xj;
            }
            if (lane < w) y[rb + lane] = yi;
        }
        __syncthreads();
        for (int r = rb + w + tid; r < n; r += TB) {
            // rows below a block exist only when the block is full (w == SB)
            y[r] = block_dot<T, V>(L + (size_t)rb * ld + r, ld, y + rb, y[r]);
        }
        __syncthreads();
    }
}

// ---- triangular solves on NR vectors at once (the refinement) -----------------
// As above, but every 64x64 diagonal block and every row of the matrix is
// read once for all NR right-hand sides: y[r] (r < NR) are LDS vectors of
// stride ys.  The serial chain of a diagonal block (64 broadcast steps) is
// shared by the NR vectors.
template <int NR>
__device__ __forceinline__ void block_dot_n(const float *p, int ld, const float *yb, int ys, float (&s)[NR]) {
    // one running address (a column step per load): precomputed addresses
    // for all 64 columns would hold 128 registers
    const size_t step = (size_t)opaque_s(ld);
#pragma unroll 1
    for (int j0 = 0; j0 < SB; j0 += 16) {
        float a[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            a[jj] = *p;
            p += step;
            asm volatile("" : "+v"(p));   // keep the walk sequential (no table of offsets)
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
#pragma unroll
            for (int r = 0; r < NR; ++r) s[r] -= a[jj] * yb[r * ys + j0 + jj];
            if ((jj & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int NR, int TB>
__device__ __forceinline__ void trsm_lower_unit(const float *L, int ld, int n, int nr, float *y, int ys, float *sblk) {
    ld = opaque_s(ld);   // address arithmetic formed here, not hoisted to the kernel entry
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + SB - 1) / SB;
    for (int blk = 0; blk < nblk; ++blk) {
        const int rb = blk * SB, w = min(SB, n - rb);
        for (int idx = tid; idx < SB * SB; idx += TB) {
            const int c = idx >> 6, r = idx & 63;
            sblk[idx] = (c < w && r < w && r > c) ? L[(size_t)(rb + c) * ld + rb + r] : 0.0f;
        }
        __syncthreads();
        if (wave == 0) {
            float yi[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) yi[r] = (r < nr && lane < w) ? y[r * ys + rb + lane] : 0.0f;
#pragma unroll 2
            for (int j = 0; j < w; ++j) {
                const float lj = sblk[j * SB + lane];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const float xj = readlane_t(yi[r], j);
                    if (lane > j) yi[r] -= lj * xj;
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr && lane < w) y[r * ys + rb + lane] = yi[r];
        }
        __syncthreads();
        for (int row = rb + w + tid; row < n; row += TB) {
            float acc[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = y[r * ys + row];
            block_dot_n<NR>(L + (size_t)rb * ld + row, ld, y + rb, ys, acc);
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr) y[r * ys + row] = acc[r];
        }
        __syncthreads();
    }
}

template <int NR, int TB>
__device__ __forceinline__ void trsm_upper(const float *U, int ld, int n, int nr, float *y, int ys, float *sblk) {
    ld = opaque_s(ld);   // address arithmetic formed here, not hoisted to the kernel entry
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + SB - 1) / SB;
    for (int blk = nblk - 1; blk >= 0; --blk) {
        const int rb = blk * SB, w = min(SB, n - rb);
        for (int idx = tid; idx < SB * SB; idx += TB) {
            const int c = idx >> 6, r = idx & 63;
            sblk[idx] = (c < w && r <= c) ? U[(size_t)(rb + c) * ld + rb + r] : 0.0f;
        }
        __syncthreads();
        if (wave == 0) {
            float yi[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) yi[r] = (r < nr && lane < w) ? y[r * ys + rb + lane] : 0.0f;
            const float dinv = (lane < w) ? 1.0f / sblk[lane * SB + lane] : 0.0f;
#pragma unroll 2
            for (int j = w - 1; j >= 0; --j) {
                const float uj = sblk[j * SB + lane];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (lane == j) yi[r] *= dinv;
                    const float xj = readlane_t(yi[r], j);
                    if (lane < j) yi[r] -= uj * xj;
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr && lane < w) y[r * ys + rb + lane] = yi[r];
        }
        __syncthreads();
        for (int row = tid; row < rb; row += TB) {
            const float *up = U + (size_t)rb * ld + row;
            float acc[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = y[r * ys + row];
            if (w == SB) {   // every block but the last, partial one
                block_dot_n<NR>(up, ld, y + rb, ys, acc);
            } else {
                for (int j = 0; j < w; ++j) {
                    const float a = up[(size_t)j * ld];
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r] -= a * y[r * ys + rb + j];
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr) y[r * ys + row] = acc[r];
        }
        __syncthreads();
    }
}

// LDS scratch of one workgroup's panel factorisation.
template <typename T, int NB, int R, int TB> struct PanelLds {
    // each wavefront's pivot candidate: all R rows of the thread that holds
    // it (double-buffered); cq names the one that is the candidate
    T crow[2][TB / 64][R][NB];
    int cq[2][TB / 64];
    T grow[2][NB];             // row g (the one the pivot replaces)
    double cval[2][TB / 64];  // candidate |a|
    int cidx[2][TB / 64];     // candidate row index
    int piv[NB];               // pivot row chosen at each column of the panel
};

// One column step of the panel factorisation.  Rows are held one per thread
// (row k0 + tid + TB q in p[q][.]); C is a compile-time column index so the
// register array is only indexed with constants.  One barrier per column:
// every wavefront publishes its best candidate together with the whole
// candidate row, and the owner of row g publishes row g, so after the
// barrier each thread can perform the exchange and the rank-1 update on its
// own rows.  The LDS slots are double-buffered by column parity.
template <typename T, int NB, int R, int C, int TB, typename Lds>
__device__ __forceinline__ void panel_step(T (&p)[R][NB], int k0, int n, int &info, Lds &L) {
    constexpr int buf = C & 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = k0 + C;
    // this thread's candidate: largest |a| among its rows >= g (rows grow
    // with q, so a strict comparison keeps the lowest index on ties)
    double best = -1.0;
    int bidx = INT_MAX, bq = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + tid + TB * q;
        const double a = fabs((double)p[q][C]);
        if (r >= g && r < n && a > best) {
            best = a;
            bidx = r;
            bq = q;
        }
    }
    // this wavefront's candidate: exact maximum, lowest row index on ties
    const double wbest = wave_max(best);
    const unsigned long long tie = __ballot(best == wbest);
    int wlane = __ffsll((long long)tie) - 1;
    int widx = __builtin_amdgcn_readlane(bidx, wlane);
    if (__popcll(tie) > 1) {   // rare: several lanes hold the maximum
        int cand = (best == wbest) ? bidx : INT_MAX;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cand = min(cand, __shfl_xor(cand, off));
        widx = cand;
        wlane = __ffsll((long long)__ballot(bidx == widx && best == wbest)) - 1;
    }
    if (!(wbest >= 0.0)) widx = INT_MAX;   // no row of this wavefront is eligible
    if (lane == wlane) {
        // all of the thread's rows go out: picking row bq here would index
        // the register array with a run-time value, which puts the whole
        // panel in scratch memory
        L.cval[buf][wave] = wbest;
        L.cidx[buf][wave] = widx;
        L.cq[buf][wave] = bq;
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) L.crow[buf][wave][q][cc] = p[q][cc];
    }
    if (tid == C) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) L.grow[buf][cc] = p[0][cc];
    }
    __syncthreads();
    double pv = L.cval[buf][0];
    int pr = L.cidx[buf][0], pw = 0;
#pragma unroll
    for (int w = 1; w < TB / 64; ++w) {
        const double v = L.cval[buf][w];
        const int i = L.cidx[buf][w];
        if (better(v, i, pv, pr)) {
            pv = v;
            pr = i;
            pw = w;
        }
    }
    // pv == 0: the column is zero at and below the diagonal (exact zero
    // pivot, LAPACK skips the step); no candidate at all (NaN column) alike.
    const bool zero = !(pv > 0.0) || pr == INT_MAX;
    if (tid == 0) L.piv[C] = zero ? g : pr;
    if (zero) {
        if (info == 0) info = g + 1;
        return;
    }
    const T *u = L.crow[buf][pw][L.cq[buf][pw]];
    if (pr != g) {
        const int pown = (pr - k0) & (TB - 1), pq = (pr - k0) / TB;
        if (tid == pown) {
            // (a select per slot, for the same reason as above)
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) {
                const T t = L.grow[buf][cc];
#pragma unroll
                for (int q = 0; q < R; ++q) p[q][cc] = (q == pq) ? t : p[q][cc];
            }
        }
        if (tid == C) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) p[0][cc] = u[cc];
        }
    }
    const T piv = u[C];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + tid + TB * q;
        if (r > g && r < n) {
            const T l = p[q][C] / piv;
            p[q][C] = l;
#pragma unroll
            for (int cc = C + 1; cc < NB; ++cc) p[q][cc] -= l * u[cc];
        }
    }
}

template <typename T, int NB, int R, int C, int TB, typename Lds>
__device__ __forceinline__ void panel_steps(T (&p)[R][NB], int k0, int nb, int n, int &info, Lds &L) {
    if constexpr (C < NB) {
        if (C < nb) {
            panel_step<T, NB, R, C, TB>(p, k0, n, info, L);
            panel_steps<T, NB, R, C + 1, TB>(p, k0, nb, n, info, L);
        }
    }
}

// Steps 1-3 of one pivot panel (columns k0..k0+nb-1, rows k0..n-1, R =
// rows / TB rounded up): rows into registers, factorisation, rows back to
// memory, L11 to LDS, pivots out.  R is chosen per panel, so the later
// panels of a system (fewer rows) run the smaller instances.
template <typename T, int NB, int R, int TB, typename Lds>
__device__ __forceinline__ void wg_panel(T *A, int ld, int n, int k0, int nb, int32_t *piv, int &info, Lds &L,
                                         T (*s_L11)[NB + 1]) {
    ld = opaque_s(ld);
    const int tid = threadIdx.x;
    T p[R][NB];
    // every load is issued (clamped addresses) before any is masked: with
    // the mask next to the load the compiler put each load in a branch of
    // its own and waited for it there, one memory latency per element
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int rr = min(k0 + tid + TB * q, n - 1);
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) p[q][cc] = A[(size_t)min(k0 + cc, n - 1) * ld + rr];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + tid + TB * q;
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) p[q][cc] = (r < n && cc < nb) ? p[q][cc] : T(0);
    }
    panel_steps<T, NB, R, 0, TB>(p, k0, nb, n, info, L);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + tid + TB * q;
        if (r < n) {
            if (nb == NB) {
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) A[(size_t)(k0 + cc) * ld + r] = p[q][cc];
            } else {
#pragma unroll
                for (int cc = 0; cc < NB; ++cc)
                    if (cc < nb) A[(size_t)(k0 + cc) * ld + r] = p[q][cc];
            }
        }
    }
    if (tid < NB) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) s_L11[tid][cc] = (tid < nb) ? p[0][cc] : T(0);
        if (tid < nb) piv[k0 + tid] = L.piv[tid];
    }
}

template <typename T, int NB, int R, int TB, typename Lds>
__device__ __forceinline__ bool wg_panel_if(int rows, T *A, int ld, int n, int k0, int nb, int32_t *piv, int &info,
                                            Lds &L, T (*s_L11)[NB + 1]) {
    if (rows != R) return false;
    wg_panel<T, NB, R, TB>(A, ld, n, k0, nb, piv, info, L, s_L11);
    return true;
}

// U12 = L11^{-1} A12 for columns [cs, cs + cw) (cw <= CH), rows k0..k0+nb:
// one thread per column, the column kept in registers, L11 (unit lower) read
// from LDS; the result goes back to memory and, k-major, to Us (ld CH + 4)
// as the B operand of the following update.
template <typename T, int NB>
__device__ __forceinline__ void trsm_cols(T *A, int ld, int k0, int nb, int cs, int cw,
                                          const T (*sL)[NB + 1], T *Us) {
    ld = opaque_s(ld);
    const int tid = threadIdx.x;
    T u[NB];
    // rows k0..k0+NB-1 always lie inside the column (ld is a multiple of NB);
    // rows past n are zero padding
    T *cp = A + (size_t)(cs + tid) * ld + k0;
    if (tid < cw) {
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const T t = cp[r];
            u[r] = (r < nb) ? t : T(0);
        }
#pragma unroll
        for (int c = 0; c < NB - 1; ++c) {
            const T uc = u[c];
#pragma unroll
            for (int r = c + 1; r < NB; ++r) u[r] -= sL[r][c] * uc;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) cp[r] = u[r];
    } else {
#pragma unroll
        for (int r = 0; r < NB; ++r) u[r] = T(0);
    }
    if (tid < CH) {
#pragma unroll
        for (int r = 0; r < NB; ++r) Us[r * (CH + 4) + tid] = u[r];
    }
}

// C[rows rowA..rowEnd, cols colA..colA+ncol) -= A[rows, kb..kb+KD) * B, on the
// matrix cores.  rowA is a multiple of 16 and rowEnd <= ld (tiles may run
// into the zero padding rows).  B lives in LDS: B(k, c) = Bs[k * ldb + c]
// when BK is true (k-major) and Bs[c * ldb + k] otherwise, c counted from
// bcol0.  Each wavefront takes row tiles; it keeps the tile's A fragments in
// registers and streams four 16x16 C tiles at a time.
template <typename T, int KD, bool BK, int TB = TPB>
__device__ __forceinline__ void gemm_sub(T *A, int ld, int rowA, int rowEnd, int colA, int ncol, int kb,
                                         const T *Bs, int ldb, int bcol0) {
    ld = opaque_s(ld);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int nrt = (rowEnd - rowA + 15) >> 4;
    const int nct = (ncol + 15) >> 4;
    if (nrt <= 0 || ncol <= 0) return;
    for (int rt = wave; rt < nrt; rt += TB / 64) {
        const int r0 = rowA + 16 * rt;
        T af[KD / 4];
        const T *lcol = A + (size_t)kb * ld + r0 + i16;
#pragma unroll
        for (int kk = 0; kk < KD / 4; ++kk) af[kk] = -lcol[(size_t)(4 * kk + k4) * ld];
        for (int ct0 = 0; ct0 < nct; ct0 += 4) {
            typename Acc<T>::type acc[4];
            T *ccol[4];
            bool cok[4];
            int cl[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                cl[t] = 16 * (ct0 + t) + i16;
                cok[t] = cl[t] < ncol;
                ccol[t] = A + (size_t)(colA + (cok[t] ? cl[t] : ncol - 1)) * ld + r0;
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[t][e] = ccol[t][Acc<T>::row(lane, e)];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int bc = bcol0 + (cok[t] ? cl[t] : 0);
#pragma unroll
                for (int kk = 0; kk < KD / 4; ++kk) {
                    const int k = 4 * kk + k4;
                    const T bv = BK ? Bs[k * ldb + bc] : Bs[bc * ldb + k];
                    acc[t] = mfma16(af[kk], bv, acc[t]);
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (cok[t]) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) ccol[t][Acc<T>::row(lane, e)] = acc[t][e];
                }
        }
    }
}

// TB threads (TB / 64 wavefronts) per airfoil; RMAX: largest number of rows
// per thread in a panel (n1 <= TB * RMAX).  With 256 threads and up to three
// rows per thread two workgroups share a CU; the other instances take the
// whole register file of one.
// LDS of one workgroup's factorisation.
template <typename T, int NB, int RMAX, int TB> struct WgLuLds {
    static constexpr int UB = NB * (CH + 4) > CtOf<TB>::v * (SP + 1) ? NB * (CH + 4) : CtOf<TB>::v * (SP + 1);
    PanelLds<T, NB, RMAX, TB> L;
    T s_L11[NB][NB + 1];
    T s_U[UB];   // NB x (CH + 4) U rows, or the CT x (SP + 1) band of step 6
    T y[PANEL_NMAX + 1];
};

template <typename T, int NB, int RMAX, int TB>
__device__ __forceinline__ void wg_lu(const WsView &v, int b, int32_t *__restrict__ info_out,
                                      WgLuLds<T, NB, RMAX, TB> &S) {
    const AirfoilMeta mt = v.meta[b];
    const int n = mt.n1, ld = mt.ld, ncols = mt.n1 + mt.K;
    const int tid = threadIdx.x;
    double *X = v.x + mt.x_off;

    if (v.flag[b] != 0) {   // screened out by the assembly
        if (tid == 0) info_out[b] = -1;
        for (int i = tid; i < n * mt.K; i += TB) X[i] = __builtin_nan("");
        return;
    }

    T *A = sys_base<T>(v, mt);
    int32_t *piv = v.piv + mt.piv_off;

    PanelLds<T, NB, RMAX, TB> &L = S.L;
    T (*s_L11)[NB + 1] = S.s_L11;
    T (*s_U)[CH + 4] = reinterpret_cast<T (*)[CH + 4]>(S.s_U);
    constexpr int CT = CtOf<TB>::v;
    int info = 0;

    // Super-panels of SP columns; inside, NB-column pivot panels update the
    // super-panel's own columns fully but only the super-panel's rows of the
    // columns to its right; those columns get one rank-SP update at the end.
    for (int K0 = 0; K0 < n; K0 += SP) {
    const int kend = min(K0 + SP, n);
    for (int k0 = K0; k0 < kend; k0 += NB) {
        const int nb = min(NB, n - k0);

        // ---- 1.-3. the panel: load, factorise, store ------------------------
        const int rows = (n - k0 + TB - 1) / TB;
        wg_panel_if<T, NB, 1, TB>(rows, A, ld, n, k0, nb, piv, info, L, s_L11) ||
            wg_panel_if<T, NB, (RMAX >= 2 ? 2 : 1), TB>(rows, A, ld, n, k0, nb, piv, info, L, s_L11) ||
            wg_panel_if<T, NB, (RMAX >= 3 ? 3 : 1), TB>(rows, A, ld, n, k0, nb, piv, info, L, s_L11) ||
            wg_panel_if<T, NB, (RMAX >= 4 ? 4 : 1), TB>(rows, A, ld, n, k0, nb, piv, info, L, s_L11) ||
            wg_panel_if<T, NB, (RMAX >= 5 ? 5 : 1), TB>(rows, A, ld, n, k0, nb, piv, info, L, s_L11);
        __syncthreads();

        // ---- 4. the panel's row exchanges on every other column ------------
        // (each thread owns whole columns; exchanges are rare for this system,
        // so the sequential per-column loop costs little)
        for (int j = tid; j < ncols - nb; j += TB) {
            const int col = j < k0 ? j : j + nb;
            T *cp = A + (size_t)col * ld;
            for (int c = 0; c < nb; ++c) {
                const int pr = L.piv[c], g = k0 + c;
                if (pr != g) {
                    const T t0 = cp[g];
                    cp[g] = cp[pr];
                    cp[pr] = t0;
                }
            }
        }
        __syncthreads();

        // ---- 5. the panel's update of the super-panel columns to its right
        const int rows0 = k0 + nb;
        if (rows0 < kend) {
            trsm_cols<T, NB>(A, ld, k0, nb, rows0, kend - rows0, s_L11, &s_U[0][0]);
            __syncthreads();
            if (rows0 < n) gemm_sub<T, NB, true, TB>(A, ld, rows0, n, rows0, kend - rows0, k0, &s_U[0][0], CH + 4, 0);
            __syncthreads();
        }
    }
    // ---- 6. columns right of the super-panel.  They saw only row exchanges so
    // far (all their rows are equally stale, so the exchanges keep them
    // consistent); now apply the super-panel's four 16-column steps to its
    // own rows (triangular solve + rank-16 update of the rows below within
    // the band), then one rank-SP update of everything below the band.
    if (kend < ncols) {
        for (int k0 = K0; k0 < kend; k0 += NB) {
            const int nb = min(NB, kend - k0);
            if (tid < NB) {
                const T *lrow = A + (size_t)k0 * ld + k0 + tid;
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) s_L11[tid][cc] = (tid < nb && cc < nb) ? lrow[(size_t)cc * ld] : T(0);
            }
            __syncthreads();
            for (int cs = kend; cs < ncols; cs += CH) {
                const int cw = min(CH, ncols - cs);
                trsm_cols<T, NB>(A, ld, k0, nb, cs, cw, s_L11, &s_U[0][0]);
                __syncthreads();
                if (k0 + nb < kend)
                    gemm_sub<T, NB, true, TB>(A, ld, k0 + nb, kend, cs, cw, k0, &s_U[0][0], CH + 4, 0);
                __syncthreads();
            }
        }
        if (kend < n) {
            T *Bs = &s_U[0][0];   // CT x SP band of U, column-major (ld SP+1)
            for (int cs = kend; cs < ncols; cs += CT) {
                const int cw = min(CT, ncols - cs);
                for (int idx = tid; idx < SP * CT; idx += TB) {
                    const int c = idx / SP, r = idx - c * SP;
                    Bs[c * (SP + 1) + r] = (c < cw) ? A[(size_t)(cs + c) * ld + K0 + r] : T(0);
                }
                __syncthreads();
                gemm_sub<T, SP, false, TB>(A, ld, kend, n, cs, cw, K0, Bs, SP + 1, 0);
                __syncthreads();
            }
        }
    }
    }

    // ---- back substitution for the K right-hand sides ----------------------
    // The right-hand-side columns now hold L^{-1} P b; solve U x = that.
    if (tid == 0) {
        info_out[b] = info;
        v.flag[b] = info;
    }
    if (info != 0) {
        for (int i = tid; i < n * mt.K; i += TB) X[i] = __builtin_nan("");
        return;
    }
    T *y = S.y;
    T *sblk = &s_U[0][0];   // SB x SB values (NB * CH >= SB * SB)
    for (int k = 0; k < mt.K; ++k) {
        __syncthreads();
        for (int i = tid; i < n; i += TB) y[i] = A[(size_t)(n + k) * ld + i];
        __syncthreads();
        trsv_upper<T, T, TB>(A, ld, n, y, sblk);
        for (int i = tid; i < n; i += TB) X[(size_t)k * n + i] = (double)y[i];
    }
}

template <typename T, int NB, int RMAX, int TB>
__global__ __launch_bounds__(TB, (TB <= 256 && RMAX <= 3) ? 2 : 1) void lu_kernel(WsView v, int32_t *__restrict__ info_out) {
    __shared__ WgLuLds<T, NB, RMAX, TB> S;
    wg_lu<T, NB, RMAX, TB>(v, v.order[blockIdx.x], info_out, S);
}

// Mixed precision: iterative refinement of X with the FP64 system in A64 and
// the FP32 factors in A32.  One sweep: r = b - A x in FP64 (one pass over A
// serving KG right-hand sides); for each right-hand side not yet converged:
// stop if r is at the FP64 backward-error floor, ||r||_inf <= sqrt(n) eps
// ||A||_inf ||x||_inf (no further sweep can improve x); otherwise
// d = U^{-1} L^{-1} P r in FP32 (one pass over the factors for the group),
// x += d, and stop by the rule of refined_enough.  KG = 4: eight would spill
// registers in the residual pass of a 512-thread workgroup.
constexpr int KG = 4;
constexpr int YS = PANEL_NMAX + 1;
template <int TB> struct WgRefLds {
    double sx[KG][YS];   // current solutions
    float sd[KG][YS];    // residuals in pivot order, then the corrections
    int perm[YS];        // position i of the factored system holds row perm[i]
    int pinv[YS];        // and row r sits at position pinv[r]
    double red[3][KG][TB / 64];
    float sblk[SB * SB];
};

// FP64 refinement of the FP32 solutions of one airfoil, KG right-hand sides
// per pass: one read of A64 forms their residuals, one read of the FP32
// factors their corrections.
template <int TB>
__device__ __forceinline__ void wg_refine(const WsView &v, int b, int32_t *__restrict__ info, double tol,
                                          int max_iter, WgRefLds<TB> &S) {
    const AirfoilMeta mt = v.meta[b];
    const int n = mt.n1, ld = mt.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (info[b] != 0) {
        if (tid == 0) {
            v.iters[b] = 0;
            v.flag[b] = info[b];
        }
        return;
    }
    const double *A = v.a64 + mt.a_off;
    const float *LU = v.a32 + mt.a_off;
    const int32_t *piv = v.piv + mt.piv_off;
    double *X = v.x + mt.x_off;
    if (tid == 0) {
        for (int i = 0; i < n; ++i) S.perm[i] = i;
        for (int i = 0; i < n; ++i) {
            const int p = piv[i];
            const int t0 = S.perm[i];
            S.perm[i] = S.perm[p];
            S.perm[p] = t0;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += TB) S.pinv[S.perm[i]] = i;
    // block-wide maxima of three values per right-hand side
    auto bmax = [&](double (&a)[3][KG]) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < KG; ++r) {
                double x = a[q][r];
                for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
                if (lane == 0) S.red[q][r][wave] = x;
            }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < KG; ++r) {
                double x = S.red[q][r][0];
                for (int w = 1; w < TB / 64; ++w) x = fmax(x, S.red[q][r][w]);
                a[q][r] = x;
            }
        __syncthreads();
    };
    const double floor_c = sqrt((double)n) * 2.220446049250313e-16;
    double anrm = -1.0;   // ||A||_inf, found during the first residual
    int worst = 0;
    bool failed = max_iter == 0;
    for (int k0 = 0; k0 < mt.K; k0 += KG) {
        const int kn = min(KG, mt.K - k0);
        for (int kk = 0; kk < kn; ++kk)
            for (int i = tid; i < n; i += TB) S.sx[kk][i] = X[(size_t)(k0 + kk) * n + i];
        __syncthreads();
        bool conv[KG];
        int sweeps[KG];
        double dprev[KG];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            conv[kk] = kk >= kn;
            sweeps[kk] = 0;
            dprev[kk] = -1.0;
        }
        for (int it = 0; it < max_iter; ++it) {
            bool all = true;
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) all = all && conv[kk];
            if (all) break;
            // r = b - A x for the group, one pass over A; the residual goes
            // straight to its pivot position (FP32) and its size is kept
            double m[3][KG];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) m[0][kk] = m[1][kk] = m[2][kk] = 0.0;
            double rowmax = 0.0;
            const bool first_pass = anrm < 0.0;
            const int ldr = opaque_s(ld);
            for (int i = tid; i < n; i += TB) {
                double sk[KG];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) sk[kk] = (kk < kn) ? A[(size_t)(n + k0 + kk) * ldr + i] : 0.0;
                double ra = 0.0;
                // JR columns per round trip: all their loads are issued
                // before the first product (left to itself the compiler put
                // a wait after every load, one memory latency per element)
                for (int j0 = 0; j0 < n; j0 += JR) {
                    double a[JR];
#pragma unroll
                    for (int jj = 0; jj < JR; ++jj) a[jj] = A[(size_t)min(j0 + jj, n - 1) * ldr + i];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int jj = 0; jj < JR; ++jj) {
                        if (j0 + jj < n) {
#pragma unroll
                            for (int kk = 0; kk < KG; ++kk)
                                if (kk < kn) sk[kk] -= a[jj] * S.sx[kk][j0 + jj];
                            if (first_pass) ra += fabs(a[jj]);
                        }
                        // keep the broadcast reads of x from being hoisted all at once
                        if ((jj & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                    }
                }
                const int pi = S.pinv[i];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) {
                    if (kk < kn) {
                        S.sd[kk][pi] = (float)sk[kk];
                        m[0][kk] = fmax(m[0][kk], fabs(sk[kk]));
                        m[1][kk] = fmax(m[1][kk], fabs(S.sx[kk][i]));
                    }
                }
                rowmax = fmax(rowmax, ra);
            }
            m[2][0] = rowmax;
            bmax(m);
            if (anrm < 0.0) anrm = m[2][0];
            // a right-hand side whose residual is at the FP64 backward-error
            // floor is done; the others take a correction
            bool need = false;
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
                if (!conv[kk] && m[0][kk] <= floor_c * anrm * m[1][kk]) conv[kk] = true;
                if (!conv[kk]) need = true;
            }
            if (!need) break;
            trsm_lower_unit<KG, TB>(LU, ld, n, kn, &S.sd[0][0], YS, S.sblk);
            trsm_upper<KG, TB>(LU, ld, n, kn, &S.sd[0][0], YS, S.sblk);
            double d[3][KG];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) d[0][kk] = d[1][kk] = d[2][kk] = 0.0;
            for (int i = tid; i < n; i += TB) {
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) {
                    if (kk < kn && !conv[kk]) {
                        const double dd = (double)S.sd[kk][i];
                        const double x1 = S.sx[kk][i] + dd;
                        S.sx[kk][i] = x1;
                        d[0][kk] = fmax(d[0][kk], fabs(dd));
                        d[1][kk] = fmax(d[1][kk], fabs(x1));
                    }
                }
            }
            bmax(d);
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
                if (kk < kn && !conv[kk]) {
                    ++sweeps[kk];
                    conv[kk] = wv::refined_enough(d[0][kk], dprev[kk], d[1][kk], tol);
                    dprev[kk] = d[0][kk];
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            if (!conv[kk]) failed = true;
            worst = max(worst, sweeps[kk]);
        }
        for (int kk = 0; kk < kn; ++kk)
            for (int i = tid; i < n; i += TB) X[(size_t)(k0 + kk) * n + i] = S.sx[kk][i];
        __syncthreads();
    }
    if (tid == 0) {
        v.iters[b] = worst;
        if (failed) info[b] = -2;
        v.flag[b] = info[b];
    }
}

template <int TB>
__global__ __launch_bounds__(TB) void refine_kernel(WsView v, int32_t *__restrict__ info, double tol,
                                                     int max_iter) {
    __shared__ WgRefLds<TB> S;
    wg_refine<TB>(v, v.order[blockIdx.x], info, tol, max_iter, S);
}

// One launch for a whole batch: persistent workgroups of four wavefronts pop
// airfoils from the plan's LPT order.  The first n_block entries (the largest
// systems) are taken by whole workgroups; once those are gone every
// wavefront pops the smaller systems on its own.  With FP32 factors each
// airfoil's FP64 refinement follows its factorisation in the same workgroup
// or wavefront, so the mixed-precision factor/solve is one launch too.
template <typename T> struct BatchWaveLds {
    union {
        wv::WaveLuLds<T> lu;
        wv::WaveRefLds ref;
    } u;
};
template <typename T> union BatchLds {
    WgLuLds<T, 16, 3, TPB> lu;
    WgRefLds<TPB> ref;
    BatchWaveLds<T> wave[TPB / 64];
};

// One item of each kind.  (Kept out of line, with separate register
// allocations, they spilled more: 600-1000 bytes of scratch per function on
// gfx950 against 216-424 for the whole kernel inlined.)
template <typename T>
__device__ __forceinline__ void batch_wg_item(const WsView &v, int b, int32_t *info, int mixed, double tol,
                                           int max_iter, BatchLds<T> &S) {
    wg_lu<T, 16, 3, TPB>(v, b, info, S.lu);
    __syncthreads();
    if (mixed) {
        wg_refine<TPB>(v, b, info, tol, max_iter, S.ref);
        __syncthreads();
    }
}

template <typename T>
__device__ __forceinline__ void batch_wave_item(const WsView &v, int b, int32_t *info, int mixed, double tol,
                                             int max_iter, BatchWaveLds<T> &W) {
    wv::wave_lu<T>(v, b, info, W.u.lu);
    wv::wave_sync();
    if (mixed) {
        wv::wave_refine(v, b, info, tol, max_iter, W.u.ref);
        wv::wave_sync();
    }
}

template <typename T>
__global__ __launch_bounds__(TPB, 2) void batch_kernel(WsView v, int32_t n_block, int32_t B, int32_t mixed,
                                                       double tol, int32_t max_iter, int32_t *__restrict__ info) {
    __shared__ BatchLds<T> S;
    __shared__ int s_item;
    int32_t *q = v.queue;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&q[0], 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: keep it scalar
        __syncthreads();
        if (it >= n_block) break;
        batch_wg_item<T>(v, v.order[it], info, mixed, tol, max_iter, S);
    }
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // this wavefront's LDS area
    for (;;) {
        int it = 0;
        if ((threadIdx.x & 63) == 0) it = atomicAdd(&q[1], 1);
        it = __builtin_amdgcn_readfirstlane(it);   // lane 0's ticket, in a scalar register
        if (it >= B - n_block) break;
        batch_wave_item<T>(v, v.order[n_block + it], info, mixed, tol, max_iter, S.wave[w]);
    }
    // every workgroup counts itself out; the last one leaves the counters at
    // zero for the next launch on this workspace
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q[2], 1) == (int)gridDim.x - 1) {
            q[0] = 0;
            q[1] = 0;
            q[2] = 0;
            __threadfence();
        }
    }
}

// Compute units of the current device (read once per process and device).
int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

// Eight wavefronts per airfoil for the workgroup kernels: by default when
// the batch has at most one airfoil per CU (measured: 256 sections at
// N = 1024, 24.4 -> 19.9 ms in FP64; with more airfoils than CUs, four per
// airfoil and two airfoils per CU keep more systems in flight: 4096
// airfoils, N = 96..512, 17.2 ms against 22.6), and always for systems of
// more than 768 rows.
bool eight_waves(int32_t n_block, int32_t max_n1, int32_t wg_waves) {
    if (max_n1 > 3 * TPB) return true;
    if (wg_waves == 4) return false;
    if (wg_waves == 8) return true;
    return n_block <= device_cus();
}

template <typename T>
hipError_t launch_lu_any(const WsView &v, int32_t B, int32_t max_n1, int32_t wg_waves, int32_t *info,
                         hipStream_t s) {
    if (eight_waves(B, max_n1, wg_waves))
        lu_kernel<T, 16, 3, 512><<<B, 512, 0, s>>>(v, info);   // n1 <= 1536
    else
        lu_kernel<T, 16, 3, TPB><<<B, TPB, 0, s>>>(v, info);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_factor_solve(const WsView &v, int32_t B, int32_t n_block, int32_t max_n1_block,
                               int32_t mixed, double tol, int32_t max_iter, int32_t *info,
                               int32_t persistent, int32_t wg_waves, hipStream_t stream) {
    hipError_t e = hipSuccess;
    if (persistent && (n_block == 0 || !eight_waves(n_block, max_n1_block, wg_waves == 0 ? 4 : wg_waves))) {
        const int n_small = B - n_block;
        const int grid = std::min(2 * device_cus(), n_block + (n_small + TPB / 64 - 1) / (TPB / 64));
        if (mixed)
            batch_kernel<float><<<grid, TPB, 0, stream>>>(v, n_block, B, 1, tol, max_iter, info);
        else
            batch_kernel<double><<<grid, TPB, 0, stream>>>(v, n_block, B, 0, tol, max_iter, info);
        return hipGetLastError();
    }
    if (n_block > 0) {
        e = mixed ? launch_lu_any<float>(v, n_block, max_n1_block, wg_waves, info, stream)
                  : launch_lu_any<double>(v, n_block, max_n1_block, wg_waves, info, stream);
        if (e != hipSuccess) return e;
    }
    e = launch_lu_wave(v, n_block, B - n_block, mixed, info, stream);
    if (e != hipSuccess) return e;
    if (mixed) {
        if (n_block > 0) {
            // the same choice of workgroup size as for the factorisation
            if (eight_waves(n_block, max_n1_block, wg_waves))
                refine_kernel<512><<<n_block, 512, 0, stream>>>(v, info, tol, max_iter);
            else
                refine_kernel<TPB><<<n_block, TPB, 0, stream>>>(v, info, tol, max_iter);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        e = launch_refine_wave(v, n_block, B - n_block, info, tol, max_iter, stream);
    }
    return e;
}

}  // namespace panel
