// lu_wave.hip -- batched LU with partial pivoting, one wavefront per airfoil,
// for systems of up to 64 * WRMAX rows.
//
// Sec. 3 of the paper: every airfoil needs the LU decomposition of its dense
// system, and the population gives many independent systems at once.  For
// the population sizes of a genetic algorithm (thousands of airfoils) there
// are more systems than SIMDs, so here a single wavefront factors a whole
// system and never waits at a workgroup barrier; two such wavefronts share a
// SIMD, and while one runs its pivot search on the vector ALUs the other's
// trailing update runs on the matrix cores.
//
// Algorithm (right-looking, blocked, LAPACK getrf semantics):
//   * super-panels of WSP = 64 columns, split into NB = 16-column pivot
//     panels;
//   * a pivot panel's rows (k0..n-1) are held in registers, row k0 + lane +
//     64 q in slot q.  Pivoting is implicit while the panel is factored:
//     rows stay in their registers, each slot tracks the position its row
//     currently occupies, the pivot search takes the largest |a| among rows
//     not yet used as pivots (lowest current position on ties), and the
//     rank-1 updates skip the rows already used.  The panel is written back
//     with every row at its final position, which is exactly the state
//     LAPACK's explicit row exchanges produce;
//   * the same row moves are applied to every other column as one gather /
//     scatter per column;
//   * the panel updates the super-panel's remaining columns at once
//     (triangular solve on its rows, rank-16 update below);
//   * columns right of the super-panel only receive the row moves until the
//     super-panel is complete; then its four triangular solves and in-band
//     updates turn their top rows into U12, and one rank-64 update
//     A22 -= L21 U12 on the matrix cores finishes the step.
// The K right-hand-side columns ride along, so afterwards they hold
// L^{-1} P b; the wavefront finishes with the back substitution.
#include <climits>

#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr int WL = 64;    // lanes: one wavefront per airfoil
constexpr int WSP = 64;   // super-panel width (rank of the trailing update)
constexpr int WCT = 32;   // trailing columns whose U fragments are held at once
constexpr int WNB = 16;   // pivot panel width

typedef double d4w_t __attribute__((ext_vector_type(4)));
typedef float f4w_t __attribute__((ext_vector_type(4)));

// The trailing updates form D = U^T L^T on v_mfma_*_16x16x4: source A is a
// 16 (columns) x 4 (k) slice of U, source B a 4 (k) x 16 (rows) slice of L,
// so D's row index is a matrix column and its column index a matrix row.
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; element v of lane l holds
// D[c(l, v)][l%16], with c(l, v) measured on gfx950: (l>>4) + 4v for FP64,
// 4(l>>4) + v for FP32.  Either way one accumulator register of the 64 lanes
// covers 16 consecutive rows of four columns.
template <typename T> struct TileMap;
template <> struct TileMap<double> {
    typedef d4w_t acc;
    static __device__ inline int col(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct TileMap<float> {
    typedef f4w_t acc;
    static __device__ inline int col(int lane, int v) { return 4 * (lane >> 4) + v; }
};
__device__ inline d4w_t mfma_t(double a, double b, d4w_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4w_t mfma_t(float a, float b, f4w_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ inline T *sys_of(const WsView &v, const AirfoilMeta &mt);
template <> __device__ inline double *sys_of<double>(const WsView &v, const AirfoilMeta &mt) {
    return v.a64 + mt.a_off;
}
template <> __device__ inline float *sys_of<float>(const WsView &v, const AirfoilMeta &mt) {
    return v.a32 + mt.a_off;
}

// Number of lanes below this one whose bit is set in m.
__device__ inline int lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <typename T> struct WaveLds {
    T l11[WNB][WNB + 1];     // unit-lower diagonal block of a pivot panel
    int mv_src[2 * WNB];     // row moves of the last panel: row mv_src[m]
    int mv_dst[2 * WNB];     //   ends at position mv_dst[m]
    int nmv;
    int ipiv[WNB];           // LAPACK pivots of the last panel (positions)
};

// ---- C[r0:r1, c0:c1) -= A[r0:r1, kb:kb+KD) * A[kb:kb+KD, c0:c1) ------------
// U fragments of WCT columns stay in registers while 16-row tiles of L and C
// stream through.  Rows past r1 and columns past c1 are clamped for the loads
// (their results are discarded), never stored.
template <typename T, int KD>
__device__ void wave_gemm(T *A, int ld, int r0, int r1, int c0, int c1, int kb) {
    constexpr int S = KD / 4;
    constexpr int NT = WCT / 16;
    const int lane = threadIdx.x, i16 = lane & 15, k4 = lane >> 4;
    if (r0 >= r1 || c0 >= c1) return;
    for (int cs = c0; cs < c1; cs += WCT) {
        T uf[NT][S];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = min(cs + 16 * t + i16, c1 - 1);
            const T *up = A + (size_t)c * ld + kb + k4;
#pragma unroll
            for (int s = 0; s < S; ++s) uf[t][s] = up[4 * s];
        }
        int ccol[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) ccol[t][e] = cs + 16 * t + TileMap<T>::col(lane, e);
        for (int rt = r0; rt < r1; rt += 16) {
            const int r = rt + i16;
            const bool rok = r < r1;
            const int rc = rok ? r : r1 - 1;
            T lf[S];
            const T *lp = A + (size_t)(kb + k4) * ld + rc;
#pragma unroll
            for (int s = 0; s < S; ++s) lf[s] = -lp[(size_t)(4 * s) * ld];
            typename TileMap<T>::acc acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[t][e] = A[(size_t)min(ccol[t][e], c1 - 1) * ld + rc];
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma_t(uf[t][s], lf[s], acc[t]);
            if (rok) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ccol[t][e] < c1) A[(size_t)ccol[t][e] * ld + r] = acc[t][e];
            }
        }
    }
}

// ---- one column step of the panel factorisation (C is compile-time) --------
template <typename T, int R, int C>
__device__ __forceinline__ void wave_col(T (&p)[R][WNB], int (&pos)[R], unsigned &live, int k0, int &info,
                                         WaveLds<T> &S) {
    const int lane = threadIdx.x;
    const int g = k0 + C;
    // this lane's candidate among its rows not yet used as pivots
    double best = -1.0;
    int bq = 0, bpos = INT_MAX;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const double a = fabs((double)p[q][C]);
        if (((live >> q) & 1u) && (a > best || (a == best && pos[q] < bpos))) {
            best = a;
            bq = q;
            bpos = pos[q];
        }
    }
    // the wavefront's: exact maximum, lowest current position on ties
    const double wbest = wave_max(best);
    const unsigned long long top = __ballot(best == wbest && best >= 0.0);
    int plane;
    if (top == 0) {
        plane = -1;
    } else if (__popcll(top) == 1) {
        plane = __ffsll((long long)top) - 1;
    } else {
        int cand = (best == wbest) ? bpos : INT_MAX;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cand = min(cand, __shfl_xor(cand, off));
        plane = __ffsll((long long)__ballot(best == wbest && bpos == cand)) - 1;
    }
    if (plane < 0 || !(wbest > 0.0)) {
        // exact zero pivot (or no finite candidate): LAPACK records the
        // column and leaves it; the row now at position g stays there
        if (info == 0) info = g + 1;
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (pos[q] == g) live &= ~(1u << q);
        if (lane == 0) S.ipiv[C] = g;
        return;
    }
    const int pq = __builtin_amdgcn_readlane(bq, plane);
    const int ppos = __builtin_amdgcn_readlane(bpos, plane);
    T u[WNB];
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (q == pq) {
#pragma unroll
            for (int cc = C; cc < WNB; ++cc) u[cc] = readlane_t(p[q][cc], plane);
        }
    const T rinv = T(1) / u[C];
    // the row at position g moves to the pivot row's position, the pivot
    // row to g (and leaves the candidate set)
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (pos[q] == g) pos[q] = ppos;
    if (lane == plane) {
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (q == pq) {
                pos[q] = g;
                live &= ~(1u << q);
            }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if ((live >> q) & 1u) {
            const T l = p[q][C] * rinv;
            p[q][C] = l;
#pragma unroll
            for (int cc = C + 1; cc < WNB; ++cc) p[q][cc] -= l * u[cc];
        }
    }
    if (lane == 0) S.ipiv[C] = ppos;
}

template <typename T, int R, int C>
__device__ __forceinline__ void wave_cols(T (&p)[R][WNB], int (&pos)[R], unsigned &live, int k0, int nb,
                                          int &info, WaveLds<T> &S) {
    if constexpr (C < WNB) {
        if (C < nb) {
            wave_col<T, R, C>(p, pos, live, k0, info, S);
            wave_cols<T, R, C + 1>(p, pos, live, k0, nb, info, S);
        }
    }
}

// ---- factor the panel of columns k0..k0+nb-1 (rows k0..n-1, R = rows/64) --
template <typename T, int R>
__device__ void wave_panel(T *A, int ld, int n, int k0, int nb, int32_t *piv, int &info, WaveLds<T> &S) {
    const int lane = threadIdx.x;
    T p[R][WNB];
    int pos[R];
    unsigned live = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + lane + WL * q;
        pos[q] = r;
        if (r < n) live |= 1u << q;
        const int rr = r < n ? r : n - 1;
#pragma unroll
        for (int cc = 0; cc < WNB; ++cc) {
            const T t = A[(size_t)(k0 + min(cc, nb - 1)) * ld + rr];
            p[q][cc] = (r < n && cc < nb) ? t : T(0);
        }
    }
    if (lane < WNB) {
#pragma unroll
        for (int cc = 0; cc < WNB; ++cc) S.l11[lane][cc] = T(0);
    }

    wave_cols<T, R, 0>(p, pos, live, k0, nb, info, S);

    // rows back at their final positions; the diagonal block to LDS
    int base = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + lane + WL * q;
        if (r < n) {
            T *dst = A + (size_t)k0 * ld + pos[q];
            if (nb == WNB) {
#pragma unroll
                for (int cc = 0; cc < WNB; ++cc) dst[(size_t)cc * ld] = p[q][cc];
            } else {
#pragma unroll
                for (int cc = 0; cc < WNB; ++cc)
                    if (cc < nb) dst[(size_t)cc * ld] = p[q][cc];
            }
            const int d = pos[q] - k0;
            if (d < WNB) {
#pragma unroll
                for (int cc = 0; cc < WNB; ++cc) S.l11[d][cc] = (cc < d) ? p[q][cc] : T(0);
            }
        }
        const bool moved = r < n && pos[q] != r;
        const unsigned long long m = __ballot(moved);
        if (moved) {
            const int idx = base + lanes_below(m);
            S.mv_src[idx] = r;
            S.mv_dst[idx] = pos[q];
        }
        base += __popcll(m);
    }
    if (lane == 0) S.nmv = base;
    __syncthreads();
    if (lane < nb) piv[k0 + lane] = S.ipiv[lane];
}

// ---- apply the panel's row moves to every column outside it ----------------
template <typename T>
__device__ void wave_moves(T *A, int ld, int ncols, int k0, int nb, const WaveLds<T> &S) {
    const int nmv = __builtin_amdgcn_readfirstlane(S.nmv);
    if (nmv == 0) return;
    const int lane = threadIdx.x;
#pragma unroll 1
    for (int j = lane; j < ncols; j += WL) {
        if (j >= k0 && j < k0 + nb) continue;
        T *cp = A + (size_t)j * ld;
        T t[2 * WNB];
#pragma unroll
        for (int m = 0; m < 2 * WNB; ++m)
            if (m < nmv) t[m] = cp[S.mv_src[m]];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < 2 * WNB; ++m)
            if (m < nmv) cp[S.mv_dst[m]] = t[m];
    }
}

// ---- U12 = L11^{-1} A12 on rows k0..k0+15 of columns [c0, c1) ---------------
// One lane per column; L11 (unit lower, zero outside the panel) from LDS.
// Rows past n inside the 16 are zero padding and stay zero.
template <typename T>
__device__ void wave_trsm(T *A, int ld, int k0, int c0, int c1, const WaveLds<T> &S) {
    for (int c = c0 + (int)threadIdx.x; c < c1; c += WL) {
        T *cp = A + (size_t)c * ld + k0;
        T u[WNB];
#pragma unroll
        for (int r = 0; r < WNB; ++r) u[r] = cp[r];
#pragma unroll
        for (int cc = 0; cc < WNB - 1; ++cc) {
            const T uc = u[cc];
#pragma unroll
            for (int r = cc + 1; r < WNB; ++r) u[r] -= S.l11[r][cc] * uc;
            // keep the scheduler from hoisting all 120 LDS reads of L11
            // ahead of the arithmetic (they would not fit in registers)
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int r = 0; r < WNB; ++r) cp[r] = u[r];
    }
}

// ---- back substitution U x = y, y in LDS ------------------------------------
// 64-row diagonal blocks from the bottom: lane = row, the solved entry of
// each step broadcast through a scalar register; then the rows above take
// the block's contribution.
template <typename T>
__device__ void wave_trsv_upper(const T *U, int ld, int n, T *y) {
    const int lane = threadIdx.x;
    for (int rb = ((n - 1) / WL) * WL; rb >= 0; rb -= WL) {
        const int w = min(WL, n - rb);
        const bool in = lane < w;
        const int r = rb + (in ? lane : 0);
        T yi = in ? y[r] : T(0);
        const T dinv = in ? T(1) / U[(size_t)r * ld + r] : T(0);
        for (int j = w - 1; j >= 0; --j) {
            const T ucol = U[(size_t)(rb + j) * ld + r];
            if (lane == j) yi *= dinv;
            const T xj = readlane_t(yi, j);
            if (lane < j) yi -= ucol * xj;
        }
        if (in) y[r] = yi;
        __syncthreads();
        for (int rr = lane; rr < rb; rr += WL) {
            const T *up = U + (size_t)rb * ld + rr;
            T s0 = y[rr], s1 = T(0);
            int j = 0;
            for (; j + 1 < w; j += 2) {
                s0 -= up[(size_t)j * ld] * y[rb + j];
                s1 -= up[(size_t)(j + 1) * ld] * y[rb + j + 1];
            }
            if (j < w) s0 -= up[(size_t)j * ld] * y[rb + j];
            y[rr] = s0 + s1;
        }
        __syncthreads();
    }
}

template <typename T, int R>
__device__ __forceinline__ bool panel_if(int rows, T *A, int ld, int n, int k0, int nb, int32_t *piv,
                                         int &info, WaveLds<T> &S) {
    if (rows != R) return false;
    wave_panel<T, R>(A, ld, n, k0, nb, piv, info, S);
    return true;
}

template <typename T>
__global__ __launch_bounds__(WL, 2) void lu_wave_kernel(WsView v, int32_t first, int32_t *__restrict__ info_out) {
    const int b = v.order[first + blockIdx.x];
    const AirfoilMeta mt = v.meta[b];
    const int n = mt.n1, ld = mt.ld, ncols = mt.n1 + mt.K;
    const int lane = threadIdx.x;
    double *X = v.x + mt.x_off;

    if (v.flag[b] != 0) {   // screened out by the assembly
        if (lane == 0) info_out[b] = -1;
        for (int i = lane; i < n * mt.K; i += WL) X[i] = __builtin_nan("");
        return;
    }

    T *A = sys_of<T>(v, mt);
    int32_t *piv = v.piv + mt.piv_off;
    __shared__ WaveLds<T> S;
    __shared__ T y[WL * PANEL_WAVE_RMAX];
    int info = 0;

    for (int K0 = 0; K0 < n; K0 += WSP) {
        const int kend = min(K0 + WSP, n);
        for (int k0 = K0; k0 < kend; k0 += WNB) {
            const int nb = min(WNB, n - k0);
            const int rows = (n - k0 + WL - 1) / WL;
            panel_if<T, 1>(rows, A, ld, n, k0, nb, piv, info, S) ||
                panel_if<T, 2>(rows, A, ld, n, k0, nb, piv, info, S) ||
                panel_if<T, 3>(rows, A, ld, n, k0, nb, piv, info, S) ||
                panel_if<T, 4>(rows, A, ld, n, k0, nb, piv, info, S) ||
                panel_if<T, 5>(rows, A, ld, n, k0, nb, piv, info, S);
            __syncthreads();
            wave_moves<T>(A, ld, ncols, k0, nb, S);
            __syncthreads();
            const int c0 = k0 + nb;
            if (c0 < kend) {
                wave_trsm<T>(A, ld, k0, c0, kend, S);
                __syncthreads();
                wave_gemm<T, WNB>(A, ld, c0, n, c0, kend, k0);
                __syncthreads();
            }
        }
        if (kend < ncols) {
            for (int kp = K0; kp < kend; kp += WNB) {
                const int nbp = min(WNB, kend - kp);
                if (lane < WNB) {
                    const T *lrow = A + (size_t)kp * ld + kp + lane;
#pragma unroll
                    for (int cc = 0; cc < WNB; ++cc)
                        S.l11[lane][cc] = (cc < lane && lane < nbp) ? lrow[(size_t)cc * ld] : T(0);
                }
                __syncthreads();
                wave_trsm<T>(A, ld, kp, kend, ncols, S);
                __syncthreads();
                if (kp + WNB < kend) {
                    wave_gemm<T, WNB>(A, ld, kp + WNB, kend, kend, ncols, kp);
                    __syncthreads();
                }
            }
            if (kend < n) {
                wave_gemm<T, WSP>(A, ld, kend, n, kend, ncols, K0);
                __syncthreads();
            }
        }
    }

    if (lane == 0) {
        info_out[b] = info;
        v.flag[b] = info;
    }
    if (info != 0) {
        for (int i = lane; i < n * mt.K; i += WL) X[i] = __builtin_nan("");
        return;
    }
    for (int k = 0; k < mt.K; ++k) {
        for (int i = lane; i < n; i += WL) y[i] = A[(size_t)(n + k) * ld + i];
        __syncthreads();
        wave_trsv_upper<T>(A, ld, n, y);
        for (int i = lane; i < n; i += WL) X[(size_t)k * n + i] = (double)y[i];
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_lu_wave(const WsView &v, int32_t first, int32_t count, int32_t mixed, int32_t *info,
                          hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    if (mixed)
        lu_wave_kernel<float><<<count, WL, 0, stream>>>(v, first, info);
    else
        lu_wave_kernel<double><<<count, WL, 0, stream>>>(v, first, info);
    return hipGetLastError();
}

}  // namespace panel
