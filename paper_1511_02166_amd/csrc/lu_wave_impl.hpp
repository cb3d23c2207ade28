// lu_wave_impl.hpp -- one wavefront factors one system: batched LU with
// partial pivoting, the solve, and the FP64 refinement of FP32 factors, for
// systems of up to 64 * PANEL_WAVE_RMAX rows.  Device functions only; the
// kernels that run them (one wavefront per workgroup, or four per workgroup
// in the persistent batch kernel) include this file.
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
//   * inside the super-panel the update is left-looking: before a panel is
//     factored, its 16 columns take the triangular solves and the rank-16p
//     update from the p panels before it in one pass (each column block is
//     read and written once, instead of once per earlier panel);
//   * columns right of the super-panel only receive the row moves until the
//     super-panel is complete; then its four triangular solves and in-band
//     updates turn their top rows into U12, and one rank-64 update
//     A22 -= L21 U12 on the matrix cores finishes the step.
// The K right-hand-side columns ride along, so afterwards they hold
// L^{-1} P b; the wavefront finishes with the back substitution.
#pragma once

#include <climits>

#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {
namespace wv {

// This wavefront's lane (0..63), whatever the workgroup size.
__device__ __forceinline__ int wlane() { return (int)(threadIdx.x & 63u); }

// Order this wavefront's LDS and global accesses before and after this point
// (the wavefront only ever exchanges data with itself).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


constexpr int WL = 64;    // lanes: one wavefront per airfoil
constexpr int WSP = 64;   // super-panel width (rank of the trailing update)
// trailing columns whose U fragments are held in registers at once (as many
// as fit in the register budget without spilling)
template <typename T> struct Wct;
template <> struct Wct<double> { static constexpr int v = 48; };
template <> struct Wct<float> { static constexpr int v = 64; };
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
// For the untransposed products D = M Y of the band solve, D must come out in
// the layout the B operand uses (lane l, index s holds row 4s + l/16), so
// the result can feed the next product without leaving the registers.  For
// FP64 that is D's own layout; for FP32 the rows of M are supplied permuted,
// row arow(i) in place of row i, which turns D's layout into it.
template <> struct TileMap<double> {
    typedef d4w_t acc;
    static __device__ inline int col(int lane, int v) { return (lane >> 4) + 4 * v; }
    static __device__ inline int arow(int i) { return i; }
};
template <> struct TileMap<float> {
    typedef f4w_t acc;
    static __device__ inline int col(int lane, int v) { return 4 * (lane >> 4) + v; }
    static __device__ inline int arow(int i) { return 4 * (i & 3) + (i >> 2); }
};
__device__ inline d4w_t mfma_t(double a, double b, d4w_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4w_t mfma_t(float a, float b, f4w_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Hide a value from loop-invariant code motion.  Without this the compiler
// forms address offsets (from ld) and lane-dependent constants once at the
// start of the kernel and keeps them live across every phase, which pushes
// the FP64 kernel past its 256 registers and spills them to scratch memory;
// behind the barrier they are formed where they are used.
__device__ __forceinline__ int opaque_s(int v) {
    v = __builtin_amdgcn_readfirstlane(v);   // uniform by contract (free if already scalar)
    asm volatile("" : "+s"(v));
    return v;
}
__device__ __forceinline__ int opaque_v(int v) {
    asm volatile("" : "+v"(v));
    return v;
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
    T linv[WSP / WNB][WNB][WNB + 1];   // inverses of the super-panel's diagonal blocks
    int mv_src[2 * WNB];     // row moves of the last panel: row mv_src[m]
    int mv_dst[2 * WNB];     //   ends at position mv_dst[m]
    int nmv;
    int ipiv[WNB];           // LAPACK pivots of the last panel (positions)
    // The pivot panels' buffers and the U tile of a super-panel's trailing
    // update are never in use at the same time: they share their memory.
    union {
        struct {
            T l11[WNB][WNB + 1];     // unit-lower diagonal block of a pivot panel
            T ub[WSP - WNB][WNB];    // U rows of the next panel's columns (left-looking step)
        };
        T ut[WSP / 4][WL];           // -U of one 16-column tile, A-operand order (k-step, lane)
    };
};

// ---- block update after pivot panels: band solve + trailing product --------
// For the columns [c0, c1) and the band of rows [kb, kb + 16 nblk) below
// which the panels kb.. have been factored (row moves already applied):
//   U  = L_band^{-1} A[band, c0:c1)      (L_band: unit lower, 16 nblk square)
//   A[kend:n, c0:c1) -= A[kend:n, band] U      (only if kend < n; then the
//                                               band is the full 16 NBLK)
// WCT columns at a time.  The band of those columns is loaded once into
// B-operand fragments (lane l, index s: row kb + 4s + l/16, column l%16 of a
// 16-column tile), solved in registers block by block on the matrix cores
// (X_i = linv_i Y_i, then Y_j -= L_ji X_i), stored once, and kept as the U
// fragments of the trailing product.  The trailing product streams 16-row
// tiles of L and C, downwards or upwards (`up`): each L fragment of the next
// tile goes into the register the current tile's product has just consumed,
// the products start from zero and the tile's C block, loaded after the
// previous tile's stores, is added after them.  Rows past n / columns past
// c1 are clamped for the loads and never stored; rows of the band past n are
// zero padding (linv is the identity there).
// One chunk of NT 16-column tiles starting at column cs (columns past c1
// are clamped for the loads and never stored).  With NL = 1 the trailing
// product also updates the tile of columns [cf, c1) (at most 16, whose band
// rows have been solved already) with its -U fragments in LDS: the last
// narrow tile of a block rides with the last full chunk instead of making a
// pass over L of its own.
template <typename T, int NBLK, int NT, bool TRAIL = true, int NL = 0>
__device__ __forceinline__ void update_chunk(T *A, int ld, int n, int kb, int kend, int cs, int c1,
                                             WaveLds<T> &S, int slot0, int nblk, int cf = 0, int up = 0) {
    ld = opaque_s(ld);
    constexpr int S4 = 4 * NBLK;   // k-steps (4 rows each) of the band
    typedef typename TileMap<T>::acc acc_t;
    const int lane = wlane(), i16 = lane & 15, k4 = lane >> 4;
    const int ar = TileMap<T>::arow(i16);
    T uf[NT][S4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = min(cs + 16 * t + i16, c1 - 1);
        const T *up = A + (size_t)c * ld + kb + k4;
#pragma unroll
        for (int s = 0; s < S4; ++s) uf[t][s] = (s < 4 * nblk) ? up[4 * s] : T(0);
    }
    // the band's off-diagonal blocks L[block i2][block i] (i < i2), rows
    // permuted by arow, all loaded here at once; a pair past nblk reads a
    // block that exists (i clamped to nblk - 2, i2 to nblk - 1, the diagonal
    // block when nblk == 1) and goes unused
    constexpr int NP = NBLK * (NBLK - 1) / 2;
    T lb[NP > 0 ? NP : 1][4];
#pragma unroll
    for (int i = 0, q = 0; i < NBLK; ++i)
#pragma unroll
        for (int i2 = i + 1; i2 < NBLK; ++i2, ++q) {
            const int ic = min(i, max(nblk - 2, 0)), i2c = min(i2, nblk - 1);
            const T *lp = A + (size_t)(kb + 16 * ic + k4) * ld + kb + 16 * i2c + ar;
#pragma unroll
            for (int s = 0; s < 4; ++s) lb[q][s] = lp[(size_t)(4 * s) * ld];
        }
    // band solve, block by block: X_i = linv_i Y_i, then Y_i2 += L_i2,i (-X_i)
    // (the sign goes on X_i, which is in registers already, so the L blocks
    // are used as loaded and their loads are waited for only where needed)
#pragma unroll
    for (int i = 0, q0 = 0; i < NBLK; q0 += NBLK - 1 - i, ++i) {
        if (i < nblk) {
            T li[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) li[s] = S.linv[slot0 + i][ar][4 * s + k4];
            T xn[NT][4];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc_t acc;
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[e] = T(0);
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = mfma_t(li[s], uf[t][4 * i + s], acc);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uf[t][4 * i + e] = acc[e];
                    xn[t][e] = -acc[e];
                    asm volatile("" : "+v"(xn[t][e]));
                }
            }
#pragma unroll
            for (int i2 = i + 1; i2 < NBLK; ++i2) {
                if (i2 < nblk) {
                    const int q = q0 + (i2 - i - 1);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        acc_t acc;
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[e] = uf[t][4 * i2 + e];
#pragma unroll
                        for (int s = 0; s < 4; ++s) acc = mfma_t(lb[q][s], xn[t][s], acc);
#pragma unroll
                        for (int e = 0; e < 4; ++e) uf[t][4 * i2 + e] = acc[e];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = cs + 16 * t + i16;
        if (c < c1) {
            T *up = A + (size_t)c * ld + kb + k4;
#pragma unroll
            for (int s = 0; s < S4; ++s)
                if (s < 4 * nblk) up[4 * s] = uf[t][s];
        }
    }
    if (!TRAIL || kend >= n) return;

    // trailing product A[kend:n, cs:cs+16NT) -= A[kend:n, band] U, formed as
    // A + L (-U): the U fragments are negated once here, so the streamed L
    // fragments go to the matrix cores as loaded (a sign flip on a loaded
    // value makes the compiler wait for the load where it flips it, which
    // would stall each tile on the next tile's prefetch)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < S4; ++s) {
            uf[t][s] = -uf[t][s];
            asm volatile("" : "+v"(uf[t][s]));   // keep the flip here, not at each use
        }
    static_assert(NL == 0 || NL == 1, "at most one tile in LDS");
    if constexpr (NL == 1) {
        const int c = min(cf + i16, c1 - 1);
        const T *up = A + (size_t)c * ld + kb + k4;
#pragma unroll
        for (int s = 0; s < S4; ++s) S.ut[s][lane] = (s < 4 * nblk) ? -up[4 * s] : T(0);
        wave_sync();
    }
    constexpr int NU = NT + NL;   // tiles of the trailing product
    int coff[NU][4];   // element offsets of this lane's C columns (clamped)
    bool cok[NU][4];
#pragma unroll
    for (int t = 0; t < NU; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = (t < NT ? cs + 16 * t : cf) + TileMap<T>::col(lane, e);
            cok[t][e] = c < c1;
            coff[t][e] = min(c, c1 - 1) * ld;
        }
    const T *lcol = A + (size_t)(kb + k4) * ld;
    if constexpr (NL == 0 && (NBLK == 1 || (NT == 1 && NBLK <= 3))) {
        // little work per tile (at most 12 dependent products): D tiles in
        // flight; each step computes one tile and issues the loads of the
        // tile D - 1 ahead into the slot just freed
        constexpr int D = 4;
        T lf[D][S4];
        acc_t acc[D][NT];
        auto load_tile = [&](int slot, int rt) {
            const int rr = min(rt + i16, n - 1);
#pragma unroll
            for (int s = 0; s < S4; ++s) lf[slot][s] = lcol[(size_t)(4 * s) * ld + rr];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[slot][t][e] = A[coff[t][e] + rr];
        };
#pragma unroll
        for (int d = 0; d < D - 1; ++d) load_tile(d, kend + 16 * d);
        for (int rt = kend; rt < n; rt += 16 * D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int r0 = rt + 16 * d;
                load_tile((d + D - 1) % D, r0 + 16 * (D - 1));
                if (r0 < n) {
#pragma unroll
                    for (int s = 0; s < S4; ++s)
#pragma unroll
                        for (int t = 0; t < NT; ++t) acc[d][t] = mfma_t(uf[t][s], lf[d][s], acc[d][t]);
                    const int r = r0 + i16;
                    if (r < n) {
#pragma unroll
                        for (int t = 0; t < NT; ++t)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (cok[t][e]) A[coff[t][e] + r] = acc[d][t][e];
                    }
                }
            }
        }
    } else {
        // 16 x 16NT x 64 per tile.  The products start from zero and the
        // tile's C block is added after them: C of the next tile is loaded
        // right after this tile's stores, each L fragment of the next tile
        // into the register this tile's product has just consumed.  Every
        // wait is then for loads issued about one tile earlier.
        // the row tiles downwards, or upwards when up != 0 (consecutive chunks
        // alternate, so each starts on the L tiles the one before ended on)
        const int ntile = (n - kend + 15) / 16, step = up ? -16 : 16;
        const int rt0 = up ? kend + 16 * (ntile - 1) : kend;
        T lf[S4];
        T cb[NU][4];
        const int rc = min(rt0 + i16, n - 1);
#pragma unroll
        for (int s = 0; s < S4; ++s) lf[s] = lcol[(size_t)(4 * s) * ld + rc];
#pragma unroll
        for (int t = 0; t < NU; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) cb[t][e] = A[coff[t][e] + rc];
        // the first tile's operands complete here, so that inside the loop
        // only the loop's own issue order decides what each product waits for
#pragma unroll
        for (int s = 0; s < S4; ++s) asm volatile("" ::"v"(lf[s]));
        for (int it = 0, rt = rt0; it < ntile; ++it, rt += step) {
            const int r = rt + i16;
            const int rn = min(max(r + step, kend), n - 1);   // next tile's row (clamped)
            acc_t acc[NU];
#pragma unroll
            for (int t = 0; t < NU; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[t][e] = T(0);
            // the LDS tile is read in the loop (hoisted out of it, its 16
            // fragments would take the registers of a fourth tile)
            const T *ut = &S.ut[0][lane] + opaque_s(0);
#pragma unroll
            for (int s = 0; s < S4; ++s) {
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma_t(uf[t][s], lf[s], acc[t]);
                if constexpr (NL == 1) acc[NT] = mfma_t(ut[s * WL], lf[s], acc[NT]);
                lf[s] = lcol[(size_t)(4 * s) * ld + rn];
            }
            if (r < n) {
#pragma unroll
                for (int t = 0; t < NU; ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (cok[t][e]) A[coff[t][e] + r] = cb[t][e] + acc[t][e];
            }
#pragma unroll
            for (int t = 0; t < NU; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) cb[t][e] = A[coff[t][e] + rn];
        }
    }
}

// The last chunk of a block update: exactly as many 16-column tiles as are
// left (1 .. R), so it makes one pass over L like a full chunk.
template <typename T, int NBLK, int R>
__device__ __forceinline__ void update_rest(int tiles, T *A, int ld, int n, int kb, int kend, int cs, int c1,
                                            WaveLds<T> &S, int slot0, int nblk, int up) {
    if constexpr (R >= 1) {
        if (tiles == R)
            update_chunk<T, NBLK, R>(A, ld, n, kb, kend, cs, c1, S, slot0, nblk, 0, up);
        else
            update_rest<T, NBLK, R - 1>(tiles, A, ld, n, kb, kend, cs, c1, S, slot0, nblk, up);
    }
}

template <typename T, int NBLK>
__device__ __forceinline__ void wave_update(T *A, int ld, int n, int kb, int kend, int c0, int c1,
                                            WaveLds<T> &S, int slot0) {
    constexpr int NTM = Wct<T>::v / 16;
    const int nblk = min(NBLK, (kend - kb + WNB - 1) / WNB);
    // full chunks, then one of the remaining width (a trailing block of
    // n1 + K columns is rarely a multiple of the chunk width)
    // (FP32: at most two tiles at a time in the rest, which keeps the kernel
    // free of scratch spills)
    constexpr int RM = sizeof(T) == 8 ? NTM - 1 : 2;
    // The chunks go from the right end to the left: the leftmost columns,
    // which the next super-panel's panels read first, are written last and
    // are then more likely still in the caches.
    const int nfull = (c1 - c0) / (16 * NTM), rest = c1 - c0 - 16 * NTM * nfull;
    if (nfull >= 1 && rest > 0 && rest <= 16) {
        // a last tile of at most 16 columns (often the last matrix column and
        // the right-hand sides) rides with the last full chunk: its band rows
        // are solved first, on their own
        const int cf = c0 + 16 * NTM * nfull;
        update_chunk<T, NBLK, 1, false>(A, ld, n, kb, kend, cf, c1, S, slot0, nblk);
        wave_sync();
        int cs = cf - 16 * NTM, up = 0;
        update_chunk<T, NBLK, NTM, true, 1>(A, ld, n, kb, kend, cs, c1, S, slot0, nblk, cf, up);
        for (cs -= 16 * NTM; cs >= c0; cs -= 16 * NTM) {
            up ^= 1;
            update_chunk<T, NBLK, NTM>(A, ld, n, kb, kend, cs, c1, S, slot0, nblk, 0, up);
        }
        return;
    }
    int ce = c0;   // end of the full chunks (the last may run past c1, clamped)
    while (c1 - ce > 16 * (NTM - 1)) ce += 16 * NTM;
    int up = 1;
    for (int cs = ce; cs < c1;) {
        const int tiles = min(RM, (c1 - cs + 15) / 16);
        up ^= 1;
        update_rest<T, NBLK, RM>(tiles, A, ld, n, kb, kend, cs, c1, S, slot0, nblk, up);
        cs += 16 * tiles;
    }
    for (int cs = ce - 16 * NTM; cs >= c0; cs -= 16 * NTM) {
        up ^= 1;
        update_chunk<T, NBLK, NTM>(A, ld, n, kb, kend, cs, c1, S, slot0, nblk, 0, up);
    }
}

// ---- one column step of the panel factorisation (C is compile-time) --------
template <typename T, int R, int C>
__device__ __forceinline__ void wave_col(T (&p)[R][WNB], int (&pos)[R], unsigned &live, int k0, int &info,
                                         WaveLds<T> &S) {
    const int lane = wlane();
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
__device__ __forceinline__ void wave_panel(T *A, int ld, int n, int k0, int nb, int kb, int32_t *piv, int &info,
                                           WaveLds<T> &S) {
    ld = opaque_s(ld);
    const int lane = wlane();
    T p[R][WNB];
    int pos[R];
    unsigned live = 0;
    // every load is issued (clamped addresses) before any is masked: with
    // the mask next to the load the compiler put each load in a branch of
    // its own and waited for it there, one memory latency per element
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int rr = min(k0 + lane + WL * q, n - 1);
#pragma unroll
        for (int cc = 0; cc < WNB; ++cc) p[q][cc] = A[(size_t)(k0 + min(cc, nb - 1)) * ld + rr];
    }
    __builtin_amdgcn_sched_barrier(0);
    // left-looking update from the super-panel's panels before this one
    // (band rows kb..k0, U block in LDS): A[k0:n, panel] -= L[k0:n, kb:k0] U,
    // on the vector ALUs in the row-per-lane layout of the factorisation, so
    // the updated panel never goes back to memory before it is factored
    // (the FP64 vector rate equals the FP64 matrix rate on this GPU)
    // (up to four slots of rows: with five the registers would spill, and
    // the caller updates such panels in memory first)
    // band columns per round trip of L loads: as many as the registers left
    // by the panel's R row slots allow (k0 - kb is a multiple of 16)
    constexpr int JG = R == 1 ? 16 : R == 2 ? 8 : R == 3 ? 4 : 2;
    if constexpr (R <= 4)
    for (int j0 = kb; j0 < k0; j0 += JG) {
        T l[JG][R];
#pragma unroll
        for (int jj = 0; jj < JG; ++jj)
#pragma unroll
            for (int q = 0; q < R; ++q)
                l[jj][q] = A[(size_t)(j0 + jj) * ld + min(k0 + lane + WL * q, n - 1)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int jj = 0; jj < JG; ++jj) {
#pragma unroll
            for (int cc = 0; cc < WNB; ++cc) {
                const T u = S.ub[j0 + jj - kb][cc];
#pragma unroll
                for (int q = 0; q < R; ++q) p[q][cc] -= l[jj][q] * u;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = k0 + lane + WL * q;
        pos[q] = r;
        if (r < n) live |= 1u << q;
#pragma unroll
        for (int cc = 0; cc < WNB; ++cc) p[q][cc] = (r < n && cc < nb) ? p[q][cc] : T(0);
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
    wave_sync();
    if (lane < nb) piv[k0 + lane] = S.ipiv[lane];
}

// ---- apply the panel's row moves to every column outside it ----------------
// M loads per column, issued together whatever nmv (<= M) is: moves past
// nmv repeat the last one, which reads and writes the same element with the
// same value.  (Each load under its own m < nmv test went into a branch of
// its own and was waited for there, one memory latency per move.)
template <typename T, int M>
__device__ __forceinline__ void wave_moves_m(T *A, int ld, int ncols, int k0, int nb, int nmv,
                                             const WaveLds<T> &S) {
    const int lane = wlane();
    int src[M], dst[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int mm = min(m, nmv - 1);
        src[m] = S.mv_src[mm];
        dst[m] = S.mv_dst[mm];
    }
#pragma unroll 1
    for (int j = lane; j < ncols; j += WL) {
        if (j >= k0 && j < k0 + nb) continue;
        T *cp = A + (size_t)j * ld;
        T t[M];
        // every element read before any is written (a row may be both the
        // source of one move and the destination of another)
#pragma unroll
        for (int m = 0; m < M; ++m) t[m] = cp[src[m]];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < M; ++m) cp[dst[m]] = t[m];
    }
}

template <typename T>
__device__ __forceinline__ void wave_moves(T *A, int ld, int ncols, int k0, int nb, const WaveLds<T> &S) {
    const int nmv = __builtin_amdgcn_readfirstlane(S.nmv);
    if (nmv == 0) return;
    ld = opaque_s(ld);
    if (nmv <= 2)
        wave_moves_m<T, 2>(A, ld, ncols, k0, nb, nmv, S);
    else if (nmv <= 8)
        wave_moves_m<T, 8>(A, ld, ncols, k0, nb, nmv, S);
    else
        wave_moves_m<T, 2 * WNB>(A, ld, ncols, k0, nb, nmv, S);
}

// ---- inverse of the panel's unit-lower diagonal block: linv = l11^{-1} -----
// Lane j < 16 solves L x = e_j by forward substitution (L from LDS).
template <typename T>
__device__ __forceinline__ void wave_linv(WaveLds<T> &S, int slot) {
    const int lane = opaque_v(wlane());
    if (lane < WNB) {
        T x[WNB];
#pragma unroll
        for (int r = 0; r < WNB; ++r) x[r] = (r == lane) ? T(1) : T(0);
#pragma unroll
        for (int cc = 0; cc < WNB - 1; ++cc) {
            const T xc = x[cc];
#pragma unroll
            for (int r = cc + 1; r < WNB; ++r) x[r] -= S.l11[r][cc] * xc;
            // keep the scheduler from hoisting all 120 LDS reads of L11
            // ahead of the arithmetic (they would not fit in registers)
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int r = 0; r < WNB; ++r) S.linv[slot][r][lane] = x[r];
    }
}

// ---- back substitution U x = y, y in LDS ------------------------------------
// 64-row diagonal blocks from the bottom: lane = row, with the lane's row of
// the block loaded into registers 32 columns at a time (one round trip each),
// and the solved entry of each step broadcast through a scalar register; then
// the rows above take the block's contribution, again 32 columns per round
// trip.  (All 64 FP64 entries at once took 128 registers; the compiler then
// spilled them and waited for each load on its own.)
template <typename T, bool BATCH>
__device__ __forceinline__ void wave_trsv_upper(const T *U, int ld, int n, T *y) {
    constexpr int H = WL / 2;
    ld = opaque_s(ld);
    const int lane = wlane();
    for (int rb = ((n - 1) / WL) * WL; rb >= 0; rb -= WL) {
        const int w = min(WL, n - rb);
        const bool in = lane < w;
        const int r = rb + (in ? lane : 0);
        T yi = in ? y[r] : T(0);
        const T dinv = in ? T(1) / U[(size_t)r * ld + r] : T(0);
        // the block's columns from the last down, the upper half first
#pragma unroll 1
        for (int h = 1; h >= 0; --h) {
            const int j0 = H * h;
            T ub[H];
#pragma unroll
            for (int j = 0; j < H; ++j) ub[j] = U[(size_t)(rb + min(j0 + j, w - 1)) * ld + r];
#pragma unroll
            for (int j = H - 1; j >= 0; --j) {
                const int jj = j0 + j;
                if (jj < w) {
                    if (lane == jj) yi *= dinv;
                    const T xj = readlane_t(yi, jj);
                    if (lane < jj) yi -= ub[j] * xj;
                }
            }
        }
        if (in) y[r] = yi;
        wave_sync();
        for (int rr = lane; rr < rb; rr += WL) {
            const T *up = U + (size_t)rb * ld + rr;
            T s0 = y[rr], s1 = T(0);
            if constexpr (BATCH) {
#pragma unroll 1
                for (int j0 = 0; j0 < WL; j0 += H) {
                    T ub[H];
#pragma unroll
                    for (int j = 0; j < H; ++j) ub[j] = up[(size_t)min(j0 + j, w - 1) * ld];
                    // the block's solution, read from LDS here (hoisted out
                    // of the loop it would hold 64 more registers)
                    const T *yb = y + opaque_s(rb + j0);
#pragma unroll
                    for (int j = 0; j < H; j += 2) {
                        const T x0 = (j0 + j < w) ? yb[j] : T(0);
                        const T x1 = (j0 + j + 1 < w) ? yb[j + 1] : T(0);
                        s0 -= ub[j] * x0;
                        s1 -= ub[j + 1] * x1;
                    }
                }
            } else {
                int j = 0;
#pragma unroll 8
                for (; j + 1 < w; j += 2) {
                    s0 -= up[(size_t)j * ld] * y[rb + j];
                    s1 -= up[(size_t)(j + 1) * ld] * y[rb + j + 1];
                }
                if (j < w) s0 -= up[(size_t)j * ld] * y[rb + j];
            }
            y[rr] = s0 + s1;
        }
        wave_sync();
    }
}

template <typename T, int R>
__device__ __forceinline__ bool panel_if(int rows, T *A, int ld, int n, int k0, int nb, int kb, int32_t *piv,
                                         int &info, WaveLds<T> &S) {
    if (rows != R) return false;
    wave_panel<T, R>(A, ld, n, k0, nb, kb, piv, info, S);
    return true;
}

// U rows of the panel's columns [k0, k0 + nb) from the band kb..k0 (the
// super-panel's panels before it), and the U block to LDS for the panel's
// left-looking update.
template <typename T, int NBLK>
__device__ __forceinline__ void wave_band_u(T *A, int ld, int n, int kb, int k0, int nb, WaveLds<T> &S) {
    update_chunk<T, NBLK, 1, false>(A, ld, n, kb, k0, k0, k0 + nb, S, 0, NBLK);
    wave_sync();
    ld = opaque_s(ld);
    for (int idx = wlane(); idx < WNB * WNB * NBLK; idx += WL) {
        const int j = idx / WNB, c = idx % WNB;
        S.ub[j][c] = c < nb ? A[(size_t)(k0 + c) * ld + kb + j] : T(0);
    }
}

// LDS of one wavefront's factorisation.
template <typename T> struct WaveLuLds {
    WaveLds<T> S;
    T y[WL * PANEL_WAVE_RMAX];
};

// Factor airfoil b's system in place and solve its K right-hand sides, one
// wavefront (any wavefront of the workgroup: it synchronises with itself
// only).
template <typename T>
__device__ __forceinline__ void wave_lu(const WsView &v, int b, int32_t *__restrict__ info_out, WaveLuLds<T> &W) {
    const AirfoilMeta mt = v.meta[b];
    const int n = mt.n1, ld = mt.ld, ncols = mt.n1 + mt.K;
    const int lane = wlane();
    double *X = v.x + mt.x_off;

    if (v.flag[b] != 0 || n > WL * PANEL_WAVE_RMAX) {
        // screened out by the assembly (-1), or a system too large for one
        // wavefront (-3: the workspace's airfoil order does not match the
        // plan it is used with)
        const int code = v.flag[b] != 0 ? -1 : -3;
        if (lane == 0) {
            info_out[b] = code;
            v.flag[b] = code;
        }
        for (int i = lane; i < n * mt.K; i += WL) X[i] = __builtin_nan("");
        return;
    }

    T *A = sys_of<T>(v, mt);
    int32_t *piv = v.piv + mt.piv_off;
    WaveLds<T> &S = W.S;
    T *y = W.y;
    int info = 0;

    for (int K0 = 0; K0 < n; K0 += WSP) {
        const int kend = min(K0 + WSP, n);
        for (int k0 = K0; k0 < kend; k0 += WNB) {
            const int nb = min(WNB, n - k0);
            const int rows = (n - k0 + WL - 1) / WL;
            // The panel's columns take the update from the super-panel's
            // panels before it (left-looking inside the super-panel): their
            // U rows here, the rows below inside the panel factorisation
            // (in registers), or, for panels of five row slots, in memory.
            int kb = K0;
            if (rows <= 4) {
                if (k0 - K0 == WNB) wave_band_u<T, 1>(A, ld, n, K0, k0, nb, S);
                if (k0 - K0 == 2 * WNB) wave_band_u<T, 2>(A, ld, n, K0, k0, nb, S);
                if (k0 - K0 == 3 * WNB) wave_band_u<T, 3>(A, ld, n, K0, k0, nb, S);
            } else {
                if (k0 - K0 == WNB) wave_update<T, 1>(A, ld, n, K0, k0, k0, k0 + nb, S, 0);
                if (k0 - K0 == 2 * WNB) wave_update<T, 2>(A, ld, n, K0, k0, k0, k0 + nb, S, 0);
                if (k0 - K0 == 3 * WNB) wave_update<T, 3>(A, ld, n, K0, k0, k0, k0 + nb, S, 0);
                kb = k0;
            }
            if (k0 > K0) wave_sync();
            panel_if<T, 1>(rows, A, ld, n, k0, nb, kb, piv, info, S) ||
                panel_if<T, 2>(rows, A, ld, n, k0, nb, kb, piv, info, S) ||
                panel_if<T, 3>(rows, A, ld, n, k0, nb, kb, piv, info, S) ||
                panel_if<T, 4>(rows, A, ld, n, k0, nb, kb, piv, info, S) ||
                panel_if<T, 5>(rows, A, ld, n, k0, nb, kb, piv, info, S);
            wave_sync();
            wave_moves<T>(A, ld, ncols, k0, nb, S);
            wave_linv<T>(S, (k0 - K0) / WNB);
            wave_sync();
        }
        // columns right of the super-panel: U12 rows and the rank-64 update
        if (kend < ncols) {
            wave_update<T, WSP / WNB>(A, ld, n, K0, kend, kend, ncols, S, 0);
            wave_sync();
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
        wave_sync();
        wave_trsv_upper<T, true>(A, ld, n, y);
        for (int i = lane; i < n; i += WL) X[(size_t)k * n + i] = (double)y[i];
        wave_sync();
    }
}

// ---- forward substitution L y = y (unit lower), y in LDS --------------------
// Same blocking as the back substitution, top down.
template <typename T>
__device__ __forceinline__ void wave_trsv_lower_unit(const T *L, int ld, int n, T *y) {
    const int lane = wlane();
    for (int rb = 0; rb < n; rb += WL) {
        const int w = min(WL, n - rb);
        const bool in = lane < w;
        const int r = rb + (in ? lane : 0);
        T lb[WL];
#pragma unroll
        for (int j = 0; j < WL; ++j) lb[j] = L[(size_t)(rb + min(j, w - 1)) * ld + r];
        T yi = in ? y[r] : T(0);
#pragma unroll
        for (int j = 0; j < WL; ++j) {
            if (j < w) {
                const T xj = readlane_t(yi, j);
                if (lane > j) yi -= lb[j] * xj;
            }
        }
        if (in) y[r] = yi;
        wave_sync();
        for (int rr = rb + w + lane; rr < n; rr += WL) {
            // rows below a block exist only when the block is full (w == 64)
            const T *lp = L + (size_t)rb * ld + rr;
            T s0 = y[rr], s1 = T(0);
#pragma unroll 8
            for (int j = 0; j < WL; j += 2) {
                s0 -= lp[(size_t)j * ld] * y[rb + j];
                s1 -= lp[(size_t)(j + 1) * ld] * y[rb + j + 1];
            }
            y[rr] = s0 + s1;
        }
        wave_sync();
    }
}

// Stop rule of the refinement after a correction of size d (inf-norm), the
// previous one dprev (< 0 if none) and the corrected solution's size xn:
// the correction itself is below tol xn, or, converging linearly at the
// observed rate r = d / dprev < 1/2, the correction still to come is:
// r d / (1 - r) = d^2 / (dprev - d) <= tol xn.  The second test saves the
// sweep whose only purpose would be to confirm a correction far below tol.
__device__ __forceinline__ bool refined_enough(double d, double dprev, double xn, double tol) {
    if (d <= tol * xn) return true;
    return dprev > 0.0 && d <= 0.5 * dprev && d * d <= tol * xn * (dprev - d);
}

// Largest value over the wavefront of three per-lane values.
__device__ __forceinline__ void wave_max3(double &a, double &b, double &c) {
    a = wave_max(a);
    b = wave_max(b);
    c = wave_max(c);
}

// ---- mixed precision: iterative refinement, one wavefront per airfoil -------
// X holds the solution from the FP32 factors; A64 the FP64 system; A32 the
// FP32 factors and piv the pivots.  One sweep: r = b - A x in FP64 (rows held
// by lanes, the matrix streamed column by column); stop if r is at the FP64
// backward-error floor, ||r||_inf <= sqrt(n) eps ||A||_inf ||x||_inf (no
// further sweep can improve x); otherwise d = U^{-1} L^{-1} P r in FP32,
// x += d, and stop once ||d||_inf <= tol ||x||_inf.
// LDS of one wavefront's refinement.
struct WaveRefLds {
    double sx[WL * PANEL_WAVE_RMAX];
    double sr[WL * PANEL_WAVE_RMAX];
    float sd[WL * PANEL_WAVE_RMAX];
    int perm[WL * PANEL_WAVE_RMAX];
};

__device__ __forceinline__ void wave_refine(const WsView &v, int b, int32_t *__restrict__ info, double tol,
                                            int max_iter, WaveRefLds &W) {
    constexpr int RM = PANEL_WAVE_RMAX;
    constexpr int JB = 4;
    const AirfoilMeta mt = v.meta[b];
    const int n = mt.n1, ld = mt.ld;
    const int lane = wlane();
    if (info[b] != 0) {
        if (lane == 0) {
            v.iters[b] = 0;
            v.flag[b] = info[b];
        }
        return;
    }
    const double *A = v.a64 + mt.a_off;
    const float *LU = v.a32 + mt.a_off;
    const int32_t *piv = v.piv + mt.piv_off;
    double *X = v.x + mt.x_off;
    double *sx = W.sx, *sr = W.sr;
    float *sd = W.sd;
    int *perm = W.perm;
    if (lane == 0) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = 0; i < n; ++i) {
            const int p = piv[i];
            const int t0 = perm[i];
            perm[i] = perm[p];
            perm[p] = t0;
        }
    }
    const double floor_c = sqrt((double)n) * 2.220446049250313e-16;
    double anrm = -1.0;   // ||A||_inf, found during the first residual
    int worst = 0;
    bool failed = max_iter == 0;
    for (int k = 0; k < mt.K; ++k) {
        for (int i = lane; i < n; i += WL) sx[i] = X[(size_t)k * n + i];
        wave_sync();
        bool conv = false;
        int sweeps = 0;
        double dprev = -1.0;   // size of the previous correction
        for (int it = 0; it < max_iter && !conv; ++it) {
            // residual, lane owns rows lane + 64 q
            double rs[RM], ra[RM];
#pragma unroll
            for (int q = 0; q < RM; ++q) {
                const int r = min(lane + WL * q, n - 1);
                rs[q] = A[(size_t)(n + k) * ld + r];
                ra[q] = 0.0;
            }
            // JB columns per round trip: all their loads are issued before
            // the first product (left to itself the compiler placed a wait
            // after every load, one memory latency per element)
            const bool first_pass = anrm < 0.0;
            for (int j0 = 0; j0 < n; j0 += JB) {
                double a[JB][RM];
#pragma unroll
                for (int jj = 0; jj < JB; ++jj) {
                    const double *col = A + (size_t)min(j0 + jj, n - 1) * ld + lane;
#pragma unroll
                    for (int q = 0; q < RM; ++q) a[jj][q] = col[min(WL * q, n - 1 - lane)];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 0; jj < JB; ++jj) {
                    if (j0 + jj < n) {
                        const double xj = sx[j0 + jj];
#pragma unroll
                        for (int q = 0; q < RM; ++q) {
                            rs[q] -= a[jj][q] * xj;
                            if (first_pass) ra[q] += fabs(a[jj][q]);
                        }
                    }
                }
            }
            double rmax = 0.0, xmax = 0.0, rowmax = 0.0;
#pragma unroll
            for (int q = 0; q < RM; ++q) {
                const int r = lane + WL * q;
                if (r < n) {
                    sr[r] = rs[q];
                    rmax = fmax(rmax, fabs(rs[q]));
                    xmax = fmax(xmax, fabs(sx[r]));
                    rowmax = fmax(rowmax, ra[q]);
                }
            }
            wave_max3(rmax, xmax, rowmax);
            if (anrm < 0.0) anrm = rowmax;
            if (rmax <= floor_c * anrm * xmax) {
                conv = true;
                break;
            }
            wave_sync();
            for (int i = lane; i < n; i += WL) sd[i] = (float)sr[perm[i]];
            wave_sync();
            wave_trsv_lower_unit<float>(LU, ld, n, sd);
            wave_trsv_upper<float, false>(LU, ld, n, sd);
            double dmax = 0.0, xn = 0.0, unused = 0.0;
            for (int i = lane; i < n; i += WL) {
                const double d = (double)sd[i];
                const double x1 = sx[i] + d;
                sx[i] = x1;
                dmax = fmax(dmax, fabs(d));
                xn = fmax(xn, fabs(x1));
            }
            wave_max3(dmax, xn, unused);
            wave_sync();
            ++sweeps;
            conv = refined_enough(dmax, dprev, xn, tol);
            dprev = dmax;
        }
        if (!conv) failed = true;
        worst = max(worst, sweeps);
        for (int i = lane; i < n; i += WL) X[(size_t)k * n + i] = sx[i];
        wave_sync();
    }
    if (lane == 0) {
        v.iters[b] = worst;
        if (failed) info[b] = -2;
        v.flag[b] = info[b];
    }
}

}  // namespace wv
}  // namespace
}  // namespace panel
