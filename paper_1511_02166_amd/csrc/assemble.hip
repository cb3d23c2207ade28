// assemble.hip -- FP64 assembly of the bordered panel system on gfx950.
//
// Sec. 2 of the paper: constant vortex density on each straight panel, the
// fundamental solution -(1/2pi) log|x| integrated in closed form over every
// panel, boundary condition psi = C collocated at the panel midpoints, the
// Kutta condition gamma_0 + gamma_{N-1} = 0 as the last row, and the free-
// stream stream function on the right-hand side.  Sec. 3 notes that every
// entry costs logarithms and arctangents, which makes this step compute
// bound.  Here each entry is written in global coordinates with
//   d1 = m_j - P_i,  d2 = m_j - P_{i+1},  h = P_{i+1} - P_i,  L = |h|:
//   G_ji = -(1/(4 pi L)) [ (d1.h) log|d1|^2 - (d2.h) log|d2|^2 - 2 L^2
//                           + 2 (d1 x d2) atan2(d1 x d2, d1.d2) ]
// which is the closed form of the integral with the difference of the two
// arctangents folded into one (the angle subtended by the panel) and the
// logarithm of |m_j - P_{i+1}|^2 shared between panels i and i+1.  The
// self-influence is the midpoint limit (L/2pi)(1 - log(L/2)) as a function of
// the panel length alone (the shared logarithm of |m_j - P_j|^2 would carry
// the rounding of the stored midpoint, which on the shortest panels moves it
// by up to ~1e-12 relative).  log and atan2 are the library's own
// (fastmath.hpp).
//
// One workgroup covers COLS consecutive columns of one airfoil's augmented
// matrix [M | rhs] (column-major, leading dimension ld, rows n1..ld-1
// zero-filled); a thread owns one row at a time, so consecutive lanes write
// consecutive addresses of a column.
#include "fastmath.hpp"
#include "panel_internal.hpp"

namespace panel {
namespace {

constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)
constexpr double kInv2Pi = 0.15915494309189535;   // 1 / (2 pi)
constexpr int COLS = 16;

template <bool MIXED>
__global__ __launch_bounds__(256) void assemble_kernel(WsView v, const double *__restrict__ xy,
                                                       const double *__restrict__ alpha_in,
                                                       const double *__restrict__ chord_in,
                                                       double vinf) {
    const int b = blockIdx.x;
    const AirfoilMeta mt = v.meta[b];
    const int N = mt.N, n1 = mt.n1, K = mt.K, ld = mt.ld;
    const int ncols = n1 + K;
    const int c0 = blockIdx.y * COLS;
    if (c0 >= ncols) return;

    __shared__ double sx[PANEL_NMAX + 1], sy[PANEL_NMAX + 1];
    __shared__ double sca[PANEL_KMAX], ssa[PANEL_KMAX];
    __shared__ int sbad;
    const double *P = xy + 2 * (size_t)mt.node_off;
    if (threadIdx.x == 0) sbad = 0;
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        sx[k] = P[2 * k];
        sy[k] = P[2 * k + 1];
    }
    if (threadIdx.x < K) {
        const double a = alpha_in[mt.alpha_off + threadIdx.x];
        sca[threadIdx.x] = cos(a);
        ssa[threadIdx.x] = sin(a);
    }
    __syncthreads();

    if (blockIdx.y == 0) {
        // Per-airfoil side outputs: input screening, panel geometry for the
        // forces and adjoint steps, chord / angles / vinf.
        int bad = 0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const double hx = sx[i + 1] - sx[i], hy = sy[i + 1] - sy[i];
            const double L = sqrt(hx * hx + hy * hy);
            PanelGeom g;
            g.L = L;
            g.tx = hx / L;
            g.ty = hy / L;
            g.pad = 0.0;
            v.geom[mt.panel_off + i] = g;
            if (!(isfinite(sx[i]) && isfinite(sy[i]) && isfinite(sx[i + 1]) && isfinite(sy[i + 1])) ||
                (hx == 0.0 && hy == 0.0))
                bad = 1;
        }
        if (bad) atomicOr(&sbad, 1);
        if (threadIdx.x < K) v.alpha[mt.alpha_off + threadIdx.x] = alpha_in[mt.alpha_off + threadIdx.x];
        if (threadIdx.x == 0) {
            v.chord[b] = chord_in ? chord_in[b] : 1.0;
            if (b == 0) v.hdr->vinf = vinf;
        }
        __syncthreads();
        if (threadIdx.x == 0) v.flag[b] = sbad ? -1 : 0;
    }

    double *A = v.a64 + mt.a_off;
    float *A32 = MIXED ? v.a32 + mt.a_off : nullptr;
    const int cend = min(c0 + COLS, ncols);

    if (c0 + COLS <= N) {
        // Interior block: all COLS columns are panel columns.  Branch-free;
        // the diagonal value of each column is formed once here.
        __shared__ double shx[COLS], shy[COLS], sL2[COLS], siL[COLS], sdg[COLS];
        if (threadIdx.x < COLS) {
            const int c = c0 + threadIdx.x;
            const double hx = sx[c + 1] - sx[c], hy = sy[c + 1] - sy[c];
            const double L2 = hx * hx + hy * hy;
            const double L = sqrt(L2);
            shx[threadIdx.x] = hx;
            shy[threadIdx.x] = hy;
            sL2[threadIdx.x] = L2;
            siL[threadIdx.x] = 1.0 / L;
            sdg[threadIdx.x] = kInv2Pi * L * (1.0 - plog(0.5 * L));
        }
        __syncthreads();
        for (int j = threadIdx.x; j < ld; j += blockDim.x) {
            double *Aj = A + (size_t)c0 * ld + j;
            float *A32j = MIXED ? A32 + (size_t)c0 * ld + j : nullptr;
            if (j < N) {
                const double mx = 0.5 * (sx[j] + sx[j + 1]);
                const double my = 0.5 * (sy[j] + sy[j + 1]);
                double d1x = mx - sx[c0], d1y = my - sy[c0];
                double l1 = plog(d1x * d1x + d1y * d1y);
#pragma unroll 2
                for (int cc = 0; cc < COLS; ++cc) {
                    const int c = c0 + cc;
                    const double d2x = mx - sx[c + 1], d2y = my - sy[c + 1];
                    const double l2 = plog(d2x * d2x + d2y * d2y);
                    const double hx = shx[cc], hy = shy[cc], L2 = sL2[cc], iL = siL[cc];
                    const double dot1 = d1x * hx + d1y * hy;
                    const double cr = d1x * d2y - d1y * d2x;
                    const double dd = d1x * d2x + d1y * d2y;
                    const double ang = patan2(cr, dd);
                    const double gen = -kInv4Pi * iL * (dot1 * l1 - (dot1 - L2) * l2 - 2.0 * L2 + 2.0 * cr * ang);
                    const double g = (c == j) ? sdg[cc] : gen;
                    Aj[(size_t)cc * ld] = g;
                    if (MIXED) A32j[(size_t)cc * ld] = (float)g;
                    d1x = d2x;
                    d1y = d2y;
                    l1 = l2;
                }
            } else {
                for (int cc = 0; cc < COLS; ++cc) {
                    const int c = c0 + cc;
                    const double g = (j == N && (c == 0 || c == N - 1)) ? 1.0 : 0.0;
                    Aj[(size_t)cc * ld] = g;
                    if (MIXED) A32j[(size_t)cc * ld] = (float)g;
                }
            }
        }
        return;
    }

    for (int j = threadIdx.x; j < ld; j += blockDim.x) {
        double val[COLS];
        if (j < N) {
            const double mx = 0.5 * (sx[j] + sx[j + 1]);
            const double my = 0.5 * (sy[j] + sy[j + 1]);
            // node c0 (start of the first panel in this block)
            double d1x = 0.0, d1y = 0.0, l1 = 0.0;
            if (c0 < N) {
                d1x = mx - sx[c0];
                d1y = my - sy[c0];
                l1 = plog(d1x * d1x + d1y * d1y);
            }
#pragma unroll
            for (int cc = 0; cc < COLS; ++cc) {
                const int c = c0 + cc;
                double g = 0.0;
                if (c < N) {
                    const double d2x = mx - sx[c + 1], d2y = my - sy[c + 1];
                    const double l2 = plog(d2x * d2x + d2y * d2y);
                    const double hx = sx[c + 1] - sx[c], hy = sy[c + 1] - sy[c];
                    const double L2 = hx * hx + hy * hy;
                    const double L = sqrt(L2);
                    if (c == j) {
                        g = L * kInv2Pi * (1.0 - plog(0.5 * L));
                    } else {
                        const double dot1 = d1x * hx + d1y * hy;
                        const double cr = d1x * d2y - d1y * d2x;
                        const double dd = d1x * d2x + d1y * d2y;
                        const double ang = patan2(cr, dd);
                        g = -kInv4Pi / L * (dot1 * l1 - (dot1 - L2) * l2 - 2.0 * L2 + 2.0 * cr * ang);
                    }
                    d1x = d2x;
                    d1y = d2y;
                    l1 = l2;
                } else if (c == N) {
                    g = -1.0;
                } else if (c < ncols) {
                    const int k = c - n1;
                    g = -vinf * (my * sca[k] - mx * ssa[k]);
                }
                val[cc] = g;
            }
        } else if (j == N) {
#pragma unroll
            for (int cc = 0; cc < COLS; ++cc) {
                const int c = c0 + cc;
                val[cc] = (c == 0 || c == N - 1) ? 1.0 : 0.0;
            }
        } else {
#pragma unroll
            for (int cc = 0; cc < COLS; ++cc) val[cc] = 0.0;
        }
#pragma unroll
        for (int cc = 0; cc < COLS; ++cc) {
            const int c = c0 + cc;
            if (c < cend) {
                A[(size_t)c * ld + j] = val[cc];
                if (MIXED) A32[(size_t)c * ld + j] = (float)val[cc];
            }
        }
    }
}

}  // namespace

hipError_t launch_assemble(const WsView &v, int32_t B, int32_t max_cols, int32_t mixed,
                           const double *xy, const double *alpha, const double *chord, double vinf,
                           hipStream_t stream) {
    dim3 grid(B, (max_cols + COLS - 1) / COLS);
    if (mixed)
        assemble_kernel<true><<<grid, 256, 0, stream>>>(v, xy, alpha, chord, vinf);
    else
        assemble_kernel<false><<<grid, 256, 0, stream>>>(v, xy, alpha, chord, vinf);
    return hipGetLastError();
}

}  // namespace panel
