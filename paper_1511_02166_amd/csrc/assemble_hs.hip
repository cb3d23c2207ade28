// assemble_hs.hip -- the Hess-Smith (source + vortex) formulation on gfx950:
// assembly of the bordered system, its Kutta row, and the surface speed /
// Cp / Cl reductions.
//
// Unknowns: a constant source density q_i on every panel and one vortex
// density g shared by all panels.  Rows j < N hold flow tangency at the
// panel midpoints m_j, (V_inf + sum_i q_i S_i + g sum_i W_i) . n_j = 0; row N
// the Kutta condition V . t_0 + V . t_{N-1} = 0 at the two trailing-edge
// panels.  With d1 = m_j - P_i, d2 = m_j - P_{i+1}, lg = log(|d1|/|d2|) and
// beta the angle panel i subtends at m_j (pi at the panel's own midpoint),
// a unit source on panel i induces (1/2pi)(lg t_i + beta n_i) and a unit
// counter-clockwise vortex (1/2pi)(beta t_i - lg n_i), n = (t_y, -t_x).
// Projected on row j's normal and tangent, with c = t_i . t_j and
// s = t_i x t_j:
//   normal,     source: (lg s + beta c) / 2pi     vortex: (beta s - lg c) / 2pi
//   tangential, source: (lg c - beta s) / 2pi     vortex: (beta c + lg s) / 2pi
// so the vortex column of the normal matrix is minus the row sum of the
// tangential source block, and the vortex column of the tangential matrix is
// the row sum of the normal source block.  The tangential matrix T is kept
// in the workspace: the surface speed is u = T x + V_inf . t.
//
// Assembly: a thread owns one row (control point) and walks all N panels, so
// the logarithm of |m_j - P_{i+1}|^2 is shared with the next panel and both
// row sums are formed in registers (no cross-workgroup reduction); lanes
// write consecutive rows of a column.  One more block per airfoil in the same
// launch forms the Kutta row from the two trailing-edge control points
// (reading rows 0 and N-1 of T back would be two strided passes).
#include "fastmath.hpp"
#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr double kInv2Pi = 0.15915494309189535;   // 1 / (2 pi)
constexpr double kPi = 3.141592653589793;
constexpr int HS_TPB = 256;

// Kutta row, formed by its own block of the assembly launch: for each panel
// i (a thread per panel), M[N][i] = T[0][i] + T[N-1][i], the tangential
// source entries of the two trailing-edge control points evaluated as the
// row threads evaluate them; M[N][N] = sum_i (A[0][i] + A[N-1][i]) (the
// vortex columns are the row sums of A); right-hand side
// -V_inf . (t_0 + t_{N-1}).
template <bool MIXED>
__device__ void hs_kutta_row(const WsView &v, const AirfoilMeta &mt, const double *sx, const double *sy,
                             const double *stx, const double *sty, const double *sca, const double *ssa,
                             double vinf) {
    const int N = mt.N, n1 = mt.n1, K = mt.K, ld = mt.ld;
    double *A = v.a64 + mt.a_off;
    float *A32 = MIXED ? v.a32 + mt.a_off : nullptr;
    __shared__ double red[HS_TPB / 64];
    double vort = 0.0;
    for (int i = threadIdx.x; i < N; i += HS_TPB) {
        double t2 = 0.0;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int j = side == 0 ? 0 : N - 1;
            const double mx = 0.5 * (sx[j] + sx[j + 1]), my = 0.5 * (sy[j] + sy[j + 1]);
            const double d1x = mx - sx[i], d1y = my - sy[i], d2x = mx - sx[i + 1], d2y = my - sy[i + 1];
            double beta = patan2(-(d1x * d2y - d1y * d2x), d1x * d2x + d1y * d2y);
            double lg = 0.5 * (plog(d1x * d1x + d1y * d1y) - plog(d2x * d2x + d2y * d2y));
            if (i == j) {
                beta = kPi;
                lg = 0.0;
            }
            const double c = stx[i] * stx[j] + sty[i] * sty[j];
            const double s = stx[i] * sty[j] - sty[i] * stx[j];
            vort += kInv2Pi * (lg * s + beta * c);
            t2 += kInv2Pi * (lg * c - beta * s);
        }
        A[(size_t)i * ld + N] = t2;
        if (MIXED) A32[(size_t)i * ld + N] = (float)t2;
    }
    vort = wave_sum(vort);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = vort;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < HS_TPB / 64; ++w) sum += red[w];
        A[(size_t)N * ld + N] = sum;
        if (MIXED) A32[(size_t)N * ld + N] = (float)sum;
    }
    const double tx = stx[0] + stx[N - 1], ty = sty[0] + sty[N - 1];
    for (int k = threadIdx.x; k < K; k += HS_TPB) {
        const double r = -vinf * (sca[k] * tx + ssa[k] * ty);
        A[(size_t)(n1 + k) * ld + N] = r;
        if (MIXED) A32[(size_t)(n1 + k) * ld + N] = (float)r;
    }
}

template <bool MIXED>
__global__ __launch_bounds__(HS_TPB) void assemble_hs_kernel(WsView v, const double *__restrict__ xy,
                                                             const double *__restrict__ alpha_in,
                                                             const double *__restrict__ chord_in, double vinf) {
    const int b = blockIdx.x;
    const AirfoilMeta mt = v.meta[b];
    const int N = mt.N, n1 = mt.n1, K = mt.K, ld = mt.ld;
    const bool kutta = blockIdx.y == gridDim.y - 1;   // the last y-block forms the Kutta row
    const int r0 = blockIdx.y * HS_TPB;
    if (!kutta && r0 >= ld) return;

    __shared__ double sx[PANEL_NMAX + 1], sy[PANEL_NMAX + 1];
    __shared__ double stx[PANEL_NMAX], sty[PANEL_NMAX];
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
    int bad = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double hx = sx[i + 1] - sx[i], hy = sy[i + 1] - sy[i];
        const double L = sqrt(hx * hx + hy * hy);
        stx[i] = hx / L;
        sty[i] = hy / L;
        if (blockIdx.y == 0) {
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
    }
    if (bad) atomicOr(&sbad, 1);
    if (kutta) {
        __syncthreads();
        hs_kutta_row<MIXED>(v, mt, sx, sy, stx, sty, sca, ssa, vinf);
        return;
    }
    if (blockIdx.y == 0) {
        if (threadIdx.x < K) v.alpha[mt.alpha_off + threadIdx.x] = alpha_in[mt.alpha_off + threadIdx.x];
        if (threadIdx.x == 0) {
            v.chord[b] = chord_in ? chord_in[b] : 1.0;
            if (b == 0) v.hdr->vinf = vinf;
        }
    }
    __syncthreads();
    if (blockIdx.y == 0 && threadIdx.x == 0) v.flag[b] = sbad ? -1 : 0;

    double *A = v.a64 + mt.a_off;
    float *A32 = MIXED ? v.a32 + mt.a_off : nullptr;
    double *T = v.tg + mt.a_off;
    const int j = r0 + threadIdx.x;
    if (j >= ld) return;
    if (j >= N) {
        // row N (the Kutta row) comes from the Kutta block; rows past it are
        // zero padding of every column
        if (j > N) {
            for (int c = 0; c < n1 + K; ++c) {
                A[(size_t)c * ld + j] = 0.0;
                if (MIXED) A32[(size_t)c * ld + j] = 0.0f;
            }
        }
        return;
    }
    const double mx = 0.5 * (sx[j] + sx[j + 1]), my = 0.5 * (sy[j] + sy[j + 1]);
    const double tjx = stx[j], tjy = sty[j];
    double d1x = mx - sx[0], d1y = my - sy[0];
    double l1 = plog(d1x * d1x + d1y * d1y);
    double sumA = 0.0, sumT = 0.0;
    for (int i = 0; i < N; ++i) {
        const double d2x = mx - sx[i + 1], d2y = my - sy[i + 1];
        const double l2 = plog(d2x * d2x + d2y * d2y);
        const double cr = d1x * d2y - d1y * d2x, dd = d1x * d2x + d1y * d2y;
        // the panel frame (t, n) is left-handed: the subtended angle is minus
        // the global angle from d1 to d2
        double beta = patan2(-cr, dd);
        double lg = 0.5 * (l1 - l2);
        if (i == j) {
            beta = kPi;
            lg = 0.0;
        }
        const double c = stx[i] * tjx + sty[i] * tjy;
        const double s = stx[i] * tjy - sty[i] * tjx;
        const double an = kInv2Pi * (lg * s + beta * c);
        const double at = kInv2Pi * (lg * c - beta * s);
        sumA += an;
        sumT += at;
        A[(size_t)i * ld + j] = an;
        if (MIXED) A32[(size_t)i * ld + j] = (float)an;
        T[(size_t)i * ld + j] = at;
        d1x = d2x;
        d1y = d2y;
        l1 = l2;
    }
    A[(size_t)N * ld + j] = -sumT;
    if (MIXED) A32[(size_t)N * ld + j] = (float)(-sumT);
    T[(size_t)N * ld + j] = sumA;
    for (int k = 0; k < K; ++k) {
        const double r = -vinf * (sca[k] * tjy - ssa[k] * tjx);   // -V_inf . n_j
        A[(size_t)(n1 + k) * ld + j] = r;
        if (MIXED) A32[(size_t)(n1 + k) * ld + j] = (float)r;
    }
}

// Surface speed u_j = (T x)_j + V_inf . t_j for up to HS_KG angles per pass
// over T, then Cp, Cl and Cl_p as in forces.hip.  One workgroup per
// (airfoil, group of angles); a thread owns rows.
constexpr int HS_KG = 4;

__global__ __launch_bounds__(HS_TPB) void forces_hs_kernel(WsView v, double *__restrict__ gamma,
                                                           double *__restrict__ cp, double *__restrict__ cl,
                                                           double *__restrict__ cl_p) {
    const int b = blockIdx.x, k0 = blockIdx.y * HS_KG;
    const AirfoilMeta mt = v.meta[b];
    if (k0 >= mt.K) return;
    const int N = mt.N, n1 = mt.n1, ld = mt.ld;
    const int kn = min(HS_KG, mt.K - k0);
    const double vinf = v.hdr->vinf, iv = 1.0 / vinf, chord = v.chord[b];
    const double *T = v.tg + mt.a_off;
    const PanelGeom *geo = v.geom + mt.panel_off;
    __shared__ double xs[HS_KG][PANEL_NMAX + 1];
    __shared__ double ca[HS_KG], sa[HS_KG];
    __shared__ double red[2][HS_KG][HS_TPB / 64];
    for (int kk = 0; kk < kn; ++kk)
        for (int i = threadIdx.x; i < n1; i += blockDim.x) xs[kk][i] = v.x[mt.x_off + (size_t)(k0 + kk) * n1 + i];
    if (threadIdx.x < kn) {
        const double a = v.alpha[mt.alpha_off + k0 + threadIdx.x];
        ca[threadIdx.x] = cos(a);
        sa[threadIdx.x] = sin(a);
    }
    __syncthreads();
    double circ[HS_KG], fl[HS_KG];
#pragma unroll
    for (int kk = 0; kk < HS_KG; ++kk) circ[kk] = fl[kk] = 0.0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const PanelGeom g = geo[j];
        double u[HS_KG];
#pragma unroll
        for (int kk = 0; kk < HS_KG; ++kk) u[kk] = (kk < kn) ? vinf * (ca[kk] * g.tx + sa[kk] * g.ty) : 0.0;
        for (int i = 0; i < n1; ++i) {
            const double t = T[(size_t)i * ld + j];
#pragma unroll
            for (int kk = 0; kk < HS_KG; ++kk) u[kk] += t * xs[kk][i];
        }
#pragma unroll
        for (int kk = 0; kk < HS_KG; ++kk) {
            if (kk < kn) {
                const size_t o = mt.s_off + (size_t)(k0 + kk) * N + j;
                const double w = u[kk] * iv;
                const double c = 1.0 - w * w;
                if (gamma) gamma[o] = u[kk];
                if (cp) cp[o] = c;
                circ[kk] += u[kk] * g.L;
                fl[kk] += c * g.L * (g.ty * (-sa[kk]) - g.tx * ca[kk]);
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < HS_KG; ++kk) {
        const double sc = wave_sum(circ[kk]), sf = wave_sum(fl[kk]);
        if (lane == 0) {
            red[0][kk][wave] = sc;
            red[1][kk][wave] = sf;
        }
    }
    __syncthreads();
    if (threadIdx.x < kn) {
        const int kk = threadIdx.x;
        double sc = 0.0, sf = 0.0;
        for (int w = 0; w < HS_TPB / 64; ++w) {
            sc += red[0][kk][w];
            sf += red[1][kk][w];
        }
        cl[mt.alpha_off + k0 + kk] = -2.0 * sc / (vinf * chord);
        if (cl_p) cl_p[mt.alpha_off + k0 + kk] = -sf / chord;
    }
}

}  // namespace

hipError_t launch_assemble_hs(const WsView &v, int32_t B, int32_t max_ld, int32_t mixed, const double *xy,
                              const double *alpha, const double *chord, double vinf, hipStream_t stream) {
    // row blocks, then one block per airfoil for the Kutta row
    dim3 grid(B, (max_ld + HS_TPB - 1) / HS_TPB + 1);
    if (mixed)
        assemble_hs_kernel<true><<<grid, HS_TPB, 0, stream>>>(v, xy, alpha, chord, vinf);
    else
        assemble_hs_kernel<false><<<grid, HS_TPB, 0, stream>>>(v, xy, alpha, chord, vinf);
    return hipGetLastError();
}

hipError_t launch_forces_hs(const WsView &v, int32_t B, int32_t max_k, double *gamma, double *cp, double *cl,
                            double *cl_p, hipStream_t stream) {
    dim3 grid(B, (max_k + HS_KG - 1) / HS_KG);
    forces_hs_kernel<<<grid, HS_TPB, 0, stream>>>(v, gamma, cp, cl, cl_p);
    return hipGetLastError();
}

}  // namespace panel
