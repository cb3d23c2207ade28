// adjoint_wave.hip -- reverse-mode lift sensitivity, one wavefront per
// airfoil, for systems of up to 64 * PANEL_WAVE_RMAX rows.
//
// Same mathematics as adjoint.hip (the shape gradient of the Kutta-Joukowski
// lift of the Sec. 2 panel system):
//   xbar   = sum_k dcl_k x_k,   lambda = M^{-T} w,  w_i = -2 L_i / (vinf c)
//   dP     = explicit (dL/dP) + right-hand-side term - sum_{j,i} lambda_j
//            xbar_i dG_ji/dP
// with the closed-form derivatives of the panel integral G_ji(m, A, B)
// (t the unit tangent, n = (t_y, -t_x), xi = (m-A).t, eta = (m-A).n,
// l1 = log|m-A|^2, l2 = log|m-B|^2, th the angle the panel subtends at m):
//   dG/dm = -(1/2pi) [ (l1-l2)/2 t - th n ]
//   dG/dB = I/(2 pi L) + (G/L) t,
//     I = (xi (l1-l2)/2 - L - eta th) t + (-xi th - eta (l1-l2)/2) n
//   dG/dA = -dG/dm - dG/dB
// and on the diagonal dG_ii/dL = -log(L/2)/2pi.
//
// Layout of the work: one wavefront per airfoil, the lanes holding control
// points (j = lane + 64 q).  The transposed solves walk each lane's own
// column of the factors (U^T and L^T rows are U and L columns).  A single
// pass over the panels i then evaluates every pair once: the logarithm of
// |m_j - P_{i+1}|^2 is shared with the next panel, as in the assembly, and
// each pair yields both the control-point term (accumulated per lane) and
// the panel-end terms (summed over the wavefront once per panel).
#include <climits>

#include "fastmath.hpp"
#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr int WL = 64;
constexpr int RM = PANEL_WAVE_RMAX;
constexpr int NW = WL * RM;   // largest system order handled here
constexpr double kInv2Pi = 0.15915494309189535;
constexpr double kInv4Pi = 0.07957747154594767;

template <typename T> __device__ inline const T *factors_of(const WsView &v, const AirfoilMeta &mt);
template <> __device__ inline const double *factors_of<double>(const WsView &v, const AirfoilMeta &mt) {
    return v.a64 + mt.a_off;
}
template <> __device__ inline const float *factors_of<float>(const WsView &v, const AirfoilMeta &mt) {
    return v.a32 + mt.a_off;
}

// ---- U^T z = y (U upper, column-major), y in LDS, top down ------------------
// Row i of U^T is column i of U: lane i walks its own column.  64-row blocks:
// first the solved entries above the block, then the block itself with the
// solved entry of each step broadcast through a scalar register.
template <typename T, typename V>
__device__ __forceinline__ void wave_trsv_upper_t(const T *U, int ld, int n, V *y) {
    const int lane = threadIdx.x;
    for (int rb = 0; rb < n; rb += WL) {
        const int w = min(WL, n - rb);
        const bool in = lane < w;
        const int i = rb + (in ? lane : 0);
        const T *col = U + (size_t)i * ld;
        V s0 = V(0), s1 = V(0);
#pragma unroll 8
        for (int j = 0; j < rb; j += 2) {
            s0 += V(col[j]) * y[j];
            s1 += V(col[j + 1]) * y[j + 1];
        }
        T ub[WL];
#pragma unroll
        for (int jj = 0; jj < WL; ++jj) ub[jj] = col[rb + min(jj, w - 1)];
        V zi = in ? y[i] - (s0 + s1) : V(0);
        const V dinv = in ? V(1) / V(col[i]) : V(0);
#pragma unroll
        for (int jj = 0; jj < WL; ++jj) {
            if (jj < w) {
                if (lane == jj) zi *= dinv;
                const V zj = readlane_t(zi, jj);
                if (lane > jj) zi -= V(ub[jj]) * zj;
            }
        }
        if (in) y[i] = zi;
        __syncthreads();
    }
}

// ---- L^T y = z (L unit lower, column-major), y in LDS, bottom up ------------
template <typename T, typename V>
__device__ __forceinline__ void wave_trsv_lower_unit_t(const T *L, int ld, int n, V *y) {
    const int lane = threadIdx.x;
    for (int rb = ((n - 1) / WL) * WL; rb >= 0; rb -= WL) {
        const int w = min(WL, n - rb), re = rb + w;
        const bool in = lane < w;
        const int i = rb + (in ? lane : 0);
        const T *col = L + (size_t)i * ld;
        V s0 = V(0), s1 = V(0);
        int j = re;
#pragma unroll 8
        for (; j + 1 < n; j += 2) {
            s0 += V(col[j]) * y[j];
            s1 += V(col[j + 1]) * y[j + 1];
        }
        if (j < n) s0 += V(col[j]) * y[j];
        T lb[WL];
#pragma unroll
        for (int jj = 0; jj < WL; ++jj) lb[jj] = col[rb + min(jj, w - 1)];
        V yi = in ? y[i] - (s0 + s1) : V(0);
#pragma unroll
        for (int jj = WL - 1; jj >= 0; --jj) {
            if (jj < w) {
                const V yj = readlane_t(yi, jj);
                if (lane < jj) yi -= V(lb[jj]) * yj;
            }
        }
        if (in) y[i] = yi;
        __syncthreads();
    }
}

// lambda = (P^T L U)^{-T} y = P^T L^{-T} U^{-T} y with the stored factors;
// the result is scattered into out (out[perm[i]] = y[i]).
template <typename T, typename V, typename O>
__device__ __forceinline__ void wave_solve_t(const T *LU, int ld, int n, const int *perm, V *y, O *out) {
    wave_trsv_upper_t<T, V>(LU, ld, n, y);
    wave_trsv_lower_unit_t<T, V>(LU, ld, n, y);
    for (int i = threadIdx.x; i < n; i += WL) out[perm[i]] = O(y[i]);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(WL, 2) void adjoint_wave_kernel(WsView v, int32_t first,
                                                             const double *__restrict__ xy,
                                                             const double *__restrict__ dcl,
                                                             const double *__restrict__ dcp, int32_t ka,
                                                             double *__restrict__ dxy,
                                                             int32_t *__restrict__ info) {
    const int b = v.order[first + blockIdx.x];
    const AirfoilMeta mt = v.meta[b];
    const int N = mt.N, n1 = mt.n1, K = mt.K, ld = mt.ld;
    const int lane = threadIdx.x;
    double *out = dxy + 2 * (size_t)mt.node_off;
    if (ka >= K) return;   // per-angle pass past this airfoil's angles
    if (v.flag[b] != 0 || n1 > NW) {
        for (int k = lane; k < 2 * (N + 1); k += WL) out[k] = __builtin_nan("");
        if (info && lane == 0) info[b] = v.flag[b] != 0 ? v.flag[b] : -3;
        return;
    }
    __shared__ double xbar[NW], lam[NW], wv[NW], tmp[NW];
    __shared__ double ox[NW + 1], oy[NW + 1];
    __shared__ int perm[NW];
    __shared__ float yf[sizeof(T) == 4 ? NW : 1];

    const double *P = xy + 2 * (size_t)mt.node_off;
    const PanelGeom *geo = v.geom + mt.panel_off;
    const double vinf = v.hdr->vinf, chord = v.chord[b];
    const double *X = v.x + mt.x_off;
    const double wscale = -2.0 / (vinf * chord);
    // Cotangent seeds.  All angles at once (ka < 0, cl cotangents only): the
    // seed w = dCl/dx is the same for every angle, so one transposed solve
    // serves them all with xbar = sum_k dcl_k x_k and the right-hand-side
    // weights S, Cc summed likewise.  One angle (ka >= 0): the seed also
    // carries dcp_i dCp_i/dgamma_i = -2 dcp_i gamma_i / vinf^2, so lambda is
    // that angle's own; xbar = x_ka, and the explicit length term keeps the
    // factor dcl_ka (escale).
    double S = 0.0, Cc = 0.0, escale = 1.0;
    if (ka < 0) {
        for (int k = 0; k < K; ++k) {
            const double a = v.alpha[mt.alpha_off + k], d = dcl[mt.alpha_off + k];
            S += d * sin(a);
            Cc += d * cos(a);
        }
    } else {
        const double a = v.alpha[mt.alpha_off + ka];
        S = sin(a);
        Cc = cos(a);
        escale = dcl[mt.alpha_off + ka];
    }
    const double *cpbar = (ka >= 0 && dcp) ? dcp + mt.s_off + (size_t)ka * N : nullptr;
    const double cpf = -2.0 / (vinf * vinf);
    for (int i = lane; i < n1; i += WL) {
        double s = 0.0;
        if (ka < 0) {
            for (int k = 0; k < K; ++k) s += dcl[mt.alpha_off + k] * X[(size_t)k * n1 + i];
        } else {
            s = X[(size_t)ka * n1 + i];
        }
        xbar[i] = s;
        double w = (i < N) ? escale * wscale * geo[i].L : 0.0;
        if (cpbar && i < N) w += cpbar[i] * cpf * s;
        wv[i] = w;
        ox[i] = 0.0;
        oy[i] = 0.0;
    }
    if (lane == 0) {
        const int32_t *piv = v.piv + mt.piv_off;
        for (int i = 0; i < n1; ++i) perm[i] = i;
        for (int i = 0; i < n1; ++i) {
            const int p = piv[i];
            const int t0 = perm[i];
            perm[i] = perm[p];
            perm[p] = t0;
        }
    }
    __syncthreads();

    // ---- lambda = M^{-T} w -------------------------------------------------
    const T *LU = factors_of<T>(v, mt);
    bool conv = true;
    if constexpr (sizeof(T) == 8) {
        for (int i = lane; i < n1; i += WL) tmp[i] = wv[i];
        __syncthreads();
        wave_solve_t<double, double, double>(LU, ld, n1, perm, tmp, lam);
    } else {
        // FP32 factors: lambda from U^T/L^T in FP32, then FP64 refinement of
        // the transposed system against the FP64 matrix in A64.
        const double *A = v.a64 + mt.a_off;
        for (int i = lane; i < n1; i += WL) yf[i] = (float)wv[i];
        __syncthreads();
        wave_solve_t<float, float, double>(LU, ld, n1, perm, yf, lam);
        const double floor_c = sqrt((double)n1) * 2.220446049250313e-16;
        double anrm = -1.0;
        conv = false;
        for (int it = 0; it < 10; ++it) {
            // r = w - A^T lambda: lane i walks column i of A
            double rmax = 0.0, lmax = 0.0, cmax = 0.0;
            for (int i = lane; i < n1; i += WL) {
                const double *col = A + (size_t)i * ld;
                double s0 = wv[i], s1 = 0.0, ca = 0.0;
                int j = 0;
                if (anrm < 0.0) {
                    for (; j < n1; ++j) {
                        s0 -= col[j] * lam[j];
                        ca += fabs(col[j]);
                    }
                } else {
#pragma unroll 8
                    for (; j + 1 < n1; j += 2) {
                        s0 -= col[j] * lam[j];
                        s1 -= col[j + 1] * lam[j + 1];
                    }
                    if (j < n1) s0 -= col[j] * lam[j];
                }
                const double s = s0 + s1;
                yf[i] = (float)s;
                rmax = fmax(rmax, fabs(s));
                lmax = fmax(lmax, fabs(lam[i]));
                cmax = fmax(cmax, ca);
            }
            rmax = wave_max(rmax);
            lmax = wave_max(lmax);
            cmax = wave_max(cmax);
            if (anrm < 0.0) anrm = cmax;   // ||A^T||_inf = largest column sum
            __syncthreads();
            if (rmax <= floor_c * anrm * lmax) {
                conv = true;
                break;
            }
            wave_solve_t<float, float, double>(LU, ld, n1, perm, yf, tmp);
            double dmax = 0.0, ln = 0.0;
            for (int i = lane; i < n1; i += WL) {
                const double d = tmp[i];
                const double l = lam[i] + d;
                lam[i] = l;
                dmax = fmax(dmax, fabs(d));
                ln = fmax(ln, fabs(l));
            }
            dmax = wave_max(dmax);
            ln = wave_max(ln);
            __syncthreads();
            if (dmax <= 1e-12 * ln) {
                conv = true;
                break;
            }
        }
    }
    // info: 0, or -2 when the FP64 refinement of lambda ran out of sweeps
    // (a later per-angle pass never clears an earlier failure)
    if (info && lane == 0) {
        if (!conv) info[b] = -2;
        else if (ka <= 0) info[b] = 0;
    }

    // ---- one pass over the panels ----------------------------------------
    // slot q: control point j = lane + 64 q (clamped to N-1 with a zero
    // weight when past the last one)
    double mx[RM], my[RM], lj[RM], d1x[RM], d1y[RM], l1[RM], ax[RM], ay[RM];
    int jq[RM];
#pragma unroll
    for (int q = 0; q < RM; ++q) {
        const int j = lane + WL * q;
        jq[q] = j < N ? j : -1;
        const int jc = min(j, N - 1);
        mx[q] = 0.5 * (P[2 * jc] + P[2 * jc + 2]);
        my[q] = 0.5 * (P[2 * jc + 1] + P[2 * jc + 3]);
        lj[q] = j < N ? lam[j] : 0.0;
        d1x[q] = mx[q] - P[0];
        d1y[q] = my[q] - P[1];
        l1[q] = plog(d1x[q] * d1x[q] + d1y[q] * d1y[q]);
        ax[q] = 0.0;
        ay[q] = 0.0;
    }
    double Ax = P[0], Ay = P[1];
    for (int i = 0; i < N; ++i) {
        const double Bx = P[2 * i + 2], By = P[2 * i + 3];
        const double hx = Bx - Ax, hy = By - Ay;
        const PanelGeom g = geo[i];
        const double L = g.L, iL = 1.0 / L, tx = g.tx, ty = g.ty, nx = ty, ny = -tx;
        const double xb = xbar[i];
        const double dGdL = -kInv2Pi * plog(0.5 * L);   // diagonal: dG_ii/dL
        double pbx = 0.0, pby = 0.0, psx = 0.0, psy = 0.0;
#pragma unroll
        for (int q = 0; q < RM; ++q) {
            if (q * WL >= N) break;   // slots past the last control point (uniform)
            const double e2x = mx[q] - Bx, e2y = my[q] - By;
            const double l2 = plog(e2x * e2x + e2y * e2y);
            const double cr = d1x[q] * e2y - d1y[q] * e2x;
            const double th = patan2(cr, d1x[q] * e2x + d1y[q] * e2y);
            const double hl = 0.5 * (l1[q] - l2);
            const double xi = d1x[q] * tx + d1y[q] * ty, eta = d1x[q] * nx + d1y[q] * ny;
            const double G = -kInv4Pi * iL *
                             ((d1x[q] * hx + d1y[q] * hy) * l1[q] - (e2x * hx + e2y * hy) * l2 - 2.0 * L * L +
                              2.0 * cr * th);
            const double fx = hl * tx - th * nx, fy = hl * ty - th * ny;   // -2pi dG/dm
            const double itt = xi * hl - L - eta * th, inn = -xi * th - eta * hl;
            const double bgx = kInv2Pi * iL * (itt * tx + inn * nx) + G * iL * tx;
            const double bgy = kInv2Pi * iL * (itt * ty + inn * ny) + G * iL * ty;
            // the diagonal (j == i): G_ii depends on the panel length only,
            // dG/dB = dG/dL t, no control-point term
            const bool dg = jq[q] == i;
            const double lq = lj[q];
            pbx += lq * (dg ? dGdL * tx : bgx);
            pby += lq * (dg ? dGdL * ty : bgy);
            psx += dg ? 0.0 : lq * (-kInv2Pi * fx);
            psy += dg ? 0.0 : lq * (-kInv2Pi * fy);
            ax[q] += dg ? 0.0 : xb * fx;
            ay[q] += dg ? 0.0 : xb * fy;
            d1x[q] = e2x;
            d1y[q] = e2y;
            l1[q] = l2;
        }
        pbx = wave_sum(pbx);
        pby = wave_sum(pby);
        psx = wave_sum(psx);
        psy = wave_sum(psy);
        // panel i from node i to node i + 1: dA = -dm - dB off the diagonal
        // (the diagonal contributed to dB only, and dA = -dB for it)
        if (lane == 0) {
            ox[i] += xb * (psx + pbx);
            oy[i] += xb * (psy + pby);
            ox[i + 1] -= xb * pbx;
            oy[i + 1] -= xb * pby;
        }
        Ax = Bx;
        Ay = By;
    }
    __syncthreads();

    // ---- explicit and right-hand-side terms, control-point terms -----------
    // control point j sits on panel j (nodes j and j + 1): each node gets
    // half of its m-derivative terms; the explicit dL/dP term moves the
    // panel's end nodes along the tangent.
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int q = 0; q < RM; ++q) {
            const int j = jq[q];
            if (j >= 0) {
                const PanelGeom g = geo[j];
                const double e = escale * wscale * xbar[j];
                const double gmx = -kInv2Pi * lj[q] * ax[q], gmy = -kInv2Pi * lj[q] * ay[q];
                const double cx = 0.5 * (lj[q] * vinf * S - gmx), cy = 0.5 * (-lj[q] * vinf * Cc - gmy);
                if (half == 0) {   // node j: start of panel j
                    ox[j] += -e * g.tx + cx;
                    oy[j] += -e * g.ty + cy;
                } else {           // node j + 1: end of panel j
                    ox[j + 1] += e * g.tx + cx;
                    oy[j + 1] += e * g.ty + cy;
                }
            }
        }
        __syncthreads();
    }
    // the first pass writes, later per-angle passes add their share
    for (int k = lane; k <= N; k += WL) {
        if (ka <= 0) {
            out[2 * k] = ox[k];
            out[2 * k + 1] = oy[k];
        } else {
            out[2 * k] += ox[k];
            out[2 * k + 1] += oy[k];
        }
    }
}

}  // namespace

hipError_t launch_adjoint_wave(const WsView &v, int32_t first, int32_t count, int32_t mixed, const double *xy,
                               const double *dcl, const double *dcp, int32_t ka, double *dxy, int32_t *info,
                               hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    if (mixed)
        adjoint_wave_kernel<float><<<count, WL, 0, stream>>>(v, first, xy, dcl, dcp, ka, dxy, info);
    else
        adjoint_wave_kernel<double><<<count, WL, 0, stream>>>(v, first, xy, dcl, dcp, ka, dxy, info);
    return hipGetLastError();
}

}  // namespace panel
