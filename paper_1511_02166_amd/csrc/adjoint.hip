// adjoint.hip -- reverse-mode sensitivity of the lift to the node coordinates
// on gfx950 (the paper optimises airfoil shapes, Sec. 2; this gives the
// shape gradient of the Kutta-Joukowski lift of its panel system).
//
// For one airfoil with solutions x_k of M x_k = r_k (angles k < K) and lift
// Cl_k = -2 sum_i x_k,i L_i / (vinf c), the cotangents dcl_k give
//   xbar   = sum_k dcl_k x_k
//   lambda = M^{-T} w,   w_i = -2 L_i / (vinf c) (i < N),  w_N = 0
//   dP     = -2/(vinf c) sum_i xbar_i dL_i/dP                 (explicit)
//          + sum_j lambda_j sum_k dcl_k dr_k,j/dP              (right-hand side)
//          - sum_{j,i} lambda_j xbar_i dG_ji/dP                (matrix)
// One transposed solve serves all K angles.  It reuses the factors left by
// the forward solve (FP64, or FP32 factors with FP64 refinement of the
// transposed system).  The matrix term re-evaluates closed-form derivatives
// of the panel integral G_ji(m, A, B) (control point m = m_j, panel i from A
// to B, unit tangent t, normal n = (t_y, -t_x), xi = (m-A).t, eta = (m-A).n,
// l1 = log|m-A|^2, l2 = log|m-B|^2, th = angle subtended by the panel):
//   dG/dm = -(1/2pi) [ (l1-l2)/2 t - th n ]
//   dG/dB = I/(2 pi L) + (G/L) t,
//     I = (xi (l1-l2)/2 - L - eta th) t + (-xi th - eta (l1-l2)/2) n
//   dG/dA = -dG/dm - dG/dB                  (translation invariance)
// and, on the diagonal, G_ii = (L/2pi)(1 - log(L/2)), dG_ii/dL = -log(L/2)/2pi.
// Pass 1 (one thread per control point) sums the m-derivatives, pass 2 (one
// thread per panel) the endpoint derivatives; no cross-thread reductions.
#include <climits>

#include "fastmath.hpp"
#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr int TPB = 256;
constexpr int SB = 64;
constexpr double kInv2Pi = 0.15915494309189535;
constexpr double kInv4Pi = 0.07957747154594767;

template <typename T> __device__ inline const T *factors(const WsView &v, const AirfoilMeta &mt);
template <> __device__ inline const double *factors<double>(const WsView &v, const AirfoilMeta &mt) {
    return v.a64 + mt.a_off;
}
template <> __device__ inline const float *factors<float>(const WsView &v, const AirfoilMeta &mt) {
    return v.a32 + mt.a_off;
}

// Solve U^T z = y in place (U upper, column-major); y in LDS, V accumulation type.
template <typename T, typename V>
__device__ void trsv_upper_t(const T *U, int ld, int n, V *y, T *sblk, V *part) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + SB - 1) / SB;
    for (int blk = 0; blk < nblk; ++blk) {
        const int rb = blk * SB, w = min(SB, n - rb);
        // y_i -= sum_{j < rb} U[j][i] y_j for the block's rows: four partial
        // sums per row (one per wavefront), each over a quarter of j
        {
            const int i = rb + lane;
            V s = V(0);
            if (lane < w) {
                const T *col = U + (size_t)i * ld;
                for (int j = wave; j < rb; j += TPB / 64) s += V(col[j]) * y[j];
            }
            part[wave * SB + lane] = s;
        }
        for (int idx = tid; idx < SB * SB; idx += TPB) {
            const int c = idx >> 6, r = idx & 63;
            sblk[idx] = (c < w && r <= c) ? U[(size_t)(rb + c) * ld + rb + r] : T(0);
        }
        __syncthreads();
        if (wave == 0) {
            V yi = V(0), dinv = V(0);
            if (lane < w) {
                yi = y[rb + lane] - ((part[lane] + part[SB + lane]) + (part[2 * SB + lane] + part[3 * SB + lane]));
                dinv = V(1) / V(sblk[lane * SB + lane]);
            }
            for (int j = 0; j < w; ++j) {
                if (lane == j) yi *= dinv;
                const V zj = readlane_t(yi, j);
                if (lane > j && lane < w) yi -= V(sblk[lane * SB + j]) * zj;
            }
            if (lane < w) y[rb + lane] = yi;
        }
        __syncthreads();
    }
}

// Solve L^T y = z in place (L unit lower, column-major); y in LDS.
template <typename T, typename V>
__device__ void trsv_lower_unit_t(const T *L, int ld, int n, V *y, T *sblk, V *part) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + SB - 1) / SB;
    for (int blk = nblk - 1; blk >= 0; --blk) {
        const int rb = blk * SB, w = min(SB, n - rb), re = rb + w;
        {
            const int i = rb + lane;
            V s = V(0);
            if (lane < w) {
                const T *col = L + (size_t)i * ld;
                for (int j = re + wave; j < n; j += TPB / 64) s += V(col[j]) * y[j];
            }
            part[wave * SB + lane] = s;
        }
        for (int idx = tid; idx < SB * SB; idx += TPB) {
            const int c = idx >> 6, r = idx & 63;
            sblk[idx] = (c < w && r < w && r > c) ? L[(size_t)(rb + c) * ld + rb + r] : T(0);
        }
        __syncthreads();
        if (wave == 0) {
            V yi = V(0);
            if (lane < w)
                yi = y[rb + lane] - ((part[lane] + part[SB + lane]) + (part[2 * SB + lane] + part[3 * SB + lane]));
            for (int j = w - 1; j >= 0; --j) {
                const V yj = readlane_t(yi, j);
                if (lane < j) yi -= V(sblk[lane * SB + j]) * yj;
            }
            if (lane < w) y[rb + lane] = yi;
        }
        __syncthreads();
    }
}

// lambda = (P^T L U)^{-T} w = P^T L^{-T} U^{-T} w with the stored factors.
template <typename T, typename V>
__device__ void solve_transposed(const T *LU, int ld, int n, const int *perm, V *y, V *tmp, T *sblk,
                                 V *part) {
    trsv_upper_t<T, V>(LU, ld, n, y, sblk, part);
    trsv_lower_unit_t<T, V>(LU, ld, n, y, sblk, part);
    // undo the row permutation: (P^T y)[perm[i]] = y[i]
    for (int i = threadIdx.x; i < n; i += TPB) tmp[perm[i]] = y[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += TPB) y[i] = tmp[i];
    __syncthreads();
}

// lambda = M^{-T} w for airfoil mt: w in tmp on entry, lambda in lam on exit
// (tmp clobbered).  FP64 factors: one transposed solve.  FP32 factors:
// lambda from U^T/L^T in FP32, then FP64 refinement of the transposed system
// against the FP64 matrix kept in A64.  Returns false when the refinement ran
// out of sweeps.
template <typename T>
__device__ bool solve_lambda(const WsView &v, const AirfoilMeta &mt, const int *perm, double *lam, double *tmp,
                             T *sblk, double *part, double (*red)[TPB / 64]) {
    const int n1 = mt.n1, ld = mt.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T *LU = factors<T>(v, mt);
    bool conv = true;
    if constexpr (sizeof(T) == 8) {
        for (int i = tid; i < n1; i += TPB) lam[i] = tmp[i];
        __syncthreads();
        solve_transposed<double, double>(LU, ld, n1, perm, lam, tmp, sblk, part);
    } else {
        // FP32 factors: lambda from U^T/L^T in FP32, then FP64 refinement of
        // the transposed system against the FP64 matrix in A64.
        const double *A = v.a64 + mt.a_off;
        __shared__ double wv[PANEL_NMAX + 1];
        __shared__ float ylo[PANEL_NMAX + 1], tlo[PANEL_NMAX + 1];
        __shared__ float partf[(TPB / 64) * SB];
        for (int i = tid; i < n1; i += TPB) {
            wv[i] = tmp[i];
            ylo[i] = (float)tmp[i];
        }
        __syncthreads();
        solve_transposed<float, float>(LU, ld, n1, perm, ylo, tlo, sblk, partf);
        for (int i = tid; i < n1; i += TPB) lam[i] = (double)ylo[i];
        __syncthreads();
        const double floor_c = sqrt((double)n1) * 2.220446049250313e-16;
        double anrm = -1.0;
        conv = false;
        for (int it = 0; it < 10; ++it) {
            // r = w - A^T lambda  (column i of A dotted with lambda)
            double rmax = 0.0, lmax = 0.0, cmax = 0.0;
            for (int i = tid; i < n1; i += TPB) {
                const double *col = A + (size_t)i * ld;
                double s = wv[i], ca = 0.0;
                for (int j = 0; j < n1; ++j) {
                    s -= col[j] * lam[j];
                    ca += fabs(col[j]);
                }
                tmp[i] = s;
                rmax = fmax(rmax, fabs(s));
                lmax = fmax(lmax, fabs(lam[i]));
                cmax = fmax(cmax, ca);
            }
            rmax = wave_max(rmax);
            lmax = wave_max(lmax);
            cmax = wave_max(cmax);
            if (lane == 0) {
                red[0][wave] = rmax;
                red[1][wave] = lmax;
                part[wave] = cmax;
            }
            __syncthreads();
            rmax = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
            lmax = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
            if (anrm < 0.0) anrm = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
            __syncthreads();
            if (rmax <= floor_c * anrm * lmax) {   // ||A^T||_inf = max column sum
                conv = true;
                break;
            }
            for (int i = tid; i < n1; i += TPB) ylo[i] = (float)tmp[i];
            __syncthreads();
            solve_transposed<float, float>(LU, ld, n1, perm, ylo, tlo, sblk, partf);
            double dmax = 0.0, ln = 0.0;
            for (int i = tid; i < n1; i += TPB) {
                const double d = (double)ylo[i];
                lam[i] += d;
                dmax = fmax(dmax, fabs(d));
                ln = fmax(ln, fabs(lam[i]));
            }
            dmax = wave_max(dmax);
            ln = wave_max(ln);
            if (lane == 0) {
                red[0][wave] = dmax;
                red[1][wave] = ln;
            }
            __syncthreads();
            dmax = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
            ln = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
            __syncthreads();
            if (dmax <= 1e-12 * ln) {
                conv = true;
                break;
            }
        }
    }
    return conv;
}

template <typename T>
__global__ __launch_bounds__(TPB) void adjoint_kernel(WsView v, const double *__restrict__ xy,
                                                      const double *__restrict__ dcl,
                                                      const double *__restrict__ dcp, int32_t ka,
                                                      double *__restrict__ dxy, int32_t *__restrict__ info) {
    const int b = v.order[blockIdx.x];
    const AirfoilMeta mt = v.meta[b];
    const int N = mt.N, n1 = mt.n1, K = mt.K;
    const int tid = threadIdx.x;
    double *out = dxy + 2 * (size_t)mt.node_off;
    if (ka >= K) return;   // per-angle pass past this airfoil's angles
    if (v.flag[b] != 0) {
        for (int k = tid; k < 2 * (N + 1); k += TPB) out[k] = __builtin_nan("");
        if (info && tid == 0) info[b] = v.flag[b];
        return;
    }
    __shared__ double sx[PANEL_NMAX + 1], sy[PANEL_NMAX + 1];
    __shared__ double xbar[PANEL_NMAX + 1], lam[PANEL_NMAX + 1];
    __shared__ double tmp[PANEL_NMAX + 1];
    __shared__ double gmx[PANEL_NMAX], gmy[PANEL_NMAX];
    __shared__ int perm[PANEL_NMAX + 1];
    __shared__ T sblk[SB * SB];
    __shared__ double part[(TPB / 64) * SB];
    __shared__ double red[2][TPB / 64];

    const double *P = xy + 2 * (size_t)mt.node_off;
    for (int k = tid; k <= N; k += TPB) {
        sx[k] = P[2 * k];
        sy[k] = P[2 * k + 1];
    }
    const double vinf = v.hdr->vinf, chord = v.chord[b];
    const double *X = v.x + mt.x_off;
    // Cotangent seeds: all angles at once with cl cotangents only (ka < 0,
    // one transposed solve; xbar = sum_k dcl_k x_k), or one angle with its
    // cl and cp cotangents (ka >= 0; xbar = x_ka, the explicit length term
    // scaled by dcl_ka).
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
    for (int i = tid; i < n1; i += TPB) {
        double s = 0.0;
        if (ka < 0) {
            for (int k = 0; k < K; ++k) s += dcl[mt.alpha_off + k] * X[(size_t)k * n1 + i];
        } else {
            s = X[(size_t)ka * n1 + i];
        }
        xbar[i] = s;
    }
    if (tid == 0) {
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
    const double wscale = -2.0 / (vinf * chord);
    for (int i = tid; i < n1; i += TPB) {
        double w = 0.0;
        if (i < N) {
            const double hx = sx[i + 1] - sx[i], hy = sy[i + 1] - sy[i];
            w = escale * wscale * sqrt(hx * hx + hy * hy);
            if (cpbar) w += cpbar[i] * cpf * xbar[i];
        }
        tmp[i] = w;
    }
    __syncthreads();

    const bool conv = solve_lambda<T>(v, mt, perm, lam, tmp, sblk, part, red);
    // info: 0, or -2 when the FP64 refinement of lambda ran out of sweeps
    // (a later per-angle pass never clears an earlier failure)
    if (info && tid == 0) {
        if (!conv) info[b] = -2;
        else if (ka <= 0) info[b] = 0;
    }

    // ---- pass 1: control points (dG/dm), one thread per row j -------------
    for (int j = tid; j < N; j += TPB) {
        const double mx = 0.5 * (sx[j] + sx[j + 1]), my = 0.5 * (sy[j] + sy[j + 1]);
        double ax = 0.0, ay = 0.0;
        double d1x = mx - sx[0], d1y = my - sy[0];
        double l1 = plog(d1x * d1x + d1y * d1y);
        for (int i = 0; i < N; ++i) {
            const double d2x = mx - sx[i + 1], d2y = my - sy[i + 1];
            const double l2 = plog(d2x * d2x + d2y * d2y);
            if (i != j) {
                const double hx = sx[i + 1] - sx[i], hy = sy[i + 1] - sy[i];
                const double iL = 1.0 / sqrt(hx * hx + hy * hy);
                const double tx = hx * iL, ty = hy * iL;
                const double cr = d1x * d2y - d1y * d2x;
                const double th = patan2(cr, d1x * d2x + d1y * d2y);
                const double hl = 0.5 * (l1 - l2);
                const double xb = xbar[i];
                // (l1-l2)/2 t - th n, n = (ty, -tx)
                ax += xb * (hl * tx - th * ty);
                ay += xb * (hl * ty + th * tx);
            }
            d1x = d2x;
            d1y = d2y;
            l1 = l2;
        }
        const double c = -kInv2Pi * lam[j];
        gmx[j] = c * ax;
        gmy[j] = c * ay;
    }
    __syncthreads();

    // ---- pass 2: panels (dG/dA, dG/dB), one thread per panel i ------------
    double *gBx = tmp;   // tmp is free once lambda is known
    __shared__ double gBy[PANEL_NMAX], gAx[PANEL_NMAX], gAy[PANEL_NMAX];
    for (int i = tid; i < N; i += TPB) {
        const double Ax = sx[i], Ay = sy[i], Bx = sx[i + 1], By = sy[i + 1];
        const double hx = Bx - Ax, hy = By - Ay;
        const double L = sqrt(hx * hx + hy * hy), iL = 1.0 / L;
        const double tx = hx * iL, ty = hy * iL, nx = ty, ny = -tx;
        double bx = 0.0, by = 0.0, sx_ = 0.0, sy_ = 0.0;   // sum lambda dG/dB, sum lambda dG/dm
        for (int j = 0; j < N; ++j) {
            const double cj = lam[j];
            if (j == i) {
                // diagonal: G_ii depends on the panel length only, so
                // dG_ii/dB = dG_ii/dL t and dG_ii/dA = -dG_ii/dL t (no m term)
                const double dGdL = -kInv2Pi * plog(0.5 * L);
                bx += cj * dGdL * tx;
                by += cj * dGdL * ty;
                continue;
            }
            const double mx = 0.5 * (sx[j] + sx[j + 1]), my = 0.5 * (sy[j] + sy[j + 1]);
            const double d1x = mx - Ax, d1y = my - Ay, d2x = mx - Bx, d2y = my - By;
            const double l1 = plog(d1x * d1x + d1y * d1y), l2 = plog(d2x * d2x + d2y * d2y);
            const double cr = d1x * d2y - d1y * d2x;
            const double th = patan2(cr, d1x * d2x + d1y * d2y);
            const double hl = 0.5 * (l1 - l2);
            const double xi = d1x * tx + d1y * ty, eta = d1x * nx + d1y * ny;
            const double G = -kInv4Pi * iL * ((d1x * hx + d1y * hy) * l1 - (d2x * hx + d2y * hy) * l2 -
                                              2.0 * L * L + 2.0 * cr * th);
            // dG/dm
            const double mxg = -kInv2Pi * (hl * tx - th * nx), myg = -kInv2Pi * (hl * ty - th * ny);
            // dG/dB
            const double it = xi * hl - L - eta * th, in = -xi * th - eta * hl;
            const double bgx = kInv2Pi * iL * (it * tx + in * nx) + G * iL * tx;
            const double bgy = kInv2Pi * iL * (it * ty + in * ny) + G * iL * ty;
            bx += cj * bgx;
            by += cj * bgy;
            sx_ += cj * mxg;
            sy_ += cj * myg;
        }
        const double xb = xbar[i];
        // dG/dA = -dG/dm - dG/dB off the diagonal; on the diagonal dA = -dB.
        gBx[i] = xb * bx;   // (tmp holds gBx from here on)
        gBy[i] = xb * by;
        gAx[i] = -xb * (sx_ + bx);
        gAy[i] = -xb * (sy_ + by);
    }
    __syncthreads();

    // ---- node gradients --------------------------------------------------------
    for (int k = tid; k <= N; k += TPB) {
        double gx = 0.0, gy = 0.0;
        if (k >= 1) {   // panel k-1 ends at node k; control point k-1
            const int i = k - 1;
            const double hx = sx[i + 1] - sx[i], hy = sy[i + 1] - sy[i];
            const double iL = 1.0 / sqrt(hx * hx + hy * hy);
            const double e = escale * wscale * xbar[i];
            gx += e * hx * iL - gBx[i];
            gy += e * hy * iL - gBy[i];
            gx += 0.5 * (lam[i] * vinf * S - gmx[i]);
            gy += 0.5 * (-lam[i] * vinf * Cc - gmy[i]);
        }
        if (k < N) {    // panel k starts at node k; control point k
            const int i = k;
            const double hx = sx[i + 1] - sx[i], hy = sy[i + 1] - sy[i];
            const double iL = 1.0 / sqrt(hx * hx + hy * hy);
            const double e = escale * wscale * xbar[i];
            gx += -e * hx * iL - gAx[i];
            gy += -e * hy * iL - gAy[i];
            gx += 0.5 * (lam[i] * vinf * S - gmx[i]);
            gy += 0.5 * (-lam[i] * vinf * Cc - gmy[i]);
        }
        if (ka <= 0) {   // the first pass writes, later per-angle passes add
            out[2 * k] = gx;
            out[2 * k + 1] = gy;
        } else {
            out[2 * k] += gx;
            out[2 * k + 1] += gy;
        }
    }
}

// ---- Hess-Smith formulation ------------------------------------------------
// Unknowns x = (q_0..q_{N-1}, g): source densities and the shared vortex
// density; surface speed u = T x + V_inf e.t (T: the tangential matrix kept
// by the assembly), Cl = -2 sum_j u_j L_j / (V_inf c), Cp_j = 1 - u_j^2/V_inf^2.
// For each angle, with g_j = dF/du_j, w = T^T g and lambda = M^{-T} w, the
// source-block entries A_ji (normal) and T_ji (tangential), i != j, carry the
// weights
//   W_A(j,i) = g_j x_N - lambda_j x_i - k_j lambda_N x_N
//   W_T(j,i) = g_j x_i + lambda_j x_N - k_j lambda_N x_i
// (k_j = 1 on the two trailing-edge rows that form the Kutta row; the
// vortex columns are row sums of the source blocks, so their derivatives
// fold into these weights).  A and T depend on d1 = m_j - P_i, d2 = m_j -
// P_{i+1} through lg = log(|d1|/|d2|) and the subtended angle beta, and on
// the panel angles through c = t_i.t_j = cos(phi_j - phi_i), s = t_i x t_j:
//   d/dd1 (W_A A + W_T T) = (a d1 + b perp(d1)) / (2 pi |d1|^2)
//   d/dd2 (W_A A + W_T T) = -(a d2 + b perp(d2)) / (2 pi |d2|^2)
//   d/dphi_j = -d/dphi_i  = (lg b - beta a) / 2pi
// with a = W_A s + W_T c, b = W_A c - W_T s, perp(v) = (-v_y, v_x).  The
// right-hand sides (-V_inf e.n_j, and -V_inf e.(t_0 + t_{N-1}) on the Kutta
// row), the free-stream part of u and the panel lengths in Cl add explicit
// terms.  Self entries (A_jj = 1/2, T_jj = 0) are constants.
// One workgroup per airfoil loops over its angles.  Pass 1 (a thread per
// row j, walking the panels) sums the control-point and row-angle terms;
// pass 2 (a thread per node k, walking the rows) sums the endpoint terms of
// the panels starting and ending at node k and the column-angle term of
// panel k.  All sums have a single owner thread; gradients w.r.t. the
// midpoints (gm) and the panel vectors (gh = dF/dphi perp(t)/L + length
// terms) reach the nodes at the end.
template <typename T>
__global__ __launch_bounds__(TPB) void adjoint_hs_kernel(WsView v, const double *__restrict__ xy,
                                                         const double *__restrict__ dcl,
                                                         const double *__restrict__ dcp,
                                                         double *__restrict__ dxy, int32_t *__restrict__ info) {
    const int b = v.order[blockIdx.x];
    const AirfoilMeta mt = v.meta[b];
    const int N = mt.N, n1 = mt.n1, K = mt.K, ld = mt.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *out = dxy + 2 * (size_t)mt.node_off;
    if (v.flag[b] != 0) {
        for (int k = tid; k < 2 * (N + 1); k += TPB) out[k] = __builtin_nan("");
        if (info && tid == 0) info[b] = v.flag[b];
        return;
    }
    __shared__ double sx[PANEL_NMAX + 1], sy[PANEL_NMAX + 1];
    __shared__ double xk[PANEL_NMAX + 1], lam[PANEL_NMAX + 1], gu[PANEL_NMAX + 1];
    __shared__ double tmp[PANEL_NMAX + 1];
    __shared__ double gmx[PANEL_NMAX], gmy[PANEL_NMAX], ghx[PANEL_NMAX], ghy[PANEL_NMAX];
    __shared__ double gnx[PANEL_NMAX + 1], gny[PANEL_NMAX + 1];
    __shared__ int perm[PANEL_NMAX + 1];
    __shared__ T sblk[SB * SB];
    __shared__ double part[(TPB / 64) * SB];
    __shared__ double red[2][TPB / 64];

    const double *P = xy + 2 * (size_t)mt.node_off;
    for (int k = tid; k <= N; k += TPB) {
        sx[k] = P[2 * k];
        sy[k] = P[2 * k + 1];
        gnx[k] = gny[k] = 0.0;
    }
    for (int j = tid; j < N; j += TPB) gmx[j] = gmy[j] = ghx[j] = ghy[j] = 0.0;
    if (tid == 0) {
        const int32_t *piv = v.piv + mt.piv_off;
        for (int i = 0; i < n1; ++i) perm[i] = i;
        for (int i = 0; i < n1; ++i) {
            const int p = piv[i];
            const int t0 = perm[i];
            perm[i] = perm[p];
            perm[p] = t0;
        }
    }
    const double vinf = v.hdr->vinf, chord = v.chord[b];
    const double lscale = -2.0 / (vinf * chord), cpf = -2.0 / (vinf * vinf);
    const PanelGeom *geo = v.geom + mt.panel_off;
    const double *Tg = v.tg + mt.a_off;
    bool conv = true;
    __syncthreads();

    for (int k = 0; k < K; ++k) {
        const double a = v.alpha[mt.alpha_off + k], ex = cos(a), ey = sin(a);
        const double dk = dcl[mt.alpha_off + k];
        const double *cpbar = dcp ? dcp + mt.s_off + (size_t)k * N : nullptr;
        for (int i = tid; i < n1; i += TPB) xk[i] = v.x[mt.x_off + (size_t)k * n1 + i];
        __syncthreads();
        // u_j = (T x)_j + V_inf e.t_j; g_j = dF/du_j; explicit length term
        for (int j = tid; j < N; j += TPB) {
            const PanelGeom g = geo[j];
            double u = vinf * (ex * g.tx + ey * g.ty);
            for (int i = 0; i < n1; ++i) u += Tg[(size_t)i * ld + j] * xk[i];
            double gj = dk * lscale * g.L;
            if (cpbar) gj += cpbar[j] * cpf * u;
            gu[j] = gj;
            const double el = dk * lscale * u;
            ghx[j] += el * g.tx;
            ghy[j] += el * g.ty;
        }
        __syncthreads();
        // w = T^T g: a wavefront per column, lanes along the rows
        for (int i = wave; i < n1; i += TPB / 64) {
            const double *col = Tg + (size_t)i * ld;
            double s = 0.0;
            for (int j = lane; j < N; j += 64) s += col[j] * gu[j];
            s = wave_sum(s);
            if (lane == 0) tmp[i] = s;
        }
        __syncthreads();
        conv = solve_lambda<T>(v, mt, perm, lam, tmp, sblk, part, red) && conv;
        __syncthreads();
        const double xN = xk[N], lN = lam[N];

        // ---- pass 1: a thread per row j -----------------------------------
        for (int j = tid; j < N; j += TPB) {
            const PanelGeom gj = geo[j];
            const double mx = 0.5 * (sx[j] + sx[j + 1]), my = 0.5 * (sy[j] + sy[j + 1]);
            const double g = gu[j], lj = lam[j], kl = (j == 0 || j == N - 1) ? lN : 0.0;
            const double wa0 = g * xN - kl * xN, wt0 = lj * xN;   // the parts of W_A, W_T free of x_i
            const double wa1 = -lj, wt1 = g - kl;                  // ... and the factors of x_i
            double d1x = mx - sx[0], d1y = my - sy[0];
            double q1 = d1x * d1x + d1y * d1y, l1 = plog(q1);
            double ax = 0.0, ay = 0.0, phi = 0.0;
            for (int i = 0; i < N; ++i) {
                const double d2x = mx - sx[i + 1], d2y = my - sy[i + 1];
                const double q2 = d2x * d2x + d2y * d2y, l2 = plog(q2);
                if (i != j) {
                    const PanelGeom gi = geo[i];
                    const double c = gi.tx * gj.tx + gi.ty * gj.ty, s = gi.tx * gj.ty - gi.ty * gj.tx;
                    const double xi = xk[i];
                    const double WA = wa0 + wa1 * xi, WT = wt0 + wt1 * xi;
                    const double aa = WA * s + WT * c, bb = WA * c - WT * s;
                    const double r1 = 1.0 / q1, r2 = 1.0 / q2;
                    // (a d + b perp(d)) / |d|^2 at d1, minus the same at d2
                    ax += (aa * d1x - bb * d1y) * r1 - (aa * d2x - bb * d2y) * r2;
                    ay += (aa * d1y + bb * d1x) * r1 - (aa * d2y + bb * d2x) * r2;
                    const double cr = d1x * d2y - d1y * d2x, dd = d1x * d2x + d1y * d2y;
                    const double beta = patan2(-cr, dd), lg = 0.5 * (l1 - l2);
                    phi += lg * bb - beta * aa;
                }
                d1x = d2x;
                d1y = d2y;
                q1 = q2;
                l1 = l2;
            }
            gmx[j] += kInv2Pi * ax;
            gmy[j] += kInv2Pi * ay;
            // dF/dphi_j: matrix rows, right-hand side, free stream in u
            const double et = ex * gj.tx + ey * gj.ty, ep = -ex * gj.ty + ey * gj.tx;   // e.t, e.perp(t)
            const double dphi = kInv2Pi * phi - lj * vinf * et + g * vinf * ep - kl * vinf * ep;
            const double f = dphi / gj.L;
            ghx[j] += -f * gj.ty;
            ghy[j] += f * gj.tx;
        }

        // ---- pass 2: a thread per node k ----------------------------------
        for (int kn = tid; kn <= N; kn += TPB) {
            const double px = sx[kn], py = sy[kn];
            const bool has_s = kn < N, has_e = kn >= 1;   // panel kn starts / panel kn-1 ends here
            PanelGeom gs{}, ge{};
            double qx = 0.0, qy = 0.0, xs = 0.0, xe = 0.0;
            if (has_s) {
                gs = geo[kn];
                qx = sx[kn + 1];
                qy = sy[kn + 1];
                xs = xk[kn];
            }
            if (has_e) {
                ge = geo[kn - 1];
                xe = xk[kn - 1];
            }
            double ex1 = 0.0, ey1 = 0.0, cphi = 0.0;
            for (int j = 0; j < N; ++j) {
                const PanelGeom gj = geo[j];
                const double mx = 0.5 * (sx[j] + sx[j + 1]), my = 0.5 * (sy[j] + sy[j + 1]);
                const double g = gu[j], lj = lam[j], kl = (j == 0 || j == N - 1) ? lN : 0.0;
                const double wa0 = g * xN - kl * xN, wt0 = lj * xN, wa1 = -lj, wt1 = g - kl;
                const double dx = mx - px, dy = my - py;
                const double q = dx * dx + dy * dy, rq = 1.0 / q;
                if (has_s && j != kn) {   // node kn is P_i of panel i = kn: -d/dd1
                    const double c = gs.tx * gj.tx + gs.ty * gj.ty, s = gs.tx * gj.ty - gs.ty * gj.tx;
                    const double WA = wa0 + wa1 * xs, WT = wt0 + wt1 * xs;
                    const double aa = WA * s + WT * c, bb = WA * c - WT * s;
                    ex1 -= (aa * dx - bb * dy) * rq;
                    ey1 -= (aa * dy + bb * dx) * rq;
                    const double d2x = mx - qx, d2y = my - qy;
                    const double q2 = d2x * d2x + d2y * d2y;
                    const double cr = dx * d2y - dy * d2x, dd = dx * d2x + dy * d2y;
                    const double beta = patan2(-cr, dd), lg = 0.5 * (plog(q) - plog(q2));
                    cphi += lg * bb - beta * aa;
                }
                if (has_e && j != kn - 1) {   // node kn is P_{i+1} of panel i = kn-1: -d/dd2
                    const double c = ge.tx * gj.tx + ge.ty * gj.ty, s = ge.tx * gj.ty - ge.ty * gj.tx;
                    const double WA = wa0 + wa1 * xe, WT = wt0 + wt1 * xe;
                    const double aa = WA * s + WT * c, bb = WA * c - WT * s;
                    ex1 += (aa * dx - bb * dy) * rq;
                    ey1 += (aa * dy + bb * dx) * rq;
                }
            }
            gnx[kn] += kInv2Pi * ex1;
            gny[kn] += kInv2Pi * ey1;
            if (has_s) {   // dF/dphi_kn from the column of panel kn
                const double f = -kInv2Pi * cphi / gs.L;
                ghx[kn] += -f * gs.ty;
                ghy[kn] += f * gs.tx;
            }
        }
        __syncthreads();
    }
    if (info && tid == 0) info[b] = conv ? 0 : -2;

    // ---- node gradients: midpoints split evenly, panel vectors P_{i+1} - P_i
    for (int kn = tid; kn <= N; kn += TPB) {
        double gx = gnx[kn], gy = gny[kn];
        if (kn >= 1) {
            gx += 0.5 * gmx[kn - 1] + ghx[kn - 1];
            gy += 0.5 * gmy[kn - 1] + ghy[kn - 1];
        }
        if (kn < N) {
            gx += 0.5 * gmx[kn] - ghx[kn];
            gy += 0.5 * gmy[kn] - ghy[kn];
        }
        out[2 * kn] = gx;
        out[2 * kn + 1] = gy;
    }
}

}  // namespace

hipError_t launch_adjoint_hs(const WsView &v, int32_t B, int32_t mixed, const double *xy, const double *dcl,
                             const double *dcp, double *dxy, int32_t *info, hipStream_t stream) {
    if (mixed)
        adjoint_hs_kernel<float><<<B, TPB, 0, stream>>>(v, xy, dcl, dcp, dxy, info);
    else
        adjoint_hs_kernel<double><<<B, TPB, 0, stream>>>(v, xy, dcl, dcp, dxy, info);
    return hipGetLastError();
}

hipError_t launch_adjoint(const WsView &v, int32_t B, int32_t n_block, int32_t max_k, int32_t mixed,
                          const double *xy, const double *dcl, const double *dcp, double *dxy, int32_t *info,
                          hipStream_t stream) {
    // without cp cotangents one pass serves all angles; with them one pass
    // per angle index (airfoils with fewer angles skip the later passes)
    const int npass = dcp ? max_k : 1;
    for (int p = 0; p < npass; ++p) {
        const int ka = dcp ? p : -1;
        if (n_block > 0) {
            if (mixed)
                adjoint_kernel<float><<<n_block, TPB, 0, stream>>>(v, xy, dcl, dcp, ka, dxy, info);
            else
                adjoint_kernel<double><<<n_block, TPB, 0, stream>>>(v, xy, dcl, dcp, ka, dxy, info);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const hipError_t e = launch_adjoint_wave(v, n_block, B - n_block, mixed, xy, dcl, dcp, ka, dxy, info, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace panel
