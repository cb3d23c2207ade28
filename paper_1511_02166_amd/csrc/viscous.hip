// viscous.hip -- laminar boundary-layer correction (Thwaites' method) on the
// surface speed of the panel solution: skin-friction drag and lift-to-drag
// ratio, the fitness of the paper's genetic algorithm (Sec. 2).
//
// Per airfoil and angle, with stations at the panel midpoints carrying the
// tangential speed u_j (counter-clockwise tangent):
//   * the stagnation point lies between the first pair u_j < 0 <= u_{j+1},
//     placed by linear interpolation of u along the arc; the upper surface
//     runs from it through panels j, j-1, ..., 0, the lower one through
//     j+1, ..., N-1;
//   * with U = |u| piecewise linear in the arc length s (U = 0 at the
//     stagnation point), theta^2 = 0.45 nu U^-6 int U^5 ds, each segment's
//     integral exact for the linear U; lambda = theta^2 U' / nu with central
//     differences between neighbouring stations;
//   * the layer separates at the first station with lambda < -0.09; up to it
//     each station's wall shear tau_w = mu U l(lambda) / theta (Thwaites'
//     correlation, the usual piecewise fits) acts over its panel along the
//     flow, and its component along the free stream is the drag;
//     nu = vinf c / Re, cd normalised by (1/2) rho vinf^2 c.
// One wavefront per (airfoil, angle).  The running integral is a blocked
// scan: each lane sums a contiguous run of stations, a shuffle scan over the
// lanes offsets the runs, and the lanes then write their stations.
#include "panel_internal.hpp"
#include "wave.hpp"

namespace panel {
namespace {

constexpr int VL = 64;

__device__ __forceinline__ double shear_corr(double lam) {
    return lam >= 0.0 ? 0.22 + 1.57 * lam - 1.8 * lam * lam : 0.22 + 1.402 * lam + 0.018 * lam / (lam + 0.107);
}

__device__ __forceinline__ double seg_u5(double ds, double a, double b) {
    const double a2 = a * a, b2 = b * b;
    return ds * (a2 * a2 * a + a2 * a2 * b + a2 * a * b2 + a2 * b2 * b + a * b2 * b2 + b2 * b2 * b) / 6.0;
}

// Exclusive prefix sum over the wavefront.
__device__ __forceinline__ double wave_exscan(double v) {
    const int lane = threadIdx.x;
    double x = v;
#pragma unroll
    for (int off = 1; off < VL; off <<= 1) {
        const double y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x - v;
}

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return v;
}

struct Side {
    int js, n, sign;   // first panel, station count, panel step (-1 upper, +1 lower)
    double ds0;        // arc length from the stagnation point to station 0
};

// One surface: stations q = 0..n-1 on panels js + sign q.  Returns this
// lane's share of the drag (summed by the caller) and writes the separation
// panel (or -1) to *sep.
__device__ double layer(const Side &sd, const double *su, const PanelGeom *geo, double nu, double vinf, double ex,
                        double ey, double *F, double *U, double *th, int *sep) {
    const int lane = threadIdx.x, n = sd.n;
    auto panel = [&](int q) { return sd.js + sd.sign * q; };
    auto seglen = [&](int q) { return q == 0 ? sd.ds0 : 0.5 * (geo[panel(q - 1)].L + geo[panel(q)].L); };
    for (int q = lane; q < n; q += VL) U[q] = fabs(su[panel(q)]);
    __syncthreads();
    // running integral of U^5 over contiguous runs of stations
    const int run = (n + VL - 1) / VL, q0 = min(lane * run, n), q1 = min(q0 + run, n);
    double part = 0.0;
    for (int q = q0; q < q1; ++q) part += seg_u5(seglen(q), q == 0 ? 0.0 : U[q - 1], U[q]);
    double acc = wave_exscan(part);
    for (int q = q0; q < q1; ++q) {
        acc += seg_u5(seglen(q), q == 0 ? 0.0 : U[q - 1], U[q]);
        F[q] = acc;
    }
    __syncthreads();
    for (int q = lane; q < n; q += VL) {
        const double u = U[q], u3 = u * u * u;
        th[q] = sqrt(0.45 * nu * F[q] / (u3 * u3));
    }
    __syncthreads();
    // pressure-gradient parameter, first separated station
    int first = n;
    for (int q = lane; q < n; q += VL) {
        double dUds;
        if (n == 1)
            dUds = U[0] / sd.ds0;
        else if (q == 0)
            dUds = U[1] / (sd.ds0 + seglen(1));
        else if (q == n - 1)
            dUds = (U[q] - U[q - 1]) / seglen(q);
        else
            dUds = (U[q + 1] - U[q - 1]) / (seglen(q) + seglen(q + 1));
        const double lam = th[q] * th[q] / nu * dUds;
        F[q] = lam;   // reuse: F now holds lambda
        if (lam < -0.09) first = min(first, q);
    }
    first = wave_min_int(first);
    __syncthreads();
    double drag = 0.0;
    for (int q = lane; q < first; q += VL) {
        const int j = panel(q);
        const PanelGeom g = geo[j];
        const double dir = su[j] >= 0.0 ? 1.0 : -1.0;
        const double cf = 2.0 * nu * U[q] * shear_corr(F[q]) / (th[q] * vinf * vinf);
        drag += cf * g.L * dir * (g.tx * ex + g.ty * ey);
    }
    *sep = first < n ? panel(first) : -1;
    __syncthreads();
    return drag;
}

__global__ __launch_bounds__(VL) void thwaites_kernel(WsView v, const double *__restrict__ gamma,
                                                     const double *__restrict__ cl, double re,
                                                     double *__restrict__ cd, double *__restrict__ ld,
                                                     int32_t *__restrict__ sep) {
    const int b = blockIdx.x, k = blockIdx.y;
    const AirfoilMeta mt = v.meta[b];
    if (k >= mt.K) return;
    const int N = mt.N, lane = threadIdx.x;
    const int ka = mt.alpha_off + k;
    const double vinf = v.hdr->vinf, chord = v.chord[b];
    const double nu = vinf * chord / re;
    const double a = v.alpha[ka], ex = cos(a), ey = sin(a);
    const PanelGeom *geo = v.geom + mt.panel_off;
    const double *u = gamma + mt.s_off + (size_t)k * N;
    __shared__ double su[PANEL_NMAX], F[PANEL_NMAX], U[PANEL_NMAX], th[PANEL_NMAX];
    for (int j = lane; j < N; j += VL) su[j] = u[j];
    __syncthreads();
    int js = N;
    for (int j = lane; j + 1 < N; j += VL)
        if (su[j] < 0.0 && su[j + 1] >= 0.0) js = min(js, j);
    js = wave_min_int(js);
    if (js >= N || v.flag[b] != 0) {
        if (lane == 0) {
            cd[ka] = ld[ka] = __builtin_nan("");
            sep[2 * ka] = sep[2 * ka + 1] = -2;
        }
        return;
    }
    const double dseg = 0.5 * (geo[js].L + geo[js + 1].L);
    const double f = -su[js] / (su[js + 1] - su[js]);
    Side up{js, js + 1, -1, f * dseg}, lo{js + 1, N - 1 - js, 1, (1.0 - f) * dseg};
    int sep_u = -1, sep_l = -1;
    double drag = layer(up, su, geo, nu, vinf, ex, ey, F, U, th, &sep_u);
    drag += layer(lo, su, geo, nu, vinf, ex, ey, F, U, th, &sep_l);
    drag = wave_sum(drag);
    if (lane == 0) {
        const double c = drag / chord;
        cd[ka] = c;
        ld[ka] = cl[ka] / c;
        sep[2 * ka] = sep_u;
        sep[2 * ka + 1] = sep_l;
    }
}

}  // namespace

hipError_t launch_thwaites(const WsView &v, int32_t B, int32_t max_k, const double *gamma, const double *cl,
                           double re, double *cd, double *ld, int32_t *sep, hipStream_t stream) {
    dim3 grid(B, max_k);
    thwaites_kernel<<<grid, VL, 0, stream>>>(v, gamma, cl, re, cd, ld, sep);
    return hipGetLastError();
}

}  // namespace panel
