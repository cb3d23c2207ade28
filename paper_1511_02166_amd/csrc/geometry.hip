// geometry.hip -- NACA 4-digit node generation and its vector-Jacobian
// product on gfx950 (geometry helper for the GA population of Sec. 2; the
// genome there is a B-spline, the seeded workloads use NACA sections).
#include "panel_internal.hpp"

namespace panel {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct NacaPoint {
    double X, Y;
    // derivatives of (X, Y) with respect to (m, p, t)
    double dX[3], dY[3];
};

// Node k of an N-panel section: station x from cosine spacing (mirrored
// index s = min(k, N-k) so both surfaces share x exactly), thickness laid
// off along the camber-line normal; cos/sin of the camber slope angle come
// from the slope s' as 1/sqrt(1+s'^2) and s'/sqrt(1+s'^2).
template <bool WITH_JAC>
__device__ NacaPoint naca_point(double m, double p, double t, int k, int N, int closed_te) {
    const double a4 = closed_te ? -0.1036 : -0.1015;
    const int half = N >> 1;
    const int s = k <= half ? k : N - k;
    const double x = 0.5 * (1.0 + cos(kPi * double(s) / double(half)));
    const double poly = 0.2969 * sqrt(x) - 0.1260 * x - 0.3516 * x * x + 0.2843 * x * x * x +
                        a4 * x * x * x * x;
    const double yt = 5.0 * t * poly;
    double yc = 0.0, dyc = 0.0;
    double dyc_m = 0.0, dyc_p = 0.0, ddyc_m = 0.0, ddyc_p = 0.0;
    if (m != 0.0) {
        if (x < p) {
            const double ip2 = 1.0 / (p * p);
            yc = m * ip2 * (2.0 * p * x - x * x);
            dyc = 2.0 * m * ip2 * (p - x);
            if (WITH_JAC) {
                dyc_m = ip2 * (2.0 * p * x - x * x);
                dyc_p = 2.0 * m * x * (x - p) * ip2 / p;
                ddyc_m = 2.0 * ip2 * (p - x);
                ddyc_p = 2.0 * m * (2.0 * x - p) * ip2 / p;
            }
        } else {
            const double q = 1.0 - p;
            const double iq2 = 1.0 / (q * q);
            const double f = (1.0 - 2.0 * p) + 2.0 * p * x - x * x;
            yc = m * iq2 * f;
            dyc = 2.0 * m * iq2 * (p - x);
            if (WITH_JAC) {
                dyc_m = iq2 * f;
                dyc_p = m * iq2 / q * ((2.0 * x - 2.0) * q + 2.0 * f);
                ddyc_m = 2.0 * iq2 * (p - x);
                ddyc_p = 2.0 * m * iq2 / q * (q + 2.0 * (p - x));
            }
        }
    }
    const double c = 1.0 / sqrt(1.0 + dyc * dyc);
    const double sn = dyc * c;
    const double sg = k <= half ? 1.0 : -1.0;  // upper: -yt sin, +yt cos
    NacaPoint r;
    r.X = x - sg * yt * sn;
    r.Y = yc + sg * yt * c;
    if (WITH_JAC) {
        // d sin/d slope = c^3, d cos/d slope = -sn c^2
        const double dsn = c * c * c, dc = -sn * c * c;
        const double dyt[3] = {0.0, 0.0, 5.0 * poly};
        const double dycv[3] = {dyc_m, dyc_p, 0.0};
        const double dsl[3] = {ddyc_m, ddyc_p, 0.0};
        for (int q = 0; q < 3; ++q) {
            r.dX[q] = -sg * (dyt[q] * sn + yt * dsn * dsl[q]);
            r.dY[q] = dycv[q] + sg * (dyt[q] * c + yt * dc * dsl[q]);
        }
    }
    return r;
}

__global__ __launch_bounds__(256) void naca4_kernel(const int32_t *__restrict__ node_off,
                                                    int32_t closed_te,
                                                    const double *__restrict__ mpt,
                                                    double *__restrict__ xy) {
    const int b = blockIdx.x;
    const int n0 = node_off[b];
    const int N = node_off[b + 1] - n0 - 1;
    const double m = mpt[3 * b], p = mpt[3 * b + 1], t = mpt[3 * b + 2];
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        const int kk = (closed_te && k == N) ? 0 : k;
        NacaPoint r = naca_point<false>(m, p, t, kk, N, closed_te);
        xy[2 * (n0 + k)] = r.X;
        xy[2 * (n0 + k) + 1] = r.Y;
    }
}

__global__ __launch_bounds__(256) void naca4_vjp_kernel(const int32_t *__restrict__ node_off,
                                                        int32_t closed_te,
                                                        const double *__restrict__ mpt,
                                                        const double *__restrict__ dxy,
                                                        double *__restrict__ dmpt) {
    const int b = blockIdx.x;
    const int n0 = node_off[b];
    const int N = node_off[b + 1] - n0 - 1;
    const double m = mpt[3 * b], p = mpt[3 * b + 1], t = mpt[3 * b + 2];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        const int kk = (closed_te && k == N) ? 0 : k;
        NacaPoint r = naca_point<true>(m, p, t, kk, N, closed_te);
        const double gx = dxy[2 * (n0 + k)], gy = dxy[2 * (n0 + k) + 1];
        for (int q = 0; q < 3; ++q) acc[q] += gx * r.dX[q] + gy * r.dY[q];
    }
    __shared__ double red[3][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < 3; ++q) {
        double v = acc[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[q][w];
        dmpt[3 * b + q] = s;
    }
}

}  // namespace

hipError_t launch_naca4(int32_t B, const int32_t *node_off, int32_t closed_te, const double *mpt,
                        double *xy, hipStream_t stream) {
    naca4_kernel<<<B, 256, 0, stream>>>(node_off, closed_te, mpt, xy);
    return hipGetLastError();
}

hipError_t launch_naca4_vjp(int32_t B, const int32_t *node_off, int32_t closed_te,
                            const double *mpt, const double *dxy, double *dmpt, hipStream_t stream) {
    naca4_vjp_kernel<<<B, 256, 0, stream>>>(node_off, closed_te, mpt, dxy, dmpt);
    return hipGetLastError();
}

}  // namespace panel
