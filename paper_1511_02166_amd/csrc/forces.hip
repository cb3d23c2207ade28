// forces.hip -- surface speed, pressure coefficient and lift on gfx950.
//
// The paper (Sec. 2, Fig. 2) reports the lift coefficient of its panel code
// without printing the formula.  With the stream function constant inside
// the contour, the outer tangential speed on panel i equals the sheet
// strength gamma_i (counter-clockwise tangent), so Cp_i = 1 - (gamma_i/vinf)^2;
// the lift follows from the circulation sum_i gamma_i L_i by Kutta-Joukowski,
// Cl = -2 sum_i gamma_i L_i / (vinf c), and from the pressure integral
// Cl_p = -(1/c) sum_i Cp_i L_i (n_i . e_L), e_L = (-sin a, cos a).
// One workgroup per (airfoil, angle); a wavefront-shuffle + LDS reduction.
#include "panel_internal.hpp"

namespace panel {
namespace {

__global__ __launch_bounds__(256) void forces_kernel(WsView v, double *__restrict__ gamma,
                                                     double *__restrict__ cp, double *__restrict__ cl,
                                                     double *__restrict__ cl_p) {
    const int b = blockIdx.x, k = blockIdx.y;
    const AirfoilMeta mt = v.meta[b];
    if (k >= mt.K) return;
    const int N = mt.N;
    const double vinf = v.hdr->vinf;
    const double chord = v.chord[b];
    const double a = v.alpha[mt.alpha_off + k];
    const double ex = -sin(a), ey = cos(a);
    const double *x = v.x + mt.x_off + (size_t)k * mt.n1;
    const PanelGeom *geo = v.geom + mt.panel_off;
    const size_t so = mt.s_off + (size_t)k * N;
    const double iv = 1.0 / vinf;
    double circ = 0.0, fl = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double g = x[i];
        const PanelGeom pg = geo[i];
        const double u = g * iv;
        const double c = 1.0 - u * u;
        if (gamma) gamma[so + i] = g;
        if (cp) cp[so + i] = c;
        circ += g * pg.L;
        fl += c * pg.L * (pg.ty * ex - pg.tx * ey);
    }
    __shared__ double red[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        circ += __shfl_xor(circ, off);
        fl += __shfl_xor(fl, off);
    }
    if (lane == 0) {
        red[0][wave] = circ;
        red[1][wave] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sc = 0.0, sf = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            sc += red[0][w];
            sf += red[1][w];
        }
        cl[mt.alpha_off + k] = -2.0 * sc / (vinf * chord);
        if (cl_p) cl_p[mt.alpha_off + k] = -sf / chord;
    }
}

}  // namespace

hipError_t launch_forces(const WsView &v, int32_t B, int32_t max_k, double *gamma, double *cp,
                         double *cl, double *cl_p, hipStream_t stream) {
    dim3 grid(B, max_k);
    forces_kernel<<<grid, 256, 0, stream>>>(v, gamma, cp, cl, cl_p);
    return hipGetLastError();
}

}  // namespace panel
