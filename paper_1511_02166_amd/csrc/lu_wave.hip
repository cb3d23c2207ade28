// lu_wave.hip -- kernels that run one wavefront per workgroup over a range of
// the plan's airfoil order: the factorisation + solve, and the refinement of
// FP32 factors (device code in lu_wave_impl.hpp).
#include "lu_wave_impl.hpp"

namespace panel {
namespace {

using namespace wv;

template <typename T>
__global__ __launch_bounds__(WL, 2) void lu_wave_kernel(WsView v, int32_t first, int32_t *__restrict__ info_out) {
    __shared__ WaveLuLds<T> W;
    wave_lu<T>(v, v.order[first + blockIdx.x], info_out, W);
}

__global__ __launch_bounds__(WL, 2) void refine_wave_kernel(WsView v, int32_t first, int32_t *__restrict__ info,
                                                         double tol, int max_iter) {
    __shared__ WaveRefLds W;
    wave_refine(v, v.order[first + blockIdx.x], info, tol, max_iter, W);
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

hipError_t launch_refine_wave(const WsView &v, int32_t first, int32_t count, int32_t *info, double tol,
                              int32_t max_iter, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    refine_wave_kernel<<<count, WL, 0, stream>>>(v, first, info, tol, max_iter);
    return hipGetLastError();
}

}  // namespace panel
