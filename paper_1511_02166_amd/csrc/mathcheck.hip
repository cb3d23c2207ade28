// mathcheck.hip -- evaluates the kernels' own log and atan2 on given inputs
// (diagnostic entry point panel_math_eval, used by the accuracy tests).
#include "fastmath.hpp"
#include "panel_internal.hpp"

namespace panel {
namespace {

__global__ void math_eval_kernel(int n, const double *__restrict__ x, const double *__restrict__ y,
                                 double *__restrict__ lg, double *__restrict__ at) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i];
    if (lg) lg[i] = plog(xi);
    if (at) at[i] = patan2(y[i], xi);
}

}  // namespace

hipError_t launch_math_eval(int32_t n, const double *x, const double *y, double *lg, double *at,
                            hipStream_t stream) {
    math_eval_kernel<<<(n + 255) / 256, 256, 0, stream>>>(n, x, y, lg, at);
    return hipGetLastError();
}

}  // namespace panel
