// adjoint.hip -- reverse-mode lift sensitivity (placeholder until the
// transposed-solve kernels land).
#include "panel_internal.hpp"

namespace panel {

hipError_t launch_adjoint(const WsView &, int32_t, int32_t, int32_t, const double *, const double *,
                          double *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace panel
