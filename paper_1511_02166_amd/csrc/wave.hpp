// wave.hpp -- wavefront-level primitives for gfx950 (64 lanes): DPP
// exchanges inside 16-lane rows and scalar-register broadcasts.
#pragma once

#include <hip/hip_runtime.h>

namespace panel {

template <int CTRL> __device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ inline float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double readlane_t(double v, int l) { return readlane_d(v, l); }
__device__ inline float readlane_t(float v, int l) { return readlane_f(v, l); }

// Maximum over the 64 lanes, returned to every lane: DPP butterflies inside
// each 16-lane row (exchange with lane^1, lane^2, the mirrored half-row and
// the mirrored row), then the four row results through scalar registers.
__device__ inline double wave_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fmax(v, dpp_d<0x4E>(v));    // quad_perm [2,3,0,1]
    v = fmax(v, dpp_d<0x141>(v));   // row_half_mirror
    v = fmax(v, dpp_d<0x140>(v));   // row_mirror
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}


template <int CTRL> __device__ inline float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes, returned to every lane (same DPP pattern as wave_max).
__device__ inline double wave_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

}  // namespace panel
