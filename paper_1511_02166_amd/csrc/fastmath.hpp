// fastmath.hpp -- the FP64 natural logarithm and two-argument arctangent used
// by the assembly and adjoint kernels.
//
// Every influence coefficient needs one logarithm and one arctangent (the
// paper's Sec. 3 names them as the cost of the assembly).  The device
// library's general-purpose versions spend ~150 instructions each on
// extended-precision internals; these spend ~35-40 and stay within 1-2 ulp
// (measured against the host libm in the tests), which is well inside what
// the 1e-10 solution tolerance needs (entry errors up to ~1e-14 relative
// leave Cp within ~1e-11 at N = 256).
//
// log(x), x > 0 normal: x = 2^e m with m in [sqrt(1/2), sqrt(2)); with
// f = m - 1 and s = f / (2 + f), log(m) = 2 atanh(s) = 2s + s R(s^2) where
// R(z) = z (2/3 + 2z/5 + 2z^2/7 + ...), |s| <= 0.172.  Since 2s = f - s f,
// log(m) = f - s (f - R): the leading term f is exact and the rounding of the
// small correction barely matters.  e ln2 is added in two pieces, the high
// one with few enough bits that e * LN2_HI is exact (Cody and Waite's
// argument-reduction split; the constants are ln 2 and pi themselves, cut
// into a short head and the remainder).
//
// atan2(y, x): fold to t = min(|x|,|y|) / max(|x|,|y|) in [0, 1], pick the
// nearest centre c = i/4 (i = 0..4), and use atan(t) = atan(c) + atan(u) with
// u = (t - c) / (1 + c t) = (num - c den) / (den + c num) (one division,
// |u| <= ~0.13); atan(u) = u + u z P(z), z = u^2, from its Taylor series.
// The octant and quadrant are restored with pi/2 - r and pi - r evaluated
// with split constants.
#pragma once

#include <hip/hip_runtime.h>

namespace panel {

// q = a / b for b of moderate size (no overflow / underflow paths): hardware
// reciprocal, one Newton step on it, and one residual correction of the
// quotient (within 1 ulp).
__device__ __forceinline__ double pdiv(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
}

namespace fm {
constexpr double kSqrtHalf = 0.7071067811865476;
constexpr double kLn2Hi = 0.6931471803691238;      // ln 2 to 32 significant bits
constexpr double kLn2Lo = 1.9082149292705877e-10;  // ln 2 - kLn2Hi
constexpr double kPiHi = 3.141592653589793;
constexpr double kPiLo = 1.2246467991473532e-16;
constexpr double kPi2Hi = 1.5707963267948966;
constexpr double kPi2Lo = 6.123233995736766e-17;
constexpr double kAtanQ1 = 0.24497866312686414;    // atan(1/4)
constexpr double kAtanQ2 = 0.4636476090008061;     // atan(1/2)
constexpr double kAtanQ3 = 0.6435011087932844;     // atan(3/4)
constexpr double kAtanQ4 = 0.7853981633974483;     // atan(1) = pi/4
// Series coefficients, read from constant memory: loaded once per kernel
// into scalar registers, they enter each FMA as a scalar operand (written
// as literals, the compiler keeps them in vector registers and copies one
// into the accumulator of every Horner step).
inline __constant__ double kLogPoly[10] = {2.0 / 21.0, 2.0 / 19.0, 2.0 / 17.0, 2.0 / 15.0, 2.0 / 13.0,
                                           2.0 / 11.0, 2.0 / 9.0,  2.0 / 7.0,  2.0 / 5.0,  2.0 / 3.0};
inline __constant__ double kAtanPoly[9] = {-1.0 / 19.0, 1.0 / 17.0, -1.0 / 15.0, 1.0 / 13.0, -1.0 / 11.0,
                                           1.0 / 9.0,   -1.0 / 7.0, 1.0 / 5.0,   -1.0 / 3.0};
}  // namespace fm

__device__ __forceinline__ double plog(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);   // [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool lo = m < fm::kSqrtHalf;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;
    const double s = pdiv(f, 2.0 + f);
    const double z = s * s;
    double R = fm::kLogPoly[0];   // z (2/3 + 2z/5 + ... + 2z^9/21)
#pragma unroll
    for (int k = 1; k < 10; ++k) R = fma(R, z, fm::kLogPoly[k]);
    R *= z;
    const double lm = f - s * (f - R);
    const double ef = (double)e;
    return fma(ef, fm::kLn2Hi, fma(ef, fm::kLn2Lo, lm));
}

__device__ __forceinline__ double patan2(double y, double x) {
    const double ax = fabs(x), ay = fabs(y);
    const bool sw = ay > ax;
    const double num = sw ? ax : ay, den = sw ? ay : ax;
    // nearest centre from an approximate quotient (any centre keeps |u| small)
    const double ta = num * __builtin_amdgcn_rcp(den);
    const double fi = fmin(fmax(__builtin_rint(4.0 * ta), 0.0), 4.0);
    const double c = 0.25 * fi;
    const double u = pdiv(fma(-c, den, num), fma(c, num, den));
    const double z = u * u;
    double P = fm::kAtanPoly[0];   // -1/3 + z/5 - ... - z^8/19
#pragma unroll
    for (int k = 1; k < 9; ++k) P = fma(P, z, fm::kAtanPoly[k]);
    const double at = fma(u * z, P, u);
    const int i = (int)fi;
    const double base = i == 0 ? 0.0 : i == 1 ? fm::kAtanQ1 : i == 2 ? fm::kAtanQ2 : i == 3 ? fm::kAtanQ3 : fm::kAtanQ4;
    double r = base + at;
    r = sw ? (fm::kPi2Hi - r) + fm::kPi2Lo : r;
    r = (x < 0.0) ? (fm::kPiHi - r) + fm::kPiLo : r;
    return copysign(r, y);
}

}  // namespace panel
