// gravity_common.h -- what the direct-sum and tree gravity kernels share:
// the per-slot source records, the DPP lane rotation and the softened
// inverse cube from the hardware rsqrt estimate.
#pragma once
#include "dem_internal.h"

namespace dem {

namespace {

struct alignas(64) Rec64 {
  double x, y, z, m, e, p0, p1, p2;
};
struct alignas(32) Rec32 {
  float x, y, z, m, e, p0, p1, p2;
};

// Records are read through the constant address space: with a uniform index
// these become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) Rec64* ConstRec64;
typedef const __attribute__((address_space(4))) Rec32* ConstRec32;

// Rotate a value by one lane across the whole wave (DPP wave_ror:1): after
// 64 rotations every value is back in its own lane.
__device__ __forceinline__ float ror1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xF, 0xF, true));
}
__device__ __forceinline__ double ror1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x13C, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x13C, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Series coefficients of the rsqrt corrections, held in VGPRs for the whole
// kernel.  Left as literals, the compiler re-materialises 1.5 into the
// accumulator of a two-operand FMA at every use (a VOP3 FMA takes no 64-bit
// literal): one extra move per pair.  The empty asm statement only hides the
// values from constant folding; it emits no instruction.
__device__ __forceinline__ void series_coeffs(double& c15) {
  c15 = 1.5;
  asm("" : "+v"(c15));
}
__device__ __forceinline__ void series_coeffs(double& c15, double& c1875) {
  c15 = 1.5;
  c1875 = 1.875;
  asm("" : "+v"(c15), "+v"(c1875));
}

// r^-3 of a softened squared distance, FP64: the hardware estimate
// y0 = r^-1 (1 + d) (|d| <= 5.3e-8 measured on MI355X over 4M arguments from
// e^-30 to e^30) and the first-order correction r^-3 = y0^3 (1 + 3e/2),
// e = 1 - r^2 y0^2 = -2d - d^2, whose relative error is 6 d^2 + O(d^3),
// at most 1.7e-14.
template <bool SOFT>
__device__ __forceinline__ double inv_cube(double r2, double c15) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double y3 = y2 * y;
  const double c3 = fma(y3 * e, c15, y3);
  if (!SOFT) return r2 > 0.0 ? c3 : 0.0;
  return c3;
}

template <bool SOFT>
__device__ __forceinline__ float inv_cube(float r2, double) {
  const float y = __builtin_amdgcn_rsqf(r2);
  const float c3 = (y * y) * y;
  if (!SOFT) return r2 > 0.f ? c3 : 0.f;
  return c3;
}

}  // namespace

}  // namespace dem
