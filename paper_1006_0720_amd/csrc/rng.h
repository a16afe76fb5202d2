// Counter-based random numbers for the particle kernels (device side).
//
// The paper draws 6 Gaussian numbers per particle and step from per-step tables
// filled by block-split streams (Ch.3, Sec. Parallel random number generation).
// Here every number is a pure function of (seed, particle id, step, sub-stream)
// through Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), so no table is
// stored and the result does not depend on thread count or storage order.
//
// Sub-streams of one particle-step: 0 and 1 give the 6 normals and the uniform
// eta of the wall test; 16 + 32*h + a is attempt a of the gamma variate drawn
// at wall hit h.  Seeding uses step tag 0xFFFFFFFF.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdfk {

struct u32x4 {
  uint32_t a, b, c, d;
};

// Philox4x32 with 10 rounds: multipliers 0xD2511F53 and 0xCD9E8D57, key
// increments 0x9E3779B9 and 0xBB67AE85 between rounds.
__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    // one 32x32 -> 64-bit product each (v_mad_u64_u32) instead of separate
    // low and high multiplies
    const uint64_t p0 = (uint64_t)m0 * c0, p1 = (uint64_t)m1 * c2;
    uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    uint32_t t0 = hi1 ^ c1 ^ k0;
    uint32_t t2 = hi0 ^ c3 ^ k1;
    c0 = t0;
    c1 = lo1;
    c2 = t2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// Uniform on (0,1) from the top 23 bits: (2k+1) 2^-24, exact in binary32.
__device__ __forceinline__ float unif_f(uint32_t r) {
  return __int2float_rn((int)(r >> 9)) * 1.1920928955078125e-07f + 5.9604644775390625e-08f;
}
__device__ __forceinline__ double unif_d(uint32_t r) {
  return ((double)(r >> 9) + 0.5) * 1.1920928955078125e-07;
}

// Box-Muller pair in binary64 (the angle through sincospi: no range reduction).
__device__ __forceinline__ void box_muller_d(uint32_t r1, uint32_t r2, double &z0, double &z1) {
  const double u1 = unif_d(r1), u2 = unif_d(r2);
  const double rad = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// Box-Muller pair in binary32 on the hardware transcendental units:
// v_log_f32 is log2, v_sin_f32 / v_cos_f32 take their argument in revolutions
// (sin(2 pi x)), so -2 ln u = -2 ln(2) log2(u) and the angle needs no scaling.
__device__ __forceinline__ void box_muller_f(uint32_t r1, uint32_t r2, float &z0, float &z1) {
  const float u1 = unif_f(r1), u2 = unif_f(r2);
  const float rad = __builtin_amdgcn_sqrtf(-1.38629436112f * __builtin_amdgcn_logf(u1));
  z0 = rad * __builtin_amdgcn_cosf(u2);
  z1 = rad * __builtin_amdgcn_sinf(u2);
}

// Gamma(shape, scale) for shape >= 1 by Marsaglia & Tsang (ACM TOMS 26, 2000),
// binary64.  Attempt a draws Philox sub-stream subbase + a; after 32
// rejections the mean is returned and *fail is set.
__device__ inline double gamma_mt(double shape, double scale, uint32_t k0, uint32_t k1, uint32_t id,
                                  uint32_t step, uint32_t subbase, int *fail) {
  const double d = shape - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  for (uint32_t a = 0; a < 32; ++a) {
    u32x4 r = philox10(id, step, subbase + a, 0u, k0, k1);
    double z, z1;
    box_muller_d(r.a, r.b, z, z1);
    double v = 1.0 + c * z;
    if (v <= 0.0) continue;
    v = v * v * v;
    double u = unif_d(r.c);
    if (log(u) < 0.5 * z * z + d - d * v + d * log(v)) return d * v * scale;
  }
  *fail = 1;
  return shape * scale;
}

}  // namespace pdfk
