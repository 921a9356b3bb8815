// Shared device helpers of the gfx950 particle-update library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

constexpr int kWave = 64;

// Philox stream tags (top byte of counter word 3); see fastloc.h.
enum : uint32_t { kStreamPix = 1, kStreamJitCoarse = 2, kStreamJitFine = 3,
                  kStreamMotion = 4, kStreamResample = 5 };

struct u32x4 { uint32_t x, y, z, w; };

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of
// (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2, x <- (hi1^x1^k0, lo1, hi0^x3^k1, lo0),
// with the key advanced by the Weyl constants between rounds.
__host__ __device__ inline u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return {c0, c1, c2, c3};
}

__host__ __device__ inline u32x4 draw(uint64_t seed, uint64_t iter, uint32_t stream,
                                      uint32_t c0, uint32_t c1, uint32_t group) {
  return philox(c0, c1, (uint32_t)iter, (stream << 24) | group, (uint32_t)seed,
                (uint32_t)(seed >> 32));
}

__host__ __device__ inline uint32_t pick(const u32x4& w, int i) {
  return i == 0 ? w.x : (i == 1 ? w.y : (i == 2 ? w.z : w.w));
}

// uniform in [0, 1) with 24 bits: exact in float
__host__ __device__ inline float unit24(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-08f; }
// uniform in (0, 1): (w + 1/2) 2^-32, exact in double
__host__ __device__ inline double unit_open(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386963e-10; }

// ---------------------------------------------------------------- wave primitives
__device__ inline float wave_incl_scan(float v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const float u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ inline int wave_min_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

}  // namespace fl
