// Shared device helpers of the gfx950 particle-update library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

constexpr int kWave = 64;

// A dispatch counts work-items per grid dimension in 32 bits, so launches of
// many workgroups are folded into rows (grid.y) of at most kGridRow
// workgroups, and the kernel recovers its workgroup number with
// flat_block(); the last row may end past the work, so a kernel leaves
// whole workgroups whose number is out of range.  Rows are short enough that
// ordinary map launches (a few million samples) already span several.
constexpr long kGridRow = 1L << 13;
inline dim3 folded_grid(const long blocks) {
  const long rows = (blocks + kGridRow - 1) / kGridRow;
  return dim3((unsigned)((blocks + rows - 1) / rows), (unsigned)rows);
}
__device__ __forceinline__ long flat_block() { return (long)blockIdx.y * gridDim.x + blockIdx.x; }

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

// ---------------------------------------------------------------- camera rays
// Ray of pixel (u, v) for a camera-to-world pose P (3 x 4, row-major): OpenGL
// camera looking along -z, pixel centres at +1/2 (Eq. 4's r(p, x) with
// intrinsics K).  Float32 throughout: the pose and the intrinsics are rounded
// to float32 once, the camera-frame direction is formed and rotated with
// explicit fused multiply-adds (so every kernel that forms a ray gets the
// same bits) and normalised.  Float64 stays with the poses themselves.
__device__ __forceinline__ void camera_ray(const double* P, int u, int v, double fx, double fy, double cx, double cy,
                                           float (&o)[3], float (&d)[3]) {
  const float dc0 = ((float)u + 0.5f - (float)cx) / (float)fx;
  const float dc1 = -(((float)v + 0.5f - (float)cy) / (float)fy);
  float r[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[3 * k] = (float)P[4 * k];
    r[3 * k + 1] = (float)P[4 * k + 1];
    r[3 * k + 2] = (float)P[4 * k + 2];
  }
  float d0 = fmaf(r[0], dc0, fmaf(r[1], dc1, -r[2]));
  float d1 = fmaf(r[3], dc0, fmaf(r[4], dc1, -r[5]));
  float d2 = fmaf(r[6], dc0, fmaf(r[7], dc1, -r[8]));
  const float inv = 1.0f / sqrtf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
  o[0] = (float)P[3]; o[1] = (float)P[7]; o[2] = (float)P[11];
  d[0] = d0 * inv; d[1] = d1 * inv; d[2] = d2 * inv;
}

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

// Eq. 6's per-particle sums in one fixed order, shared by every kernel that
// forms them: with G = particle_group(B) lanes per particle, lane g adds
// E_j F_j and F_j for j = g, g + G, ... in float64, then a butterfly (xor
// G/2, ..., 1) within the group combines the G partial sums; addition being
// commutative, every lane of the group ends with the same totals.
// get(j, ef, f) supplies the float32 E_j F_j and F_j.  The G lanes must be an
// aligned group of a wave, and all lanes of the wave must call together.
__host__ __device__ inline int particle_group(int B) {
  int G = 1;
  while (G * 2 <= B && G < kWave) G *= 2;
  return G;
}

template <class Get>
__device__ inline void particle_sums(Get get, int B, int G, int g, double& S, double& Fs) {
  double s = 0.0, f = 0.0;
  for (int j = g; j < B; j += G) {
    float ef, fj;
    get(j, ef, fj);
    s += (double)ef;
    f += (double)fj;
  }
  for (int o = G / 2; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, kWave);
    f += __shfl_xor(f, o, kWave);
  }
  S = s;
  Fs = f;
}

}  // namespace fl
