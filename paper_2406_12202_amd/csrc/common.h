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
// Scans and reductions over a 64-lane wave by DPP lane moves: an inclusive
// scan is row shifts by 1, 2, 4 and 8 lanes (within 16-lane rows), then the
// row broadcasts of lane 15 (into rows 1 and 3) and of lane 31 (into rows 2
// and 3); a few cycles per step where a lane shuffle through LDS takes about
// a hundred.  After the first five steps each 32-lane half holds the scan of
// its own lanes; the sixth joins the halves.  The order is fixed, so every
// result is deterministic.

// a 4- or 8-byte value moved by DPP control CTRL (row mask RM); `fill` where
// the control has no source lane or the row is masked off
template <int CTRL, int RM, class T>
__device__ __forceinline__ T dpp_move(const T v, const T fill) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  if constexpr (sizeof(T) == 4) {
    const int u = __builtin_bit_cast(int, v), f = __builtin_bit_cast(int, fill);
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(f, u, CTRL, RM, 0xf, false));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long f = __builtin_bit_cast(unsigned long long, fill);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)u, CTRL, RM, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(u >> 32),
                                                              CTRL, RM, 0xf, false);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// inclusive scan within each 32-lane half, with the associative op whose
// identity is `id`
template <class T, class Op>
__device__ __forceinline__ T half_scan(T v, const T id, Op op) {
  v = op(v, dpp_move<0x111, 0xf>(v, id));   // row_shr:1
  v = op(v, dpp_move<0x112, 0xf>(v, id));   // row_shr:2
  v = op(v, dpp_move<0x114, 0xf>(v, id));   // row_shr:4
  v = op(v, dpp_move<0x118, 0xf>(v, id));   // row_shr:8
  v = op(v, dpp_move<0x142, 0xa>(v, id));   // row_bcast:15 into rows 1 and 3
  return v;
}
// inclusive scan over the whole wave
template <class T, class Op>
__device__ __forceinline__ T wave_scan(T v, const T id, Op op) {
  v = half_scan(v, id, op);
  return op(v, dpp_move<0x143, 0xc>(v, id));   // row_bcast:31 into rows 2 and 3
}

// the value of lane `lane` (wave-uniform)
template <class T>
__device__ __forceinline__ T lane_value(const T v, const int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

struct OpAddF {
  __device__ float operator()(const float a, const float b) const { return a + b; }
};
struct OpMinI {
  __device__ int operator()(const int a, const int b) const { return min(a, b); }
};

__device__ inline float wave_incl_scan(float v, int) { return wave_scan(v, 0.0f, OpAddF{}); }
__device__ inline float wave_sum(float v) { return lane_value(wave_scan(v, 0.0f, OpAddF{}), 63); }
__device__ inline int wave_min_int(int v) { return lane_value(wave_scan(v, 0x7fffffff, OpMinI{}), 63); }

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
