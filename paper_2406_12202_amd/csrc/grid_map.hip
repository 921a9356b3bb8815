// Multi-resolution grid map (the map type of Sec. IV-B, restated as a
// multiresolution hash encoding with a tiny MLP): per sample, L levels of
// trilinear blends of two-feature table entries at the 8 cell corners (dense
// index while the level's vertices fit the table, the spatial hash of three
// primes otherwise), then z = W2 relu(W1 f + b1) + b2, sigma = softplus(z_0),
// rgb = sigmoid(W4 relu(W3 [z, gamma(d)] + b3) + b4).  Points outside the
// box [-bound, bound]^3 are empty.
//
// One thread per sample, the same sample sets and stratified placement as the
// MLP kernels (MlpArgs).  The tables hold half-precision feature pairs (one
// 32-bit word per entry).  The work is 8 L random 4-byte table reads per
// sample (512 B for 16 levels) against about 5 K multiply-adds, so the kernel is
// bound by the gather: the coarse levels stay in L2, the fine ones come from
// the last-level cache or HBM, so the reads' latency sets the pace.  The tiny MLP's weights are read with
// wave-uniform indices (scalar loads, operands of the vector multiply-adds).
#include "common.h"
#include "kernels.h"

namespace fl {

namespace gm {
constexpr int H = 64, GEO = 16;
}  // namespace gm

__device__ __forceinline__ float gm_softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float gm_sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// gamma_LD(d) in canonical order (d, sin 2^0 pi d, cos 2^0 pi d, ...): band 0
// from sincospif, band b + 1 from band b by the double-angle identities (each
// doubling at most doubles the absolute error: a few float32 roundings for
// LD <= 4)
template <int LD>
__device__ __forceinline__ void gm_dir_encoding(const float4 d, float (&gd)[3 + 6 * LD]) {
  const float v[3] = {d.x, d.y, d.z};
  gd[0] = d.x;
  gd[1] = d.y;
  gd[2] = d.z;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float sn, cs;
    sincospif(v[c], &sn, &cs);
#pragma unroll
    for (int l = 0; l < LD; ++l) {
      gd[3 + 6 * l + c] = sn;
      gd[3 + 6 * l + 3 + c] = cs;
      const float s2 = 2.0f * sn * cs, c2 = (cs - sn) * (cs + sn);
      sn = s2;
      cs = c2;
    }
  }
}

// Two waves per SIMD (measured on gfx950): the gather of all levels is
// unrolled so that a wave keeps up to 8 L table reads in flight, which needs
// about 250 registers; fewer reads in flight at three or four waves per SIMD
// (the features folded into the first layer level by level) ran 15-30% slower.
#ifndef FL_GRID_WAVES
#define FL_GRID_WAVES 2
#endif

template <int L, int LD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FL_GRID_WAVES))) void k_grid_map(
    const GridDev g, const MlpArgs a) {
  // the tiny MLP, flat canonical order: every index below is the same for all
  // lanes, so the weights arrive through scalar loads as instruction operands
  const float* __restrict__ w = g.mlp;
  const long n_tot = a.n_samples + a.n_samples2;
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_tot) return;
  const bool second = s >= a.n_samples;
  const long sl = second ? s - a.n_samples : s;
  const int spr = second ? a.spr2 : a.spr;
  const int ray = (int)(sl / spr);
  const int k = (int)(sl - (long)ray * spr);
  const float4 o = a.ray_o[ray];
  const float4 d = a.ray_d[ray];
  float t;
  if (second) {
    t = a.t_in2[sl];
  } else if (a.t_in) {
    t = a.t_in[sl];
  } else {
    float xi = 0.0f;
    if (a.jitter) {
      const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
      xi = unit24(pick(draw(a.seed, a.iter, kStreamJitCoarse, i, j, k >> 2), k & 3));
    }
    t = a.near_ + ((float)k + xi) * a.dt;
    a.t_out[sl] = t;
  }
  const float x0 = fmaf(t, d.x, o.x), x1 = fmaf(t, d.y, o.y), x2 = fmaf(t, d.z, o.z);
  const float inv = 1.0f / (2.0f * g.bound);
  float u0 = (x0 + g.bound) * inv, u1 = (x1 + g.bound) * inv, u2 = (x2 + g.bound) * inv;
  const bool inside = u0 >= 0.0f && u0 <= 1.0f && u1 >= 0.0f && u1 <= 1.0f && u2 >= 0.0f && u2 <= 1.0f;
  u0 = fminf(fmaxf(u0, 0.0f), 1.0f);
  u1 = fminf(fmaxf(u1, 0.0f), 1.0f);
  u2 = fminf(fmaxf(u2, 0.0f), 1.0f);
  // offsets of the tiny MLP in its flat canonical order
  constexpr int NF = 2 * L;
  const int o_b1 = gm::H * NF, o_w2 = o_b1 + gm::H, o_b2 = o_w2 + gm::GEO * gm::H, o_w3 = o_b2 + gm::GEO;
  constexpr int ID = 3 + 6 * LD;
  constexpr int in3 = gm::GEO + ID;
  const int o_b3 = o_w3 + gm::H * in3, o_w4 = o_b3 + gm::H, o_b4 = o_w4 + 3 * gm::H;
  // encoding: all levels' features first (many table reads in flight), then the layers
  float f[NF];
  const uint32_t tmask = (1u << g.log2_table) - 1u;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const int N = g.res[l];
    const float p0 = u0 * (float)N, p1 = u1 * (float)N, p2 = u2 * (float)N;
    const int c0 = min((int)floorf(p0), N - 1), c1 = min((int)floorf(p1), N - 1), c2 = min((int)floorf(p2), N - 1);
    const float w0 = p0 - (float)c0, w1 = p1 - (float)c1, w2 = p2 - (float)c2;
    const uint32_t* tab = g.tables + ((long)l << g.log2_table);
    const bool dense = (g.dense_mask >> l) & 1u;
    const uint32_t n1 = (uint32_t)N + 1u;
    float fa = 0.0f, fb = 0.0f;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
      const uint32_t a0 = (uint32_t)(c0 + (corner & 1)), a1 = (uint32_t)(c1 + ((corner >> 1) & 1)),
                     a2 = (uint32_t)(c2 + ((corner >> 2) & 1));
      const uint32_t idx = dense ? a0 + n1 * (a1 + n1 * a2) : ((a0 * 1u) ^ (a1 * 2654435761u) ^ (a2 * 805459861u)) & tmask;
      const float wt = ((corner & 1) ? w0 : 1.0f - w0) * (((corner >> 1) & 1) ? w1 : 1.0f - w1) *
                       (((corner >> 2) & 1) ? w2 : 1.0f - w2);
      const uint32_t e = tab[idx];
      fa = fmaf(wt, (float)__builtin_bit_cast(_Float16, (uint16_t)(e & 0xffffu)), fa);
      fb = fmaf(wt, (float)__builtin_bit_cast(_Float16, (uint16_t)(e >> 16)), fb);
    }
    f[2 * l] = fa;
    f[2 * l + 1] = fb;
  }
  float h1[gm::H];
#pragma unroll
  for (int j = 0; j < gm::H; ++j) {
    float hj = w[o_b1 + j];
#pragma unroll
    for (int q = 0; q < NF; ++q) hj = fmaf(w[j * NF + q], f[q], hj);
    h1[j] = hj;
  }
  // tiny MLP (weights in LDS, offsets of the flat canonical order)
  float z[gm::GEO];
#pragma unroll
  for (int q = 0; q < gm::GEO; ++q) z[q] = w[o_b2 + q];
#pragma unroll
  for (int j = 0; j < gm::H; ++j) {
    const float hj = fmaxf(h1[j], 0.0f);
#pragma unroll
    for (int q = 0; q < gm::GEO; ++q) z[q] = fmaf(w[o_w2 + q * gm::H + j], hj, z[q]);
  }
  float gd[ID];
  gm_dir_encoding<LD>(d, gd);
  float r0 = w[o_b4], r1 = w[o_b4 + 1], r2 = w[o_b4 + 2];
  for (int j = 0; j < gm::H; ++j) {
    const float* row = w + o_w3 + j * in3;
    float hj = w[o_b3 + j];
#pragma unroll
    for (int q = 0; q < gm::GEO; ++q) hj = fmaf(row[q], z[q], hj);
#pragma unroll
    for (int q = 0; q < ID; ++q) hj = fmaf(row[gm::GEO + q], gd[q], hj);
    hj = fmaxf(hj, 0.0f);
    r0 = fmaf(w[o_w4 + j], hj, r0);
    r1 = fmaf(w[o_w4 + gm::H + j], hj, r1);
    r2 = fmaf(w[o_w4 + 2 * gm::H + j], hj, r2);
  }
  float4 res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (inside) res = make_float4(gm_softplus(z[0]), gm_sigmoid(r0), gm_sigmoid(r1), gm_sigmoid(r2));
  (second ? a.out2 : a.out)[sl] = res;
}

template <int L, int LD>
hipError_t launch_grid_t(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  const long n = a.n_samples + a.n_samples2;
  hipLaunchKernelGGL((k_grid_map<L, LD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, a);
  return hipGetLastError();
}

template <int L>
hipError_t launch_grid_l(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  switch (g.in_d) {
    case 3 + 6 * 2: return launch_grid_t<L, 2>(g, a, st);
    case 3 + 6 * 4: return launch_grid_t<L, 4>(g, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid_map(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  if (a.n_samples + a.n_samples2 <= 0) return hipSuccess;
  switch (g.levels) {
    case 4: return launch_grid_l<4>(g, a, st);
    case 8: return launch_grid_l<8>(g, a, st);
    case 16: return launch_grid_l<16>(g, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fl
