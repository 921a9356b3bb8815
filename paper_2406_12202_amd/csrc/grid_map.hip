// Multi-resolution grid map (the map type of Sec. IV-B, restated as a
// multiresolution hash encoding with a tiny MLP): per sample, L levels of
// trilinear blends of two-feature table entries at the 8 cell corners (dense
// index while the level's vertices fit the table, the spatial hash of three
// primes otherwise), then z = W2 relu(W1 f + b1) + b2, sigma = softplus(z_0),
// rgb = sigmoid(W4 relu(W3 [z, gamma(d)] + b3) + b4).  Points outside the
// box [-bound, bound]^3 are empty.
//
// Same sample sets and stratified placement as the MLP kernels (MlpArgs).
// The tables hold half-precision feature pairs (one 32-bit word per entry).
// Three passes over a chunk of at most feat_cap samples:
//   depths   coarse stratified depths written once (when not given);
//   encode   one thread per (sample, level), launched level-major (grid.y is
//            the level, so the blocks in flight read one level's table, 2 MB
//            at 2^19 entries, which stays in every XCD's L2), the 8 corner
//            reads and the blend, float32 features to the workspace;
//   mlp      one thread per sample: features from the workspace, the tiny
//            MLP with its weights read at wave-uniform indices (scalar loads).
// The arithmetic per sample is the fused single-pass kernel's, so results do
// not depend on the chunking.
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

// depth of sample sl of the pass's sample set
__device__ __forceinline__ float grid_sample_t(const MlpArgs& a, const bool second, const long sl) {
  return second ? a.t_in2[sl] : (a.t_in ? a.t_in[sl] : a.t_out[sl]);
}

__global__ __launch_bounds__(256) void k_grid_depths(const MlpArgs a) {
  const long sl = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= a.n_samples) return;
  const int ray = (int)(sl / a.spr);
  const int k = (int)(sl - (long)ray * a.spr);
  float xi = 0.0f;
  if (a.jitter) {
    const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
    xi = unit24(pick(draw(a.seed, a.iter, kStreamJitCoarse, i, j, k >> 2), k & 3));
  }
  a.t_out[sl] = a.near_ + ((float)k + xi) * a.dt;
}

// position of sample s (of both sets) in the box's unit cube, and whether it
// lies inside the box
struct GridPoint {
  float u0, u1, u2;
  bool inside, second;
  long sl;
  int ray;
};

__device__ __forceinline__ GridPoint grid_point(const GridDev& g, const MlpArgs& a, const long s) {
  GridPoint p;
  p.second = s >= a.n_samples;
  p.sl = p.second ? s - a.n_samples : s;
  const int spr = p.second ? a.spr2 : a.spr;
  p.ray = (int)(p.sl / spr);
  const float4 o = a.ray_o[p.ray];
  const float4 d = a.ray_d[p.ray];
  const float t = grid_sample_t(a, p.second, p.sl);
  const float x0 = fmaf(t, d.x, o.x), x1 = fmaf(t, d.y, o.y), x2 = fmaf(t, d.z, o.z);
  const float inv = 1.0f / (2.0f * g.bound);
  float u0 = (x0 + g.bound) * inv, u1 = (x1 + g.bound) * inv, u2 = (x2 + g.bound) * inv;
  p.inside = u0 >= 0.0f && u0 <= 1.0f && u1 >= 0.0f && u1 <= 1.0f && u2 >= 0.0f && u2 <= 1.0f;
  p.u0 = fminf(fmaxf(u0, 0.0f), 1.0f);
  p.u1 = fminf(fmaxf(u1, 0.0f), 1.0f);
  p.u2 = fminf(fmaxf(u2, 0.0f), 1.0f);
  return p;
}

// samples c0 .. c0 + n - 1, level blockIdx.y
__global__ __launch_bounds__(256) void k_grid_encode(const GridDev g, const MlpArgs a, const long c0, const long n) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int l = blockIdx.y;
  const GridPoint p = grid_point(g, a, c0 + q);
  const int N = g.res[l];
  const float p0 = p.u0 * (float)N, p1 = p.u1 * (float)N, p2 = p.u2 * (float)N;
  const int c0i = min((int)floorf(p0), N - 1), c1i = min((int)floorf(p1), N - 1), c2i = min((int)floorf(p2), N - 1);
  const float w0 = p0 - (float)c0i, w1 = p1 - (float)c1i, w2 = p2 - (float)c2i;
  const uint32_t* tab = g.tables + ((long)l << g.log2_table);
  const bool dense = (g.dense_mask >> l) & 1u;
  const uint32_t n1 = (uint32_t)N + 1u;
  const uint32_t tmask = (1u << g.log2_table) - 1u;
  uint32_t e[8];
  float wt[8];
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const uint32_t a0 = (uint32_t)(c0i + (corner & 1)), a1 = (uint32_t)(c1i + ((corner >> 1) & 1)),
                   a2 = (uint32_t)(c2i + ((corner >> 2) & 1));
    const uint32_t idx = dense ? a0 + n1 * (a1 + n1 * a2) : ((a0 * 1u) ^ (a1 * 2654435761u) ^ (a2 * 805459861u)) & tmask;
    wt[corner] = ((corner & 1) ? w0 : 1.0f - w0) * (((corner >> 1) & 1) ? w1 : 1.0f - w1) *
                 (((corner >> 2) & 1) ? w2 : 1.0f - w2);
    e[corner] = tab[idx];
  }
  float fa = 0.0f, fb = 0.0f;
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    fa = fmaf(wt[corner], (float)__builtin_bit_cast(_Float16, (uint16_t)(e[corner] & 0xffffu)), fa);
    fb = fmaf(wt[corner], (float)__builtin_bit_cast(_Float16, (uint16_t)(e[corner] >> 16)), fb);
  }
  g.feat[(long)l * g.feat_cap + q] = make_float2(fa, fb);
}

template <int L, int LD>
__global__ __launch_bounds__(256) void k_grid_mlp(const GridDev g, const MlpArgs a, const long c0, const long n) {
  // the tiny MLP, flat canonical order: every index below is the same for all
  // lanes, so the weights arrive through scalar loads as instruction operands
  const float* __restrict__ w = g.mlp;
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const GridPoint p = grid_point(g, a, c0 + q);
  const float4 d = a.ray_d[p.ray];
  constexpr int NF = 2 * L;
  const int o_b1 = gm::H * NF, o_w2 = o_b1 + gm::H, o_b2 = o_w2 + gm::GEO * gm::H, o_w3 = o_b2 + gm::GEO;
  constexpr int ID = 3 + 6 * LD;
  constexpr int in3 = gm::GEO + ID;
  const int o_b3 = o_w3 + gm::H * in3, o_w4 = o_b3 + gm::H, o_b4 = o_w4 + 3 * gm::H;
  float f[NF];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const float2 v = g.feat[(long)l * g.feat_cap + q];
    f[2 * l] = v.x;
    f[2 * l + 1] = v.y;
  }
  float h1[gm::H];
#pragma unroll
  for (int j = 0; j < gm::H; ++j) {
    float hj = w[o_b1 + j];
#pragma unroll
    for (int k = 0; k < NF; ++k) hj = fmaf(w[j * NF + k], f[k], hj);
    h1[j] = hj;
  }
  float z[gm::GEO];
#pragma unroll
  for (int k = 0; k < gm::GEO; ++k) z[k] = w[o_b2 + k];
#pragma unroll
  for (int j = 0; j < gm::H; ++j) {
    const float hj = fmaxf(h1[j], 0.0f);
#pragma unroll
    for (int k = 0; k < gm::GEO; ++k) z[k] = fmaf(w[o_w2 + k * gm::H + j], hj, z[k]);
  }
  float gd[ID];
  gm_dir_encoding<LD>(d, gd);
  float r0 = w[o_b4], r1 = w[o_b4 + 1], r2 = w[o_b4 + 2];
  for (int j = 0; j < gm::H; ++j) {
    const float* row = w + o_w3 + j * in3;
    float hj = w[o_b3 + j];
#pragma unroll
    for (int k = 0; k < gm::GEO; ++k) hj = fmaf(row[k], z[k], hj);
#pragma unroll
    for (int k = 0; k < ID; ++k) hj = fmaf(row[gm::GEO + k], gd[k], hj);
    hj = fmaxf(hj, 0.0f);
    r0 = fmaf(w[o_w4 + j], hj, r0);
    r1 = fmaf(w[o_w4 + gm::H + j], hj, r1);
    r2 = fmaf(w[o_w4 + 2 * gm::H + j], hj, r2);
  }
  float4 res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (p.inside) res = make_float4(gm_softplus(z[0]), gm_sigmoid(r0), gm_sigmoid(r1), gm_sigmoid(r2));
  (p.second ? a.out2 : a.out)[p.sl] = res;
}

template <int L, int LD>
hipError_t launch_grid_t(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  const long n_tot = a.n_samples + a.n_samples2;
  if (!a.t_in && a.n_samples > 0) {
    hipLaunchKernelGGL(k_grid_depths, dim3((unsigned)((a.n_samples + 255) / 256)), dim3(256), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (long c0 = 0; c0 < n_tot; c0 += g.feat_cap) {
    const long n = n_tot - c0 < g.feat_cap ? n_tot - c0 : g.feat_cap;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_grid_encode, dim3(nb, L), dim3(256), 0, st, g, a, c0, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_grid_mlp<L, LD>), dim3(nb), dim3(256), 0, st, g, a, c0, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
  if (!g.feat || g.feat_cap <= 0) return hipErrorInvalidValue;
  switch (g.levels) {
    case 4: return launch_grid_l<4>(g, a, st);
    case 8: return launch_grid_l<8>(g, a, st);
    case 16: return launch_grid_l<16>(g, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fl
