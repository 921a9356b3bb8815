// FP32 map evaluation on MFMA (v_mfma_f32_16x16x4_f32) with register-chained
// activations: positional encoding (gamma), the ReLU MLP, the density head
// (softplus) and the colour head (sigmoid) for a batch of ray samples.
//
// One wave evaluates 16 samples.  Each layer is D^T (out x 16) = W (out x in)
// X^T (in x 16); the accumulator layout of one layer is the operand layout of
// the next (see maplayout.h), so the only memory traffic per sample is the ray
// (o, d), the sample depth t, and the 16-byte (sigma, r, g, b) result.  Weight
// fragments stream from L2 through L1; the waves of a workgroup walk the same
// weights in step.
#include "common.h"
#include "maplayout.h"
#include "kernels.h"

namespace fl {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// gamma(p) for lane group g in the k-block order of maplayout.h
template <int L, int KB>
__device__ __forceinline__ void posenc_f32(const float p0, const float p1, const float p2,
                                           const int g, float (&out)[KB]) {
  constexpr int NP = 3 * L + 2;
#pragma unroll
  for (int q = 0; q < KB / 2; ++q) {
    const int p = 4 * q + g;
    float a = 0.0f, b = 0.0f;
    if (p < 3 * L) {
      const int c = p % 3;
      const float x = c == 0 ? p0 : (c == 1 ? p1 : p2);
      sincospif(ldexpf(x, p / 3), &a, &b);
    } else if (p == 3 * L) {
      a = p0; b = p1;
    } else if (p < NP) {
      a = p2;
    }
    out[2 * q] = a;
    out[2 * q + 1] = b;
  }
}

// y[4 mt + r] = act(b + W [x1, x2]) for MTO output m-tiles.  x2 joins the
// input only when use2 (a uniform runtime flag); act(z) = max(z, lo) with
// lo = 0 (ReLU) or -inf (linear).
template <int MTO, int KB1, int KB2, int NY>
__device__ __forceinline__ void dense_f32(const float* __restrict__ Wp,
                                          const float (&x1)[KB1], const float (&x2)[KB2],
                                          const bool use2, const float lo, float (&y)[NY],
                                          const int lane) {
  static_assert(KB1 % 4 == 0 && KB2 % 4 == 0 && 4 * MTO <= NY, "layout");
  const int kb_row = KB1 + (use2 ? KB2 : 0);
  const int g = lane >> 4;
  const float4* __restrict__ W4 = reinterpret_cast<const float4*>(Wp) + lane;
  const float4* __restrict__ B4 = reinterpret_cast<const float4*>(Wp + (long)MTO * kb_row * 64) + g;
#pragma unroll
  for (int mt = 0; mt < MTO; ++mt) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const float4* __restrict__ Wm = W4 + (long)mt * (kb_row / 4) * 64;
#pragma unroll
    for (int q = 0; q < KB1 / 4; ++q) {
      const float4 a = Wm[q * 64];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x1[4 * q + 0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x1[4 * q + 1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, x1[4 * q + 2], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, x1[4 * q + 3], acc, 0, 0, 0);
    }
    if (use2) {
#pragma unroll
      for (int q = 0; q < KB2 / 4; ++q) {
        const float4 a = Wm[(KB1 / 4 + q) * 64];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x2[4 * q + 0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x2[4 * q + 1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, x2[4 * q + 2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, x2[4 * q + 3], acc, 0, 0, 0);
      }
    }
    const float4 b = B4[mt * 4];
    y[4 * mt + 0] = fmaxf(acc[0] + b.x, lo);
    y[4 * mt + 1] = fmaxf(acc[1] + b.y, lo);
    y[4 * mt + 2] = fmaxf(acc[2] + b.z, lo);
    y[4 * mt + 3] = fmaxf(acc[3] + b.w, lo);
  }
}

template <int KB, int N>
__device__ __forceinline__ float dot_part(const float* __restrict__ w, const float (&x)[N]) {
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < KB; ++k) s = fmaf(w[k], x[k], s);
  return s;
}

__device__ __forceinline__ float softplus_f(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoid_f(float z) { return 1.0f / (1.0f + expf(-z)); }

template <class S>
__global__ __launch_bounds__(256) void k_mlp_f32(const MlpArgs a) {
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const long blk = flat_block();
  if (blk * 64 >= a.n_samples) return;   // whole workgroup
  const long tile = blk * 4 + (threadIdx.x >> 6);
  const long s = tile * 16 + n;
  const bool valid = s < a.n_samples;
  const long sc = valid ? s : a.n_samples - 1;
  const int ray = (int)(sc / a.spr);
  const int k = (int)(sc - (long)ray * a.spr);
  const float4 o = a.ray_o[ray];
  const float4 d = a.ray_d[ray];
  float t;
  if (a.t_in) {
    t = a.t_in[sc];
  } else {
    float xi = 0.0f;
    if (a.jitter) {
      const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
      xi = unit24(pick(draw(a.seed, a.iter, kStreamJitCoarse, i, j, k >> 2), k & 3));
    }
    t = a.near_ + ((float)k + xi) * a.dt;
    if (valid && g == 0) a.t_out[s] = t;
  }
  const float px = fmaf(t, d.x, o.x), py = fmaf(t, d.y, o.y), pz = fmaf(t, d.z, o.z);

  float gx[S::KBX], gd[S::KBD];
  posenc_f32<S::LX>(px, py, pz, g, gx);
  posenc_f32<S::LD>(d.x, d.y, d.z, g, gd);

  const float* __restrict__ P = a.weights;
  float xa[S::KBH], xb[S::KBH];
  dense_f32<S::MT, S::KBX, S::KBD, S::KBH>(P + S::layer_off(0), gx, gd, false, 0.0f, xa, lane);
#pragma unroll 1
  for (int l = 1; l < S::D; ++l) {
    const bool skip = (l == S::SKIP);
    const long off = skip ? S::layer_off(S::SKIP) : S::layer_off(l);
    dense_f32<S::MT, S::KBH, S::KBX, S::KBH>(P + off, xa, gx, skip, 0.0f, xb, lane);
#pragma unroll
    for (int i = 0; i < S::KBH; ++i) xa[i] = xb[i];
  }
  // density head: each lane group holds a quarter of the features of its sample
  const float* sw = P + S::SIG_OFF;
  float zs = dot_part<S::KBH>(sw + g * S::KBH, xa);
  zs += __shfl_xor(zs, 16, 64);
  zs += __shfl_xor(zs, 32, 64);
  const float sigma = softplus_f(zs + sw[4 * S::KBH]);

  float rgb[3];
  const float* cw = P + S::RGB_OFF;
  if constexpr (S::DW > 0) {
    dense_f32<S::MT, S::KBH, S::KBD, S::KBH>(P + S::FEAT_OFF, xa, gd, false, -INFINITY, xb, lane);
    dense_f32<S::MTD, S::KBH, S::KBD, S::KBH>(P + S::DIR_OFF, xb, gd, true, 0.0f, xa, lane);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float z = dot_part<S::KBG>(cw + (4 * c + g) * S::KBG, xa);
      z += __shfl_xor(z, 16, 64);
      z += __shfl_xor(z, 32, 64);
      rgb[c] = sigmoid_f(z + cw[12 * S::KBG + c]);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* w = cw + (4 * c + g) * S::KBG;
      float z = dot_part<S::KBH>(w, xa);
      float z2 = 0.0f;
#pragma unroll
      for (int q = 0; q < S::KBD; ++q) z2 = fmaf(w[S::KBH + q], gd[q], z2);
      z += z2;
      z += __shfl_xor(z, 16, 64);
      z += __shfl_xor(z, 32, 64);
      rgb[c] = sigmoid_f(z + cw[12 * S::KBG + c]);
    }
  }
  if (valid && g == 0) a.out[s] = make_float4(sigma, rgb[0], rgb[1], rgb[2]);
}

template <class S>
hipError_t launch_mlp_f32(const MlpArgs& a, hipStream_t st) {
  const long tiles = (a.n_samples + 15) / 16;
  const long blocks = (tiles + 3) / 4;
  hipLaunchKernelGGL(k_mlp_f32<S>, folded_grid(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp(int map_kind, const MlpArgs& a, hipStream_t st) {
  if (a.n_samples <= 0) return hipSuccess;
  if (map_kind == kMapSmall) return launch_mlp_f32<SmallMap>(a, st);
  return launch_mlp_f32<NerfMap>(a, st);
}

}  // namespace fl
