// Pieces shared by the MFMA map kernels with LDS-streamed weights (BF16 and
// FP8 paths): operand vector types, the bf16 positional-encoding operands,
// direct global->LDS weight streaming, and the per-tile sample set-up.
#pragma once

#include <type_traits>
#include <utility>

#include "common.h"
#include "kernels.h"

namespace fl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void_t;

// compile-time loop: fn(std::integral_constant<int, i>) for i = 0 .. N-1,
// each call inlined with i a constant (register arrays stay registers)
template <class Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn& fn, std::integer_sequence<int, I...>) {
  (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  static_for_impl(fn, std::make_integer_sequence<int, N>{});
}

// sin(pi x) and cos(pi x) for band 0 of the encoding: x = j / 2 + r with
// j = rint(2 x) and |r| <= 1/4 (r is exact in float32), sin(pi r) and
// cos(pi r) by polynomials in r^2 fitted on [0, 1/4] toward the minimax
// error (odd terms to r^9, even to r^10), then the j quarter turns:
// sin(pi x) = +-sin(pi r) or +-cos(pi r) by j mod 4.  Largest absolute
// error 8.4e-8 on |x| <= 12 (float32 arithmetic against exact values);
// positions are finite and small, so the long-argument reduction of a
// library sincospi is not needed.
__device__ __forceinline__ void sincospi_enc(const float x, float& s, float& c) {
  const float j = __builtin_rintf(x + x);
  const float r = fmaf(j, -0.5f, x);
  const float z = r * r;
  float ps = fmaf(z, 0x1.3e17e8p-4f, -0x1.32535cp-1f);
  ps = fmaf(z, ps, 0x1.4668f2p+1f);
  ps = fmaf(z, ps, -0x1.4abbc4p+2f);
  ps = fmaf(z, ps, 0x1.921fb6p+1f);
  const float sr = r * ps;
  float pc = fmaf(z, -0x1.901bd6p-6f, 0x1.e12f86p-3f);
  pc = fmaf(z, pc, -0x1.55d0b8p+0f);
  pc = fmaf(z, pc, 0x1.03c1e6p+2f);
  pc = fmaf(z, pc, -0x1.3bd3ccp+2f);
  const float cr = fmaf(z, pc, 1.0f);
  const int q = (int)j;
  const float a = (q & 1) ? cr : sr;
  const float b = (q & 1) ? sr : cr;
  s = __int_as_float(__float_as_int(a) ^ ((q & 2) << 30));
  c = __int_as_float(__float_as_int(b) ^ (((q + 1) & 2) << 30));
}

// bf16 operands of the encoding gamma(p) (pseudo-pair layout of
// maplayout_bf16.h).  sin and cos of band 0 come from sincospi_enc; band
// b + 1 follows from band b by the double-angle identities
// sin 2a = 2 sin a cos a, cos 2a = (cos a - sin a)(cos a + sin a).  Each
// doubling at most doubles the absolute error, so band L - 1 is within
// 2^(L-1) float32 roundings (1e-4 for L = 10) of the exact value, far inside
// the bf16 rounding of the operands (2^-9 relative).
// values of both lane halves: out[hh][kb] is the operand of half hh
template <int L, int KB>
__device__ __forceinline__ void posenc_both(const float p0, const float p1, const float p2, bf16x8 (&out)[2][KB]) {
  float sn[3][L], cs[3][L];
  const float pc[3] = {p0, p1, p2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    sincospi_enc(pc[c], sn[c][0], cs[c][0]);
#pragma unroll
    for (int l = 1; l < L; ++l) {
      const float sa = sn[c][l - 1], ca = cs[c][l - 1];
      sn[c][l] = 2.0f * sa * ca;
      cs[c][l] = (ca - sa) * (ca + sa);
    }
  }
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      f32x8 v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = 8 * kb + 4 * hh + j;
        float a = 0.0f, b = 0.0f;
        if (p < 3 * L) {
          a = sn[p % 3][p / 3];
          b = cs[p % 3][p / 3];
        } else if (p == 3 * L) {
          a = p0; b = p1;
        } else if (p == 3 * L + 1) {
          a = p2;
        }
        v[2 * j] = a;
        v[2 * j + 1] = b;
      }
      out[hh][kb] = __builtin_convertvector(v, bf16x8);   // round to nearest even, two values per instruction
    }
}

// the operands of lane half h
template <int L, int KB>
__device__ __forceinline__ void posenc_b(const float p0, const float p1, const float p2, const int h,
                                         bf16x8 (&out)[KB]) {
  bf16x8 both[2][KB];
  posenc_both<L, KB>(p0, p1, p2, both);
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) out[kb] = h ? both[1][kb] : both[0][kb];
}

// raw buffer resource over n_bytes at p (stride 0, 32-bit data format):
// reads past n_bytes return zero
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, const int n_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, n_bytes, 0x00020000);
}

// direct loads of nkb consecutive 1 KB units into an LDS slot, wave wv
// taking units wv, wv + WAVES, ..., through the buffer path (buffer_load ...
// lds): while loads of this form are in flight the compiler still counts
// outstanding LDS reads one by one, whereas with the global form
// (global_load_lds) in flight it waits for all of them at every use
template <int WAVES>
__device__ __forceinline__ void issue_blocks_buf(const __amdgpu_buffer_rsrc_t r, const long base, const int nkb,
                                                 uint4* slot, const int wv, const int lane) {
  for (int b = wv; b < nkb; b += WAVES)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)(slot + b * 64), 16,
                                             (unsigned)(((base + b) * 64 + lane) * 16), 0, 0, 0);
}


// Sample set-up of one wave's NTL column tiles of 32 samples: depth (given, or
// stratified with jitter and written out), then gamma(x) and gamma(d) as bf16
// operands into the wave's LDS blocks laid out [column tile][k-block][lane].
// Each lane later reads back only its own entries, so no barrier is needed.
// Samples past n_samples belong to the optional second set (t_in2, out2):
// sidx is the index within the sample's set, seg2 tells which set.
template <int LX, int LD, int KBX, int KBD, int NTL>
__device__ __forceinline__ void stage_samples(const MlpArgs& a, const long tile, const int lane, uint4* gx_lds,
                                              uint4* gd_lds, long (&sidx)[NTL], bool (&valid)[NTL],
                                              bool (&seg2)[NTL]) {
  const int n = lane & 31, h = lane >> 5;
  const long n_tot = a.n_samples + a.n_samples2;
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt) {
    const long s = tile * (32 * NTL) + nt * 32 + n;
    valid[nt] = s < n_tot;
    const long sc = valid[nt] ? s : n_tot - 1;
    const bool second = sc >= a.n_samples;
    seg2[nt] = second;
    const long sl = second ? sc - a.n_samples : sc;
    sidx[nt] = sl;
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
      if (valid[nt] && h == 0) a.t_out[sl] = t;
    }
    bf16x8 gx[KBX], gd[KBD];
    posenc_b<LX>(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z), h, gx);
    posenc_b<LD>(d.x, d.y, d.z, h, gd);
#pragma unroll
    for (int kb = 0; kb < KBX; ++kb) gx_lds[(nt * KBX + kb) * 64 + lane] = __builtin_bit_cast(uint4, gx[kb]);
#pragma unroll
    for (int kb = 0; kb < KBD; ++kb) gd_lds[(nt * KBD + kb) * 64 + lane] = __builtin_bit_cast(uint4, gd[kb]);
  }
}

// two float32 values rounded to bf16 (nearest even) as one packed word, one
// conversion instruction; with relu, max with 0 on the packed int16 halves (a
// non-negative bf16 is a non-negative int16, a negative one a negative int16)
__device__ __forceinline__ uint32_t pack_bf16(const float a, const float b, const bool relu) {
  const f32x2 f = {a, b};
  s16x2 w = __builtin_bit_cast(s16x2, __builtin_convertvector(f, bf16x2));
  if (relu) {
    const s16x2 z = {0, 0};
    w = __builtin_elementwise_max(w, z);
  }
  return __builtin_bit_cast(uint32_t, w);
}

// rounded bf16 operands of the next layer from one finished output tile; the
// bias is already in the accumulators
template <int NTL, int NY>
__device__ __forceinline__ void epilogue_b(const f32x16 (&acc)[NTL], const bool relu, const int mt,
                                           bf16x8 (&y)[NTL][NY]) {
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint4 u;
      u.x = pack_bf16(acc[nt][8 * c + 0], acc[nt][8 * c + 1], relu);
      u.y = pack_bf16(acc[nt][8 * c + 2], acc[nt][8 * c + 3], relu);
      u.z = pack_bf16(acc[nt][8 * c + 4], acc[nt][8 * c + 5], relu);
      u.w = pack_bf16(acc[nt][8 * c + 6], acc[nt][8 * c + 7], relu);
      y[nt][2 * mt + c] = __builtin_bit_cast(bf16x8, u);
    }
  }
}

template <int KB, int N>
__device__ __forceinline__ float dot_b(const float* __restrict__ w, const bf16x8 (&x)[N]) {
  float s = 0.0f;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const float4* w4 = reinterpret_cast<const float4*>(w + kb * 8);
    const float4 u = w4[0], v = w4[1];
    s = fmaf(u.x, (float)x[kb][0], s); s = fmaf(u.y, (float)x[kb][1], s);
    s = fmaf(u.z, (float)x[kb][2], s); s = fmaf(u.w, (float)x[kb][3], s);
    s = fmaf(v.x, (float)x[kb][4], s); s = fmaf(v.y, (float)x[kb][5], s);
    s = fmaf(v.z, (float)x[kb][6], s); s = fmaf(v.w, (float)x[kb][7], s);
  }
  return s;
}

// Density and colour nonlinearities of the bf16 heads, on the hardware
// base-2 exponential and reciprocal (each within a few float32 ulps; the
// heads' inputs are sums of bf16 products, rounded to 2^-9 relative).
// softplus(z) = max(z, 0) + log1p(u), u = e^-|z| in (0, 1], with
// log1p(u) = 2 atanh(s), s = u / (2 + u) <= 1/3, summed as the odd series
// 2 s (1 + s^2/3 + ... + s^12/13) (next term below 2e-8 of the sum).
__device__ __forceinline__ float exp_b(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

__device__ __forceinline__ float softplus_b(float z) {
  const float u = exp_b(-fabsf(z));
  const float s = u * __builtin_amdgcn_rcpf(2.0f + u);
  const float s2 = s * s;
  float p = fmaf(s2, 1.0f / 13.0f, 1.0f / 11.0f);
  p = fmaf(s2, p, 1.0f / 9.0f);
  p = fmaf(s2, p, 1.0f / 7.0f);
  p = fmaf(s2, p, 1.0f / 5.0f);
  p = fmaf(s2, p, 1.0f / 3.0f);
  p = fmaf(s2, p, 1.0f);
  return fmaxf(z, 0.0f) + 2.0f * s * p;
}

__device__ __forceinline__ float sigmoid_b(float z) { return __builtin_amdgcn_rcpf(1.0f + exp_b(-z)); }

// both heads of a map without direction layer as one MFMA tile: acc rows 0
// (density) and 1..3 (colour) in lanes of half 0, from the head chunk w
// (KBH blocks over the trunk output x, then KBD over gamma(d) in gd_lds)
template <class S, int NTL>
__device__ __forceinline__ void head_tile(const uint4* w, const float* bl, const bf16x8 (&x)[NTL][S::KBH],
                                          const uint4* gd_lds, const int lane, f32x16 (&acc)[NTL]) {
  f32x16 binit;
  const float4* b4 = reinterpret_cast<const float4*>(bl);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 v = b4[i];
    binit[4 * i] = v.x; binit[4 * i + 1] = v.y; binit[4 * i + 2] = v.z; binit[4 * i + 3] = v.w;
  }
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt) acc[nt] = binit;
#pragma unroll
  for (int kb = 0; kb < S::KBH; ++kb) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, w[kb * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x[nt][kb], acc[nt], 0, 0, 0);
  }
#pragma unroll
  for (int kb = 0; kb < S::KBD; ++kb) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, w[(S::KBH + kb) * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      const bf16x8 bx = __builtin_bit_cast(bf16x8, gd_lds[(nt * S::KBD + kb) * 64 + lane]);
      acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[nt], 0, 0, 0);
    }
  }
}

}  // namespace fl
