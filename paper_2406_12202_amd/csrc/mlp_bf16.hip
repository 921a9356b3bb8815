// BF16 map evaluation on MFMA (v_mfma_f32_32x32x16_bf16, float32 accumulate)
// with register-chained bf16 activations and weights streamed through LDS.
//
// A workgroup is WAVES waves; each wave evaluates NTL column tiles of 32
// samples.  The packed weights are a sequence of chunks (one per layer and
// 32-row output tile, see maplayout_bf16.h); the workgroup streams MPC
// consecutive chunks at a time through two LDS slots with direct global->LDS
// loads (global_load_lds_dwordx4), prefetching the next group while all waves
// multiply the current one.  Each 16-byte weight fragment read from LDS feeds
// NTL MFMAs.  The bias enters as the accumulator input of the first MFMA of a
// tile, and ReLU runs on packed bf16 pairs after rounding, so the epilogue of a
// tile is one conversion and one packed max per pair of outputs.
#include "mfma_util.h"
#include "maplayout_bf16.h"

namespace fl {

// One MFMA layer: y = act(b + W [x1, x2]) for MTO output tiles of 32 rows.
// Chunk groups of MPC m-tiles alternate between slot0 and slot1 (every layer
// has an even number of groups, so the slot of a tile is static).  On entry
// the loads of this layer's first group are in flight.  x1 is a register
// array (chained activations) or, when X1_LDS, the wave's encoding block in
// LDS; x2 (the encoding segment) comes from LDS, laid out
// [column tile][k-block][lane].
template <class S, int NTL, int WAVES, int MPC, int MTO, int KB1, int KB2, int NY, bool X1_LDS, int NX1>
__device__ __forceinline__ void dense_b(const uint4* __restrict__ wb, const float* bias_lds, const int l,
                                        const bool use2, const bool relu, uint4* slot0, uint4* slot1,
                                        const bf16x8 (&x1)[NTL][NX1], const uint4* x1s, const uint4* x2s,
                                        bf16x8 (&y)[NTL][NY], const int wv, const int lane) {
  static_assert(MTO % (2 * MPC) == 0 && 2 * MTO <= NY && (X1_LDS || KB1 <= NX1), "layout");
  const int h = lane >> 5;
  const int kb_tot = KB1 + (use2 ? KB2 : 0);
  const long base = S::block_base(l);
  const float* bl = bias_lds + S::bias_base(l) + h * 16;
#pragma unroll
  for (int mt = 0; mt < MTO; ++mt) {
    uint4* grp = ((mt / MPC) & 1) ? slot1 : slot0;
    if (mt % MPC == 0) {
      uint4* nxt = ((mt / MPC) & 1) ? slot0 : slot1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (mt + MPC < MTO)
        issue_blocks<WAVES>(wb, base + (long)(mt + MPC) * kb_tot, MPC * kb_tot, nxt, wv, lane);
      else if (l + 1 < S::NL)
        issue_blocks<WAVES>(wb, S::block_base(l + 1), MPC * S::layer_kb(l + 1), nxt, wv, lane);
      else if (S::HEAD_KB > 0)
        issue_blocks<WAVES>(wb, S::HEAD_BLOCK, S::HEAD_KB, nxt, wv, lane);
    }
    const uint4* cur = grp + (mt % MPC) * kb_tot * 64;
    // bias of this tile's 16 rows (lane half h), used as the accumulator input
    f32x16 binit;
    {
      const float4* b4 = reinterpret_cast<const float4*>(bl + mt * 32);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float4 v = b4[i];
        binit[4 * i] = v.x; binit[4 * i + 1] = v.y; binit[4 * i + 2] = v.z; binit[4 * i + 3] = v.w;
      }
    }
    f32x16 acc[NTL];
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) acc[nt] = binit;
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, cur[kb * 64 + lane]);
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        bf16x8 bx;
        if constexpr (X1_LDS) bx = __builtin_bit_cast(bf16x8, x1s[(nt * KB1 + kb) * 64 + lane]);
        else bx = x1[nt][kb];
        acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[nt], 0, 0, 0);
      }
    }
    if (use2) {
      const int kb1 = X1_LDS ? 0 : KB1;
#pragma unroll
      for (int kb = 0; kb < KB2; ++kb) {
        const bf16x8 a = __builtin_bit_cast(bf16x8, cur[(kb1 + kb) * 64 + lane]);
#pragma unroll
        for (int nt = 0; nt < NTL; ++nt) {
          const bf16x8 bx = __builtin_bit_cast(bf16x8, x2s[(nt * KB2 + kb) * 64 + lane]);
          acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[nt], 0, 0, 0);
        }
      }
    }
    epilogue_b<NTL>(acc, relu, mt, y);
  }
}

template <class S, int NTL, int WAVES, int MPC>
struct BCfg {
  static constexpr int SLOT_KB = MPC * S::MAX_KB;   // 1 KB blocks per LDS slot
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int SAMPLES = 32 * NTL * WAVES;  // per workgroup
};

template <class S, int NTL, int WAVES, int MPC>
__global__ __launch_bounds__(64 * WAVES) void k_mlp_bf16(const MlpArgs a) {
  using C = BCfg<S, NTL, WAVES, MPC>;
  __shared__ uint4 slot0[C::SLOT_KB * 64];
  __shared__ uint4 slot1[C::SLOT_KB * 64];
  __shared__ uint4 s_gx[WAVES][NTL * S::KBX * 64];   // per wave: [column tile][k-block][lane]
  __shared__ uint4 s_gd[WAVES][NTL * S::KBD * 64];
  __shared__ float4 s_bias[S::BIASES / 4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const uint4* __restrict__ wb = reinterpret_cast<const uint4*>(a.wblocks);
  // weights of layer 0's first chunk group start loading while the inputs
  // are encoded; biases go to LDS (visible after the first barrier)
  issue_blocks<WAVES>(wb, 0, MPC * S::layer_kb(0), slot0, wv, lane);
  for (int i = threadIdx.x; i < S::BIASES / 4; i += C::THREADS)
    s_bias[i] = reinterpret_cast<const float4*>(a.bias)[i];

  const long tile = (long)blockIdx.x * WAVES + wv;
  long sidx[NTL];
  bool valid[NTL];
  stage_samples<S::LX, S::LD, S::KBX, S::KBD, NTL>(a, tile, lane, s_gx[wv], s_gd[wv], sidx, valid);

  const float* bias = reinterpret_cast<const float*>(s_bias);
  bf16x8 xa[NTL][S::KBH], xb[NTL][S::KBH];
  dense_b<S, NTL, WAVES, MPC, S::MT, S::KBX, S::KBD, S::KBH, true>(wb, bias, 0, false, true, slot0, slot1, xb,
                                                                  s_gx[wv], s_gd[wv], xa, wv, lane);
#pragma unroll 1
  for (int l = 1; l < S::D; ++l) {
    dense_b<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBX, S::KBH, false>(wb, bias, l, l == S::SKIP, true, slot0,
                                                                     slot1, xa, nullptr, s_gx[wv], xb, wv, lane);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
      for (int i = 0; i < S::KBH; ++i) xa[nt][i] = xb[nt][i];
  }
  float sigma[NTL], rgb[NTL][3];
  if constexpr (S::HEAD_KB > 0) {
    // both heads as one MFMA tile (rows 0: density, 1..3: colour) from the
    // chunk that follows the last layer's; it sits in slot0 (each layer has
    // an even number of chunk groups)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    f32x16 acc[NTL];
    head_tile<S, NTL>(slot0, bias + S::HEAD_BIAS + h * 16, xa, s_gd[wv], lane, acc);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      sigma[nt] = softplus_b(acc[nt][0]);
#pragma unroll
      for (int c = 0; c < 3; ++c) rgb[nt][c] = sigmoid_b(acc[nt][1 + c]);
    }
  } else {
    const float* __restrict__ hs = a.heads + S::SIG_OFF;
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      float z = dot_b<S::KBH>(hs + h * S::KBH * 8, xa[nt]);
      z += __shfl_xor(z, 32, 64);
      sigma[nt] = softplus_b(z + hs[16 * S::KBH]);
    }
    const float* __restrict__ hr = a.heads + S::RGB_OFF;
    dense_b<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBD, S::KBH, false>(wb, bias, S::D, false, false, slot0, slot1,
                                                                     xa, nullptr, s_gd[wv], xb, wv, lane);
    dense_b<S, NTL, WAVES, MPC, S::MTD, S::KBH, S::KBD, S::KBH, false>(wb, bias, S::D + 1, true, true, slot0,
                                                                      slot1, xb, nullptr, s_gd[wv], xa, wv, lane);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float z = dot_b<S::KBG>(hr + (c * 2 + h) * S::KBG * 8, xa[nt]);
        z += __shfl_xor(z, 32, 64);
        rgb[nt][c] = sigmoid_b(z + hr[48 * S::KBG + c]);
      }
  }
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt)
    if (valid[nt] && h == 0) a.out[sidx[nt]] = make_float4(sigma[nt], rgb[nt][0], rgb[nt][1], rgb[nt][2]);
}

template <class S, int NTL, int WAVES, int MPC>
hipError_t launch_mlp_bf16_t(const MlpArgs& a, hipStream_t st) {
  using C = BCfg<S, NTL, WAVES, MPC>;
  const long blocks = (a.n_samples + C::SAMPLES - 1) / C::SAMPLES;
  hipLaunchKernelGGL((k_mlp_bf16<S, NTL, WAVES, MPC>), dim3((unsigned)blocks), dim3(C::THREADS), 0, st, a);
  return hipGetLastError();
}

// Tiling (measured on MI355X, 8x256 map): one 32-sample column tile per wave
// and 8 waves per workgroup keep two waves on every SIMD (225 VGPRs), so one
// wave's epilogue, LDS latency and barrier waits overlap the other's MFMAs;
// streaming two m-tiles per chunk group halves the barriers.  1155 TFLOP/s,
// against 922 for two column tiles per wave at one wave per SIMD.
#ifndef FL_BF16_NTL
#define FL_BF16_NTL 1
#endif
#ifndef FL_BF16_WAVES
#define FL_BF16_WAVES 8
#endif
#ifndef FL_BF16_MPC
#define FL_BF16_MPC 2
#endif

hipError_t launch_mlp_bf16(int map_kind, const MlpArgs& a, hipStream_t st) {
  if (a.n_samples <= 0) return hipSuccess;
  if (map_kind == kMapSmall) return launch_mlp_bf16_t<SmallMapB, FL_BF16_NTL, FL_BF16_WAVES, 1>(a, st);
  return launch_mlp_bf16_t<NerfMapB, FL_BF16_NTL, FL_BF16_WAVES, FL_BF16_MPC>(a, st);
}

}  // namespace fl
