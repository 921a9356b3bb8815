// BF16 map evaluation on MFMA (v_mfma_f32_32x32x16_bf16, float32 accumulate)
// with register-chained bf16 activations and weights streamed through LDS.
//
// A workgroup is WAVES waves; each wave evaluates NTL column tiles of 32
// samples.  The packed weights are a sequence of chunks (one per layer and
// 32-row output tile, then the head tiles, see maplayout_bf16.h); the
// workgroup streams up to MPC consecutive chunks of one item at a time (a
// "group") through two LDS slots with direct global->LDS loads
// (global_load_lds_dwordx4), prefetching the next group while all waves
// multiply the current one; groups alternate between the slots by a running
// count.  Each 16-byte weight fragment read from LDS feeds NTL MFMAs.  The
// bias enters as the accumulator input of the first MFMA of a tile, and ReLU
// runs on packed bf16 pairs after rounding, so the epilogue of a tile is one
// conversion and one packed max per pair of outputs.  The density and colour
// heads are tiles of the same stream, evaluated on MFMA like the layers, with
// each head weight split into a high and a low bf16 part in two rows of the
// tile (the density head carries the map's density gain, so its weights keep
// 16 significant bits; the tile has rows to spare).
#include "mfma_util.h"
#include "maplayout_bf16.h"

namespace fl {

// chunk stream of one workgroup: weights, the two LDS slots, running group count
struct ChunkStream {
  const uint4* wb;
  uint4* slot0;
  uint4* slot1;
  int g;
  int wv, lane;
};

// first group of an item: (first block, 1 KB units)
struct NextGroup {
  long base;
  int units;
};

// start of the next group: wait for its loads (issued when the previous group
// started, or by the prologue), then issue the loads of the group after it
// into the other slot
template <int WAVES>
__device__ __forceinline__ const uint4* group_begin(ChunkStream& st, const NextGroup nx) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  uint4* cur = (st.g & 1) ? st.slot1 : st.slot0;
  uint4* nxt = (st.g & 1) ? st.slot0 : st.slot1;
  if (nx.units > 0) issue_blocks<WAVES>(st.wb, nx.base, nx.units, nxt, st.wv, st.lane);
  ++st.g;
  return cur;
}

// One MFMA layer: y = act(b + W [x1, x2]) for MTO output tiles of 32 rows,
// chunks of kb_tot blocks from `base`; `after` is the first group of the
// item that follows.  x1 is a register array (chained activations) or, when
// X1_LDS, the wave's encoding block in LDS; x2 (the encoding segment) comes
// from LDS, laid out [column tile][k-block][lane].
template <class S, int NTL, int WAVES, int MPC, int MTO, int KB1, int KB2, int NY, bool X1_LDS, int NX1>
__device__ __forceinline__ void dense_b(ChunkStream& st, const long base, const float* bl, const bool use2,
                                        const bool relu, const NextGroup after, const bf16x8 (&x1)[NTL][NX1],
                                        const uint4* x1s, const uint4* x2s, bf16x8 (&y)[NTL][NY]) {
  static_assert(2 * MTO <= NY && (X1_LDS || KB1 <= NX1), "layout");
  const int lane = st.lane;
  const int kb_tot = KB1 + (use2 ? KB2 : 0);
  const uint4* grp = nullptr;
#pragma unroll
  for (int mt = 0; mt < MTO; ++mt) {
    if (mt % MPC == 0) {
      NextGroup nx = after;
      if (mt + MPC < MTO) {
        nx.base = base + (long)(mt + MPC) * kb_tot;
        nx.units = (MTO - mt - MPC < MPC ? MTO - mt - MPC : MPC) * kb_tot;
      }
      grp = group_begin<WAVES>(st, nx);
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
    {
      // A fragments in pairs, the next pair read while this one multiplies
      constexpr int G = 2;
      constexpr int NG = (KB1 + G - 1) / G;
      bf16x8 abuf[2][G];
#pragma unroll
      for (int kk = 0; kk < G; ++kk)
        if (kk < KB1) abuf[0][kk] = __builtin_bit_cast(bf16x8, cur[kk * 64 + lane]);
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) {
        if (gg + 1 < NG) {
#pragma unroll
          for (int kk = 0; kk < G; ++kk)
            if ((gg + 1) * G + kk < KB1)
              abuf[(gg + 1) & 1][kk] = __builtin_bit_cast(bf16x8, cur[((gg + 1) * G + kk) * 64 + lane]);
        }
#pragma unroll
        for (int kk = 0; kk < G; ++kk) {
          const int kb = gg * G + kk;
          if (kb < KB1) {
#pragma unroll
            for (int nt = 0; nt < NTL; ++nt) {
              bf16x8 bx;
              if constexpr (X1_LDS) bx = __builtin_bit_cast(bf16x8, x1s[(nt * KB1 + kb) * 64 + lane]);
              else bx = x1[nt][kb];
              acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(abuf[gg & 1][kk], bx, acc[nt], 0, 0, 0);
            }
          }
        }
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

// a head tile of the stream: acc = b + W [x, x2] (one 32-row tile, one group)
template <int NTL, int WAVES, int KB1, int KB2, int NX>
__device__ __forceinline__ void head_b(ChunkStream& st, const float* bl, const NextGroup after,
                                       const bf16x8 (&x)[NTL][NX], const uint4* x2s, f32x16 (&acc)[NTL]) {
  const uint4* cur = group_begin<WAVES>(st, after);
  const int lane = st.lane;
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
  for (int kb = 0; kb < KB1; ++kb) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, cur[kb * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x[nt][kb], acc[nt], 0, 0, 0);
  }
#pragma unroll
  for (int kb = 0; kb < KB2; ++kb) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, cur[(KB1 + kb) * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      const bf16x8 bx = __builtin_bit_cast(bf16x8, x2s[(nt * KB2 + kb) * 64 + lane]);
      acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[nt], 0, 0, 0);
    }
  }
}

template <class S, int NTL, int WAVES, int MPC>
struct BCfg {
  static constexpr int SLOT_KB = MPC * S::MAX_KB;   // 1 KB blocks per LDS slot
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int SAMPLES = 32 * NTL * WAVES;  // per workgroup
};

// first group of layer l (execution order)
template <class S, int MPC>
__device__ __forceinline__ NextGroup first_group(const int l) {
  const int mt = S::layer_mt(l) < MPC ? S::layer_mt(l) : MPC;
  return NextGroup{S::block_base(l), mt * S::layer_kb(l)};
}

template <class S, int NTL, int WAVES, int MPC>
__global__ __launch_bounds__(64 * WAVES) void k_mlp_bf16(const MlpArgs a) {
  using C = BCfg<S, NTL, WAVES, MPC>;
  const long blk = flat_block();
  if (blk * C::SAMPLES >= a.n_samples + a.n_samples2) return;   // whole workgroup, before any barrier
  __shared__ uint4 slot0[C::SLOT_KB * 64];
  __shared__ uint4 slot1[C::SLOT_KB * 64];
  __shared__ uint4 s_gx[WAVES][NTL * S::KBX * 64];   // per wave: [column tile][k-block][lane]
  __shared__ uint4 s_gd[WAVES][NTL * S::KBD * 64];
  __shared__ float4 s_bias[S::BIASES / 4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5;
  ChunkStream st{reinterpret_cast<const uint4*>(a.wblocks), slot0, slot1, 0, wv, lane};
  // weights of layer 0's first chunk group start loading while the inputs
  // are encoded; biases go to LDS (visible after the first barrier)
  {
    const NextGroup g0 = first_group<S, MPC>(0);
    issue_blocks<WAVES>(st.wb, g0.base, g0.units, slot0, wv, lane);
  }
  for (int i = threadIdx.x; i < S::BIASES / 4; i += C::THREADS)
    s_bias[i] = reinterpret_cast<const float4*>(a.bias)[i];

  const long tile = blk * WAVES + wv;
  long sidx[NTL];
  bool valid[NTL], seg2[NTL];
  stage_samples<S::LX, S::LD, S::KBX, S::KBD, NTL>(a, tile, lane, s_gx[wv], s_gd[wv], sidx, valid, seg2);

  const float* bias = reinterpret_cast<const float*>(s_bias);
  const NextGroup sig_group{S::SIG_BLOCK, S::SIG_KB};
  bf16x8 xa[NTL][S::KBH], xb[NTL][S::KBH];
  dense_b<S, NTL, WAVES, MPC, S::MT, S::KBX, S::KBD, S::KBH, true>(
      st, S::block_base(0), bias + S::bias_base(0) + h * 16, false, true,
      S::D > 1 ? first_group<S, MPC>(1) : sig_group, xb, s_gx[wv], s_gd[wv], xa);
  // hidden layers 1 .. D-1, ping-ponging between xa and xb; the result ends
  // in xa (a final copy when D - 1 is odd)
#pragma unroll 1
  for (int l = 1; l < S::D; l += 2) {
    dense_b<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBX, S::KBH, false>(
        st, S::block_base(l), bias + S::bias_base(l) + h * 16, l == S::SKIP, true,
        l + 1 < S::D ? first_group<S, MPC>(l + 1) : sig_group, xa, nullptr, s_gx[wv], xb);
    if (l + 1 < S::D)
      dense_b<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBX, S::KBH, false>(
          st, S::block_base(l + 1), bias + S::bias_base(l + 1) + h * 16, l + 1 == S::SKIP, true,
          l + 2 < S::D ? first_group<S, MPC>(l + 2) : sig_group, xb, nullptr, s_gx[wv], xa);
  }
  if constexpr ((S::D - 1) % 2 == 1) {
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
      for (int i = 0; i < S::KBH; ++i) xa[nt][i] = xb[nt][i];
  }
  // heads: rows of the head tiles in lanes of half 0 (density row 0; colour
  // rows 1..3 of the single tile, or rows 0..2 of the colour tile); each
  // head weight is a pair of bf16 numbers whose low parts sit 8 rows further
  // down (accumulator values v + 4), so a head output is the sum of two rows
  float sigma[NTL], rgb[NTL][3];
  f32x16 hacc[NTL];
  if constexpr (S::DW == 0) {
    head_b<NTL, WAVES, S::KBH, S::KBD>(st, bias + S::SIG_BIAS + h * 16, NextGroup{0, 0}, xa, s_gd[wv], hacc);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      sigma[nt] = softplus_b(hacc[nt][0] + hacc[nt][4]);
#pragma unroll
      for (int c = 0; c < 3; ++c) rgb[nt][c] = sigmoid_b(hacc[nt][1 + c] + hacc[nt][5 + c]);
    }
  } else {
    head_b<NTL, WAVES, S::KBH, 0>(st, bias + S::SIG_BIAS + h * 16, first_group<S, MPC>(S::D), xa, nullptr, hacc);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) sigma[nt] = softplus_b(hacc[nt][0] + hacc[nt][4]);
    dense_b<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBD, S::KBH, false>(
        st, S::block_base(S::D), bias + S::bias_base(S::D) + h * 16, false, false, first_group<S, MPC>(S::D + 1),
        xa, nullptr, s_gd[wv], xb);
    dense_b<S, NTL, WAVES, MPC, S::MTD, S::KBH, S::KBD, S::KBH, false>(
        st, S::block_base(S::D + 1), bias + S::bias_base(S::D + 1) + h * 16, true, true,
        NextGroup{S::RGB_BLOCK, S::RGB_KB}, xb, nullptr, s_gd[wv], xa);
    head_b<NTL, WAVES, S::RGB_KB, 0>(st, bias + S::RGB_BIAS + h * 16, NextGroup{0, 0}, xa, nullptr, hacc);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
      for (int c = 0; c < 3; ++c) rgb[nt][c] = sigmoid_b(hacc[nt][c] + hacc[nt][4 + c]);
  }
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt)
    if (valid[nt] && h == 0)
      (seg2[nt] ? a.out2 : a.out)[sidx[nt]] = make_float4(sigma[nt], rgb[nt][0], rgb[nt][1], rgb[nt][2]);
}

template <class S, int NTL, int WAVES, int MPC>
hipError_t launch_mlp_bf16_t(const MlpArgs& a, hipStream_t st) {
  using C = BCfg<S, NTL, WAVES, MPC>;
  const long blocks = (a.n_samples + a.n_samples2 + C::SAMPLES - 1) / C::SAMPLES;
  hipLaunchKernelGGL((k_mlp_bf16<S, NTL, WAVES, MPC>), folded_grid(blocks), dim3(C::THREADS), 0, st, a);
  return hipGetLastError();
}

// Tiling (measured on MI355X, 8x256 map): one 32-sample column tile per wave
// and 8 waves per workgroup keep two waves on every SIMD, so one wave's
// epilogue, LDS latency and barrier waits overlap the other's MFMAs;
// streaming two m-tiles per chunk group halves the barriers.  Two column
// tiles per wave (one wave per SIMD) and 4-wave workgroups were slower.
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
  if (a.n_samples + a.n_samples2 <= 0) return hipSuccess;
  if (map_kind == kMapSmall) return launch_mlp_bf16_t<SmallMapB, FL_BF16_NTL, FL_BF16_WAVES, 1>(a, st);
  return launch_mlp_bf16_t<NerfMapB, FL_BF16_NTL, FL_BF16_WAVES, FL_BF16_MPC>(a, st);
}

}  // namespace fl
