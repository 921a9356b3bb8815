// BF16 map evaluation on MFMA (v_mfma_f32_32x32x16_bf16, float32 accumulate)
// with register-chained bf16 activations and weights streamed through LDS.
//
// A workgroup is WAVES waves; each wave evaluates NTL column tiles of 32
// samples.  The packed weights are a sequence of chunks (one per layer and
// 32-row output tile, then the head tiles, see maplayout_bf16.h); the
// workgroup streams up to MPC consecutive chunks of one item at a time (a
// "group") through two LDS slots with direct loads into LDS (buffer_load ...
// lds), prefetching the next group while all waves multiply the current one;
// groups alternate between the slots by a running count.  Within a group the
// A fragments are read from LDS a batch ahead of their MFMAs (dense_p).  Each
// 16-byte weight fragment read from LDS feeds NTL MFMAs.  The bias enters as
// the accumulator input of the first MFMA of a tile, and ReLU runs on packed
// bf16 pairs after rounding, so the epilogue of a tile is one conversion and
// one packed max per pair of outputs.  The density and colour heads are tiles
// of the same stream, evaluated on MFMA like the layers, with each head
// weight split into a high and a low bf16 part in two rows of the tile (the
// density head carries the map's density gain, so its weights keep 16
// significant bits; the tile has rows to spare).
#include "mfma_util.h"
#include "maplayout_bf16.h"

namespace fl {

// A fragments read ahead of their MFMAs, per batch (dense_p)
constexpr int kBf16Batch = 2;

// chunk stream of one workgroup: weights, the two LDS slots, running group count
struct ChunkStream {
  __amdgpu_buffer_rsrc_t wr;
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
// into the other slot.  The loads go through the buffer path: while loads of
// the global form (global_load_lds) are in flight the compiler waits for all
// outstanding LDS reads at every use, which undoes dense_p's read-ahead.
template <int WAVES>
__device__ __forceinline__ const uint4* group_begin(ChunkStream& st, const NextGroup nx) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  uint4* cur = (st.g & 1) ? st.slot1 : st.slot0;
  uint4* nxt = (st.g & 1) ? st.slot0 : st.slot1;
  if (nx.units > 0) issue_blocks_buf<WAVES>(st.wr, nx.base, nx.units, nxt, st.wv, st.lane);
  ++st.g;
  return cur;
}

// accumulator initialised with the 16 biases of lane half h of one tile
template <int NTL>
__device__ __forceinline__ void bias_init(f32x16 (&acc)[NTL], const float* b) {
  const float4* b4 = reinterpret_cast<const float4*>(b);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 v = b4[i];
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      acc[nt][4 * i] = v.x; acc[nt][4 * i + 1] = v.y; acc[nt][4 * i + 2] = v.z; acc[nt][4 * i + 3] = v.w;
    }
  }
}

// One MFMA layer: y = act(b + W [x1, x2]) for MTO output tiles of 32 rows,
// chunks of KB1 (+ KB2 with USE2) blocks from `base`; `after` is the first
// group of the item that follows.  x1 is a register array (chained
// activations) or, when X1_LDS, the wave's encoding block in LDS; x2 (the
// encoding segment) comes from LDS, laid out [column tile][k-block][lane].
// The A fragments of a chunk group are one sequence (m-tile by m-tile,
// k-block by k-block) read from LDS in batches of DEPTH into two register
// batches: the reads of batch k + 1 issue right after the first MFMA of batch
// k, so they have the DEPTH MFMAs of batch k to land, and scheduling barriers
// keep that order (left alone, the compiler sinks every read next to its
// use, and each pair of MFMAs then waits out a full LDS latency).  Two
// accumulators alternate between the m-tiles of a group: a tile's bias is
// read into its accumulator while the tile before it still multiplies, and
// the tile before's epilogue runs once this tile's first MFMAs have issued.
// B operands that live in LDS (layer 0's encoding, the encoding segment of
// the skip and direction layers) are read once per layer.
template <class S, int NTL, int WAVES, int MPC, int MTO, int KB1, int KB2, int NY, bool X1_LDS, int NX1, bool USE2,
          int DEPTH>
__device__ __forceinline__ void dense_p(ChunkStream& st, const long base, const float* bl, const bool relu,
                                        const NextGroup after, const bf16x8 (&x1)[NTL][NX1], const uint4* x1s,
                                        const uint4* x2s, bf16x8 (&y)[NTL][NY]) {
  static_assert(2 * MTO <= NY && (X1_LDS || KB1 <= NX1), "layout");
  static_assert(!(X1_LDS && USE2), "one LDS operand segment per layer");
  constexpr int KBT = KB1 + (USE2 ? KB2 : 0);
  static_assert(KBT >= 3, "the next tile's bias is read at k-block 2");
  constexpr int NB1 = X1_LDS ? KB1 : 1;
  constexpr int NB2 = USE2 ? KB2 : 1;
  constexpr int NG = (MTO + MPC - 1) / MPC;
  const int lane = st.lane;
  bf16x8 b1[NTL][NB1], b2[NTL][NB2];
  if constexpr (X1_LDS) {
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
      for (int kb = 0; kb < KB1; ++kb) b1[nt][kb] = __builtin_bit_cast(bf16x8, x1s[(nt * KB1 + kb) * 64 + lane]);
  }
  if constexpr (USE2) {
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
      for (int kb = 0; kb < KB2; ++kb) b2[nt][kb] = __builtin_bit_cast(bf16x8, x2s[(nt * KB2 + kb) * 64 + lane]);
  }
  static_for<NG>([&](auto gc) __attribute__((always_inline)) {
    constexpr int g0 = decltype(gc)::value * MPC;
    constexpr int NM = MTO - g0 < MPC ? MTO - g0 : MPC;
    constexpr int F = NM * KBT;
    NextGroup nx = after;
    if constexpr (g0 + MPC < MTO) {
      nx.base = base + (long)(g0 + MPC) * KBT;
      nx.units = (MTO - g0 - MPC < MPC ? MTO - g0 - MPC : MPC) * KBT;
    }
    const uint4* cur = group_begin<WAVES>(st, nx);
    f32x16 acc[2][NTL];
    bf16x8 ring[2 * DEPTH];
    bias_init<NTL>(acc[0], bl + g0 * 32);
    static_for<(DEPTH < F ? DEPTH : F)>([&](auto ic) __attribute__((always_inline)) {
      constexpr int i = decltype(ic)::value;
      ring[i] = __builtin_bit_cast(bf16x8, cur[i * 64 + lane]);
    });
    __builtin_amdgcn_sched_barrier(0);
    static_for<F>([&](auto fc) __attribute__((always_inline)) {
      constexpr int f = decltype(fc)::value;
      constexpr int mt = f / KBT, kb = f % KBT, p = mt & 1;
      const bf16x8 a = ring[f % (2 * DEPTH)];
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        bf16x8 bx;
        if constexpr (kb < KB1) {
          if constexpr (X1_LDS) bx = b1[nt][kb];
          else bx = x1[nt][kb];
        } else {
          bx = b2[nt][kb - KB1];
        }
        acc[p][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[p][nt], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (f % DEPTH == 0) {
        static_for<DEPTH>([&](auto jc) __attribute__((always_inline)) {
          constexpr int q = f + DEPTH + decltype(jc)::value;
          if constexpr (q < F) ring[q % (2 * DEPTH)] = __builtin_bit_cast(bf16x8, cur[q * 64 + lane]);
        });
      }
      if constexpr (kb == 1 && mt > 0) epilogue_b<NTL>(acc[p ^ 1], relu, g0 + mt - 1, y);
      if constexpr (kb == 2 && mt + 1 < NM) bias_init<NTL>(acc[p ^ 1], bl + (g0 + mt + 1) * 32);
      __builtin_amdgcn_sched_barrier(0);
    });
    epilogue_b<NTL>(acc[(NM - 1) & 1], relu, g0 + NM - 1, y);
  });
}

// a head tile of the stream: acc = b + W [x, x2] (one 32-row tile, one group)
template <int NTL, int WAVES, int KB1, int KB2, int NX>
__device__ __forceinline__ void head_b(ChunkStream& st, const float* bl, const NextGroup after,
                                       const bf16x8 (&x)[NTL][NX], const uint4* x2s, f32x16 (&acc)[NTL]) {
  const uint4* cur = group_begin<WAVES>(st, after);
  const int lane = st.lane;
  bias_init<NTL>(acc, bl);
  static_for<KB1 + KB2>([&](auto kc) __attribute__((always_inline)) {
    constexpr int kb = decltype(kc)::value;
    const bf16x8 a = __builtin_bit_cast(bf16x8, cur[kb * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      bf16x8 bx;
      if constexpr (kb < KB1) bx = x[nt][kb];
      else bx = __builtin_bit_cast(bf16x8, x2s[(nt * KB2 + kb - KB1) * 64 + lane]);
      acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[nt], 0, 0, 0);
    }
  });
}

// hidden layer l >= 1 (the skip layer appends the position encoding)
template <class S, int NTL, int WAVES, int MPC>
__device__ __forceinline__ void hidden(ChunkStream& st, const int l, const float* bias, const int h,
                                       const NextGroup after, const bf16x8 (&x)[NTL][S::KBH], const uint4* gx,
                                       bf16x8 (&y)[NTL][S::KBH]) {
  if (l == S::SKIP)
    dense_p<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBX, S::KBH, false, S::KBH, true, kBf16Batch>(
        st, S::block_base(l), bias + S::bias_base(l) + h * 16, true, after, x, nullptr, gx, y);
  else
    dense_p<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBX, S::KBH, false, S::KBH, false, kBf16Batch>(
        st, S::block_base(l), bias + S::bias_base(l) + h * 16, true, after, x, nullptr, gx, y);
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
  ChunkStream st{raw_rsrc(a.wblocks, (int)(S::BLOCKS * 1024)), slot0, slot1, 0, wv, lane};
  // weights of layer 0's first chunk group start loading while the inputs
  // are encoded; biases go to LDS (visible after the first barrier)
  {
    const NextGroup g0 = first_group<S, MPC>(0);
    issue_blocks_buf<WAVES>(st.wr, g0.base, g0.units, slot0, wv, lane);
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
  dense_p<S, NTL, WAVES, MPC, S::MT, S::KBX, S::KBD, S::KBH, true, S::KBH, false, kBf16Batch>(
      st, S::block_base(0), bias + S::bias_base(0) + h * 16, true,
      S::D > 1 ? first_group<S, MPC>(1) : sig_group, xb, s_gx[wv], s_gd[wv], xa);
  // hidden layers 1 .. D-1, ping-ponging between xa and xb; the result ends
  // in xa (a final copy when D - 1 is odd)
#pragma unroll 1
  for (int l = 1; l < S::D; l += 2) {
    hidden<S, NTL, WAVES, MPC>(st, l, bias, h, l + 1 < S::D ? first_group<S, MPC>(l + 1) : sig_group, xa, s_gx[wv],
                               xb);
    if (l + 1 < S::D)
      hidden<S, NTL, WAVES, MPC>(st, l + 1, bias, h, l + 2 < S::D ? first_group<S, MPC>(l + 2) : sig_group, xb,
                                 s_gx[wv], xa);
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
    dense_p<S, NTL, WAVES, MPC, S::MT, S::KBH, S::KBD, S::KBH, false, S::KBH, false, kBf16Batch>(
        st, S::block_base(S::D), bias + S::bias_base(S::D) + h * 16, false, first_group<S, MPC>(S::D + 1),
        xa, nullptr, s_gd[wv], xb);
    dense_p<S, NTL, WAVES, MPC, S::MTD, S::KBH, S::KBD, S::KBH, false, S::KBH, true, kBf16Batch>(
        st, S::block_base(S::D + 1), bias + S::bias_base(S::D + 1) + h * 16, true,
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
// tiles per wave (one wave per SIMD) and 4-wave workgroups were slower, and
// so were read-ahead batches of 3 or 4 fragments.  Staging the weights
// through registers (plain loads, then LDS stores) instead of direct loads
// into LDS measured the same: the cost of the weight stream is the stream
// itself, 1.2 MB from L2 per 256 samples.
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
