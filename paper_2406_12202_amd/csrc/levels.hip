// Coarse-to-fine update of the small map (4x64, bf16 MFMA, 32 stratified
// samples per ray): a begin kernel, then per level one persistent fused ray
// kernel, a scores kernel and one single-workgroup level kernel.
//
// k_level_begin writes the call's key, predicts the first level's particles
// and draws the motion increments of the later levels.
//
// k_level_rays keeps the whole packed map (30 KB of bf16 chunks, biases,
// heads) resident in LDS, beside 1.6 KB of staging rows per wave, and
// walks the level's rays with a grid-stride loop over waves: for each ray
// (one 32-sample column tile) it generates the pixel
// ray of the particle's predicted pose, the box-averaged observation, the
// stratified samples and their encodings, evaluates the map, composites along
// the ray with a wave scan of log transmittance, finds Eq. 5's depths, and
// writes the ray's (C, A) and (F, E).  Every ray is computed by one wave with
// the same instruction sequence as the unfused kernels (raygen, k_mlp_bf16,
// k_composite), so the results do not depend on the tile configuration.
//
// k_level_scores reduces each particle's rays in fixed order to S_i, l_i and
// the mean uncertainty (Eq. 6).
//
// k_level_finish applies the 1-sigma rejection, normalises, reads out the
// pose, resamples to the next level's particle count, gathers the drawn
// poses and applies the next level's prediction.
#include "filter_dev.h"
#include "compositing.h"
#include "maplayout_bf16.h"
#include "mfma_util.h"

namespace fl {

using LS = SmallMapB;
constexpr int kLevelSpr = 32;   // samples per ray on this path

// the call's key written for the later kernels, the first level's
// prediction from the same values (passed by value), and in further
// workgroups the motion increments of the later levels (they depend on the
// drawn slot k, not on which particle is drawn, so the level kernels only
// apply them); one wave per workgroup: the float64 arithmetic spreads over
// as many CUs
__global__ __launch_bounds__(64) void k_level_begin(LevelKey* key, const LevelKey v, const double* pose_in,
                                                     double* pose_out, int N, const LevelIncs incs) {
  const int nb0 = (N + 63) / 64;
  int b = blockIdx.x;
  if (b < nb0) {
    const int i = b * 64 + threadIdx.x;
    if (i == 0) *key = v;
    if (i < N) predict_pose(pose_in + (long)i * 12, pose_out + (long)i * 12, v.motion, v.sigma_t, v.sigma_r, v.seed,
                            v.iter, i);
    return;
  }
  b -= nb0;
  for (int L = 0; L < kMaxLevels; ++L) {
    const int nb = (incs.n[L] + 63) / 64;
    if (b < nb) {
      const int k = b * 64 + threadIdx.x;
      if (k < incs.n[L]) {
        double E[12];
        motion_increment(v.sigma_t, v.sigma_r, v.seed, v.iter + (uint64_t)L + 1, k, E);
        for (int q = 0; q < 12; ++q) incs.inc[L][(long)k * 12 + q] = E[q];
      }
      return;
    }
    b -= nb;
  }
}

static unsigned begin_blocks(const int N, const LevelIncs& incs) {
  long nb = (N + 63) / 64;
  for (int L = 0; L < kMaxLevels; ++L) nb += (incs.n[L] + 63) / 64;
  return (unsigned)nb;
}

hipError_t launch_level_begin(LevelKey* key, const LevelKey& v, const double* pose_in, double* pose_out, int N,
                              const LevelIncs& incs, hipStream_t st) {
  hipLaunchKernelGGL(k_level_begin, dim3(begin_blocks(N, incs)), dim3(64), 0, st, key, v, pose_in, pose_out, N, incs);
  return hipGetLastError();
}

// the k_level_begin node of an instantiated graph given the next call's key
// (the node keeps its launch shape; its arguments are copied when set)
hipError_t set_level_begin_node(hipGraphExec_t ge, hipGraphNode_t node, LevelKey* key, const LevelKey& v,
                                const double* pose_in, double* pose_out, int N, const LevelIncs& incs) {
  hipKernelNodeParams p{};
  hipError_t e = hipGraphKernelNodeGetParams(node, &p);
  if (e != hipSuccess) return e;
  if (p.func != reinterpret_cast<void*>(&k_level_begin)) return hipErrorInvalidValue;
  if (p.gridDim.x != begin_blocks(N, incs)) return hipErrorInvalidValue;
  LevelKey* k = key;
  LevelKey vv = v;
  const double* pi = pose_in;
  double* po = pose_out;
  int n = N;
  LevelIncs ic = incs;
  void* args[] = {&k, &vv, &pi, &po, &n, &ic};
  p.kernelParams = args;
  p.extra = nullptr;
  return hipGraphExecKernelNodeSetParams(ge, node, &p);
}

// one layer with weights resident in LDS: y = act(b + W x), MTO output tiles
template <int NTL, int MTO, int KB1, int NX1, bool X1_LDS, int NY>
__device__ __forceinline__ void dense_res(const uint4* w, const float* bl, const bool relu,
                                          const bf16x8 (&x1)[NTL][NX1], const uint4* x1s, bf16x8 (&y)[NTL][NY],
                                          const int lane) {
#pragma unroll
  for (int mt = 0; mt < MTO; ++mt) {
    f32x16 binit;
    const float4* b4 = reinterpret_cast<const float4*>(bl + mt * 32);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 v = b4[i];
      binit[4 * i] = v.x; binit[4 * i + 1] = v.y; binit[4 * i + 2] = v.z; binit[4 * i + 3] = v.w;
    }
    f32x16 acc[NTL];
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) acc[nt] = binit;
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, w[(mt * KB1 + kb) * 64 + lane]);
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        bf16x8 bx;
        if constexpr (X1_LDS) bx = __builtin_bit_cast(bf16x8, x1s[(nt * KB1 + kb) * 64 + lane]);
        else bx = x1[nt][kb];
        acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bx, acc[nt], 0, 0, 0);
      }
    }
    epilogue_b<NTL>(acc, relu, mt, y);
  }
}

// per-lane set-up of ray r as k_raygen computes it: query pixel p_j, the
// unit direction through it (camera_ray, float32),
// the origin, and the S x S box average of the observation (row-major sum in
// float32, as k_raygen); S is the level factor
constexpr int kRayBatch = 8;   // rays set up per wave at once (one per lane)

struct RaySetup {
  float o[3], d[3], obs[3];
  int i, j;
};

template <int S>
__device__ __forceinline__ void ray_setup(const LevelRayArgs& a, uint64_t seed, uint64_t iter, long r, RaySetup& rs) {
  const int i = (int)(r / a.B), j = (int)(r - (r / a.B) * a.B);
  rs.i = i;
  rs.j = j;
  const uint32_t w = draw(seed, iter, kStreamPix, (uint32_t)j, 0, 0).x;
  const uint32_t npix = (uint32_t)a.Wl * (uint32_t)a.Hl;
  const uint32_t p = (uint32_t)(((uint64_t)w * npix) >> 32);
  const int u = (int)(p % (uint32_t)a.Wl), v = (int)(p / (uint32_t)a.Wl);
  camera_ray(a.pose + (long)i * 12, u, v, a.fx, a.fy, a.cx, a.cy, rs.o, rs.d);
  float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
  for (int yy = 0; yy < S; ++yy) {
    const float* row = a.image + ((long)(v * S + yy) * a.W_full + (long)u * S) * 3;
    float px[3 * S];
#pragma unroll
    for (int e = 0; e < 3 * S; ++e) px[e] = row[e];
#pragma unroll
    for (int xx = 0; xx < S; ++xx) { c0 += px[3 * xx]; c1 += px[3 * xx + 1]; c2 += px[3 * xx + 2]; }
  }
  const float sc = 1.0f / (float)(S * S);
  rs.obs[0] = c0 * sc; rs.obs[1] = c1 * sc; rs.obs[2] = c2 * sc;
}

// segmented wave primitives over the two 32-lane halves (DPP scans; for the
// lanes of either half they give bitwise the results of the full-wave
// primitives on a wave whose lanes 32..63 hold zeros, which is how the
// unfused compositing kernel uses them); h: the lane's half
__device__ __forceinline__ float half_incl_scan(float v, int) { return half_scan(v, 0.0f, OpAddF{}); }
__device__ __forceinline__ float half_sum(float v, int h) {
  const float s = half_scan(v, 0.0f, OpAddF{});
  const float s0 = lane_value(s, 31), s1 = lane_value(s, 63);
  return h ? s1 : s0;
}
__device__ __forceinline__ int half_min_int(int v, int h) {
  const int s = half_scan(v, 0x7fffffff, OpMinI{});
  const int s0 = lane_value(s, 31), s1 = lane_value(s, 63);
  return h ? s1 : s0;
}

// Waves per SIMD the ray kernel is compiled for (at most 168 registers, a
// few spilled): measured on MI355X, three waves hide more of each ray pair's
// dependent chain than two at 240 registers (185 against 201 us per
// coarse-to-fine update).
#ifndef FL_LEVEL_WAVES_PER_EU
#define FL_LEVEL_WAVES_PER_EU 3
#endif

template <int WAVES>
struct LevelCfg {
  static constexpr int THREADS = 64 * WAVES;
  static constexpr long LDS = LS::BLOCKS * 1024 + LS::BIASES * 4 + WAVES * (1024 + kRayBatch * (48 + 32 * LS::KBD));
};

// the head tile with the direction operands in registers (head_tile's
// arithmetic, operand gd[nt][kb] for column tile nt)
template <int NTL>
__device__ __forceinline__ void head_tile_r(const uint4* w, const float* bl, const bf16x8 (&x)[NTL][LS::KBH],
                                            const bf16x8 (&gd)[NTL][LS::KBD], const int lane, f32x16 (&acc)[NTL]) {
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
  for (int kb = 0; kb < LS::KBH; ++kb) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, w[kb * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x[nt][kb], acc[nt], 0, 0, 0);
  }
#pragma unroll
  for (int kb = 0; kb < LS::KBD; ++kb) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, w[(LS::KBH + kb) * 64 + lane]);
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, gd[nt][kb], acc[nt], 0, 0, 0);
  }
}

// orders one wave's LDS writes before its later reads of other lanes' words
// (a wave's LDS operations complete in issue order; this keeps the compiler
// from moving them across)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column-tile operands from a lane's two k-halves.  On entry lane (n, h)
// holds k-half 0 of sample n of ray h in t0 and k-half 1 in t1; on return t0
// is column tile 0's operand (lane (n, h): k-half h of ray 0's sample n) and
// t1 column tile 1's.  v_permlane32_swap exchanges the upper 32 lanes of its
// first operand with the lower 32 lanes of its second, which is exactly the
// move of ray 0's k-half 1 up and ray 1's k-half 0 down.
__device__ __forceinline__ uint32_t swap_lo(uint32_t& a, const uint32_t b) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  return r[1];
}

__device__ __forceinline__ void tile_pair(bf16x8& t0, bf16x8& t1) {
  uint4 u = __builtin_bit_cast(uint4, t0), v = __builtin_bit_cast(uint4, t1);
  v.x = swap_lo(u.x, v.x);
  v.y = swap_lo(u.y, v.y);
  v.z = swap_lo(u.z, v.z);
  v.w = swap_lo(u.w, v.w);
  t0 = __builtin_bit_cast(bf16x8, u);
  t1 = __builtin_bit_cast(bf16x8, v);
}

// Rays go through the wave in pairs: lane (n, h) = lane n + 32 h owns sample
// n of ray h of the pair for everything outside the MFMAs (jitter, depth,
// encoding, head nonlinearities, compositing), so no lane repeats another's
// work; a lane computes both k-halves of its sample's encoding operands and
// exchanges one half with lane xor 32 (v_permlane32_swap) to hold the MFMA
// operands of both column tiles, the map runs on the two tiles, and the head
// rows of tile 1 move from half 0 to half 1 by the same swap.  A batch's ray
// data (origin, direction, observation, direction-encoding operands, jitter
// draws) is staged once in the wave's LDS rows and read back per pair.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(FL_LEVEL_WAVES_PER_EU))) void
k_level_rays(const LevelRayArgs a) {
  using C = LevelCfg<WAVES>;
  constexpr int NTL = 2;
  __shared__ uint4 s_w[LS::BLOCKS * 64];
  __shared__ float4 s_bias[LS::BIASES / 4];
  __shared__ uint32_t s_jit[WAVES][4 * 64];   // per wave: the batch's jitter draws, [lane][word]
  __shared__ float4 s_ray[WAVES][kRayBatch][3];   // per wave: the batch's rays, {o, obs0}, {d, obs1}, {obs2}
  __shared__ uint4 s_gdir[WAVES][kRayBatch][2 * LS::KBD];   // per wave: their direction operands [ray][half][k-block]
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 31, h = lane >> 5;
  {
    const uint4* wb = reinterpret_cast<const uint4*>(a.wblocks);
    for (int i = threadIdx.x; i < LS::BLOCKS * 64; i += C::THREADS) s_w[i] = wb[i];
    for (int i = threadIdx.x; i < LS::BIASES / 4; i += C::THREADS)
      s_bias[i] = reinterpret_cast<const float4*>(a.bias)[i];
  }
  __syncthreads();
  const uint64_t seed = a.key->seed, iter = a.key->iter + (uint64_t)a.level;
  const float* bias = reinterpret_cast<const float*>(s_bias);
  const long n_rays = (long)a.N * a.B;
  const long n_batches = (n_rays + kRayBatch - 1) / kRayBatch;
  const long n_waves = (long)gridDim.x * WAVES;
  for (long bt = (long)blockIdx.x * WAVES + wv; bt < n_batches; bt += n_waves) {
    // lane q (mod kRayBatch) sets up ray bt * kRayBatch + q
    RaySetup rs;
    {
      long r = bt * kRayBatch + (lane & (kRayBatch - 1));
      if (r >= n_rays) r = n_rays - 1;
      switch (a.s) {
        case 1: ray_setup<1>(a, seed, iter, r, rs); break;
        case 2: ray_setup<2>(a, seed, iter, r, rs); break;
        case 4: ray_setup<4>(a, seed, iter, r, rs); break;
        default: ray_setup<8>(a, seed, iter, r, rs); break;
      }
    }
    // once per batch, into the wave's LDS rows: lane q's ray (origin,
    // direction, observation) and the bf16 operands of its direction
    // encoding for q < kRayBatch, and the jitter draws of all its rays, lane
    // 8 q + g drawing ray q's samples 4 g .. 4 g + 3 (word 32 q + k of the
    // jitter row is then sample k of ray q)
    bf16x8 gdr[2][LS::KBD];
    posenc_both<LS::LD, LS::KBD>(rs.d[0], rs.d[1], rs.d[2], gdr);
    static_assert(kRayBatch * kLevelSpr / 4 == 64, "one draw per lane covers a batch");
    u32x4 jd = {0u, 0u, 0u, 0u};
    if (a.jitter) {
      const int qd = lane >> 3;
      jd = draw(seed, iter, kStreamJitCoarse, __shfl(rs.i, qd, 64), __shfl(rs.j, qd, 64), lane & 7);
    }
    wave_lds_sync();   // the previous batch's reads are done
    if (lane < kRayBatch) {
      s_ray[wv][lane][0] = make_float4(rs.o[0], rs.o[1], rs.o[2], rs.obs[0]);
      s_ray[wv][lane][1] = make_float4(rs.d[0], rs.d[1], rs.d[2], rs.obs[1]);
      s_ray[wv][lane][2] = make_float4(rs.obs[2], 0.0f, 0.0f, 0.0f);
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int kb = 0; kb < LS::KBD; ++kb) s_gdir[wv][lane][hh * LS::KBD + kb] = __builtin_bit_cast(uint4, gdr[hh][kb]);
    }
    if (a.jitter) {
      s_jit[wv][4 * lane] = jd.x;
      s_jit[wv][4 * lane + 1] = jd.y;
      s_jit[wv][4 * lane + 2] = jd.z;
      s_jit[wv][4 * lane + 3] = jd.w;
    }
    wave_lds_sync();
    for (int q0 = 0; q0 < kRayBatch; q0 += 2) {
      // this lane's ray (q0 + h) and sample n
      const int q = q0 + h;
      const long ray = bt * kRayBatch + q;
      const float4 o = s_ray[wv][q][0], d = s_ray[wv][q][1];
      const float ob0 = o.w, ob1 = d.w, ob2 = s_ray[wv][q][2].x;
      const int k = n;
      float xi = 0.0f;
      if (a.jitter) xi = unit24(s_jit[wv][32 * q0 + lane]);   // sample k of ray q
      const float tk = a.near_ + ((float)k + xi) * a.dt;
      bf16x8 x0[NTL][LS::KBX], gdt[NTL][LS::KBD];
      posenc_both<LS::LX, LS::KBX>(fmaf(tk, d.x, o.x), fmaf(tk, d.y, o.y), fmaf(tk, d.z, o.z), x0);
#pragma unroll
      for (int kb = 0; kb < LS::KBX; ++kb) tile_pair(x0[0][kb], x0[1][kb]);
      // column tile nt: k-half h of ray q0 + nt's direction operands
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
        for (int kb = 0; kb < LS::KBD; ++kb)
          gdt[nt][kb] = __builtin_bit_cast(bf16x8, s_gdir[wv][q0 + nt][h * LS::KBD + kb]);
      // the map on both column tiles (layer order and arithmetic of k_mlp_bf16)
      bf16x8 xa[NTL][LS::KBH], xb[NTL][LS::KBH];
      dense_res<NTL, LS::MT, LS::KBX, LS::KBX, false, LS::KBH>(s_w + LS::block_base(0) * 64,
                                                              bias + LS::bias_base(0) + h * 16, true, x0, nullptr,
                                                              xa, lane);
#pragma unroll
      for (int l = 1; l < LS::D; ++l) {
        dense_res<NTL, LS::MT, LS::KBH, LS::KBH, false, LS::KBH>(s_w + LS::block_base(l) * 64,
                                                                bias + LS::bias_base(l) + h * 16, true, xa, nullptr,
                                                                xb, lane);
#pragma unroll
        for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
          for (int qq = 0; qq < LS::KBH; ++qq) xa[nt][qq] = xb[nt][qq];
      }
      f32x16 hacc[NTL];
      head_tile_r<NTL>(s_w + LS::HEAD_BLOCK * 64, bias + LS::HEAD_BIAS + h * 16, xa, gdt, lane, hacc);
      // head rows 0..3 of tile h (each the sum of a weight row's high and
      // low bf16 parts, rows r and r + 8): half 0 holds them for both tiles
      float hv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        uint32_t r0 = __float_as_uint(hacc[0][v] + hacc[0][v + 4]);
        swap_lo(r0, __float_as_uint(hacc[1][v] + hacc[1][v + 4]));
        hv[v] = __uint_as_float(r0);
      }
      // everything below reads only lanes of the same half before the
      // shuffles of the next pair
      __builtin_amdgcn_wave_barrier();
      const float sg = softplus_b(hv[0]);
      const float cr0 = sigmoid_b(hv[1]), cg0 = sigmoid_b(hv[2]), cb0 = sigmoid_b(hv[3]);
      // compositing along the ray (as k_composite with one sample per lane)
      float tn = __shfl_down(tk, 1, 32);
      if (n + 1 >= kLevelSpr) tn = a.far_;
      float lsum = 0.0f;
      lsum += sg * (tn - tk);
      const float incl = half_incl_scan(lsum, n);
      float run = -(incl - lsum);
      float cr = 0.0f, cg = 0.0f, cb = 0.0f, accw = 0.0f;
      int ktr = 1 << 30, kop = 1 << 30;
      const float tau = sg * (tn - tk);
      const float w = transmittance(run) * opacity(tau);
      const float lt = run;
      cr = fmaf(w, cr0, cr); cg = fmaf(w, cg0, cg); cb = fmaf(w, cb0, cb);
      accw += w;
      run -= tau;
      if (run <= a.log_trans) ktr = n;
      if (run < a.log_opq) kop = n;
      cr = half_sum(cr, h); cg = half_sum(cg, h); cb = half_sum(cb, h); accw = half_sum(accw, h);
      ktr = half_min_int(ktr, h);
      kop = half_min_int(kop, h);
      float F = a.empty_F;
      if (ktr < kLevelSpr) {
        const float t_tr = __shfl(tk, ktr, 32), l_tr = __shfl(lt, ktr, 32), s_tr = __shfl(sg, ktr, 32);
        const int ko = kop < kLevelSpr ? kop : 0;
        const float t_op = __shfl(tk, ko, 32), l_op = __shfl(lt, ko, 32), s_op = __shfl(sg, ko, 32);
        const float zt = crossing_depth(t_tr, l_tr, a.log_trans, s_tr);
        const float zo = (kop < kLevelSpr) ? crossing_depth(t_op, l_op, a.log_opq, s_op) : a.far_;
        F = fmaxf(zo - zt, a.tau);
      }
      const float er = ob0 - cr, eg = ob1 - cg, eb = ob2 - cb;
      const float E = er * er + eg * eg + eb * eb;
      if (ray < n_rays && n == 0) {
        a.ray_rgba[ray] = make_float4(cr, cg, cb, accw);
        a.ray_fe[ray] = make_float2(F, E);
      }
    }
  }
}

template <int WAVES>
hipError_t launch_level_rays_t(const LevelRayArgs& a, int blocks, hipStream_t st) {
  static_assert(LevelCfg<WAVES>::LDS <= 160 * 1024, "LDS budget");
  hipLaunchKernelGGL((k_level_rays<WAVES>), dim3(blocks), dim3(64 * WAVES), 0, st, a);
  return hipGetLastError();
}

bool level_rays_config_ok(int ntl, int waves) { return ntl == 2 && (waves == 2 || waves == 4 || waves == 8); }

hipError_t launch_level_rays(const LevelRayArgs& a, int ntl, int waves, int blocks, hipStream_t st) {
  if ((long)a.N * a.B <= 0) return hipSuccess;
  if (blocks < 1 || ntl != 2) return hipErrorInvalidValue;
  if (waves == 2) return launch_level_rays_t<2>(a, blocks, st);
  if (waves == 4) return launch_level_rays_t<4>(a, blocks, st);
  if (waves == 8) return launch_level_rays_t<8>(a, blocks, st);
  return hipErrorInvalidValue;
}

// per-particle scores: groups of G lanes per particle (the order of
// particle_sums), 256 threads per workgroup; the float64 mean F waits in
// weight[] for the rejection statistics
constexpr int kScoreThreads = 256;

__global__ __launch_bounds__(kScoreThreads) void k_level_scores(const LevelFinishArgs a) {
  const int G = particle_group(a.B);
  const int tid = blockIdx.x * kScoreThreads + threadIdx.x;
  const int g = threadIdx.x & (G - 1);
  const int i = tid / G;
  if (i >= a.N) return;   // whole groups leave together
  double S_i, Fs;
  particle_sums([&](int jj, float& ef, float& f) {
    const float2 fe = a.ray_fe[(long)i * a.B + jj];
    ef = fe.y * fe.x;
    f = fe.x;
  }, a.B, G, g, S_i, Fs);
  if (g == 0) {
    const double Sfl = (S_i > 1e-12 || isnan(S_i)) ? S_i : 1e-12;   // NaN stays NaN
    a.loglik[i] = 4.0 * (log((double)a.B) - log(Sfl));
    a.uncert[i] = (float)(Fs / a.B);
    a.weight[i] = Fs / a.B;
  }
}

hipError_t launch_level_scores(const LevelFinishArgs& a, hipStream_t st) {
  const long threads = (long)a.N * particle_group(a.B);
  const int score_blocks = (int)((threads + kScoreThreads - 1) / kScoreThreads);
  hipLaunchKernelGGL(k_level_scores, dim3((unsigned)score_blocks), dim3(kScoreThreads), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rejection (mean F above mean + one standard deviation, Sec. III-C),
// normalisation, read-out and the draw of one level on the particles' l and
// mean F (L, W: LDS copies for small sets, else the global arrays; W holds
// the weights on return).
__device__ __forceinline__ void level_weigh_and_draw(const LevelFinishArgs& a, double* L, double* W, double* s_d,
                                                     u64* s_u, u64* s_prefix, const uint64_t seed,
                                                     const uint64_t iter, int32_t* idx_lds) {
  const int tid = threadIdx.x;
  if (a.reject) {
    // mean and population standard deviation of the mean F over particles
    // with finite mean F and finite l; particles above mean + std get -inf
    double cnt = 0.0, sum = 0.0;
    for (int i = tid; i < a.N; i += kRedThreads) {
      const double U = W[i];
      if (isfinite(U) && isfinite(L[i])) { cnt += 1.0; sum += U; }
    }
    const double2 cs = block_sum2(cnt, sum, s_d);
    const double n_ok = cs.x;
    const double mu = n_ok > 0.0 ? cs.y / n_ok : 0.0;
    double ss = 0.0;
    for (int i = tid; i < a.N; i += kRedThreads) {
      const double U = W[i];
      if (isfinite(U) && isfinite(L[i])) ss += (U - mu) * (U - mu);
    }
    const double sd = block_sum(ss, s_d);
    const double thr = mu + (n_ok > 0.0 ? sqrt(sd / n_ok) : 0.0);
    for (int i = tid; i < a.N; i += kRedThreads) {
      const double U = W[i];
      const bool ok = isfinite(U) && isfinite(L[i]);
      if (!ok || U > thr) L[i] = -INFINITY;
    }
    __threadfence_block();
    __syncthreads();
  }
  const double wmax = normalize_block(L, W, a.N, a.flags, s_d);
  if (a.est) pose_estimate_block(a.pose, W, a.N, a.est, a.flags, reinterpret_cast<double(*)[13]>(s_d));
  resample_block(W, a.N, a.n_out, seed, iter, a.prefix, a.idx, a.flags, s_d, s_u, s_prefix, wmax, idx_lds);
}

// sets up to this size have their poses read into registers at the start
// (two per thread) and staged in LDS for the gather once the draw is done
constexpr int kPoseStage = 2 * kRedThreads;

__global__ __launch_bounds__(kRedThreads) void k_level_finish(const LevelFinishArgs a) {
  __shared__ double s_d[kEstThreads * 13];   // reused by every phase
  __shared__ u64 s_u[kRedThreads / 64];
  // l, w and the integer prefix of a set that fits; after the draw, the
  // staged poses (12 doubles per particle)
  __shared__ double s_lw[3 * kPrefixLds];
  __shared__ int32_t s_idx[kPrefixLds];
  __shared__ double s_sink;
  static_assert(12 * kPoseStage <= 3 * kPrefixLds, "staged poses fit");
  double* s_l = s_lw;
  double* s_w = s_lw + kPrefixLds;
  u64* s_prefix = reinterpret_cast<u64*>(s_lw + 2 * kPrefixLds);
  const int tid = threadIdx.x;
  const uint64_t seed = a.key->seed, iter = a.key->iter + (uint64_t)a.level;
  // scores, mean F (in weight[]) come from k_level_scores; a set that fits is
  // read once into LDS, so the passes over it do not wait on memory
  const bool small = a.N <= kPrefixLds;
  if (small)
    for (int i = tid; i < a.N; i += kRedThreads) {
      s_l[i] = a.loglik[i];
      s_w[i] = a.weight[i];
    }
  // The gather's inputs, read now so that their latency passes while the
  // phases below run: the poses (written by the kernel before the scores,
  // mostly on other XCDs), this thread's motion increment and O_t.
  const bool stage = a.N <= kPoseStage;
  double pr[2][12];
  if (stage) {
    for (int j = 0; j < 2; ++j) {
      const int i = tid + j * kRedThreads;
      if (i < a.N)
        for (int q = 0; q < 12; ++q) pr[j][q] = a.pose[(long)i * 12 + q];
    }
  } else {
    double t = 0.0;
    for (int i = tid; i < (a.N * 12 + 15) / 16; i += kRedThreads) t += a.pose[i * 16];   // one read per 128 B
    if (t != t) s_sink = t;   // keeps the reads: the gather then finds the poses in this XCD's L2
  }
  const bool inc_r = a.predict_next && a.n_out <= kRedThreads;
  double inc[12], mo[12];
  if (inc_r && tid < a.n_out)
    for (int q = 0; q < 12; ++q) inc[q] = a.inc[(long)tid * 12 + q];
  for (int q = 0; q < 12; ++q) mo[q] = a.key->motion[q];
  int32_t* idx_lds = a.n_out <= kPrefixLds ? s_idx : nullptr;
  if (small) {
    __syncthreads();
    level_weigh_and_draw(a, s_l, s_w, s_d, s_u, s_prefix, seed, iter, idx_lds);
    for (int i = tid; i < a.N; i += kRedThreads) {
      a.loglik[i] = s_l[i];
      a.weight[i] = s_w[i];
    }
  } else {
    level_weigh_and_draw(a, a.loglik, a.weight, s_d, s_u, s_prefix, seed, iter, idx_lds);
  }
  if (stage) {
    __syncthreads();   // l, w and the prefix are read for the last time
    for (int j = 0; j < 2; ++j) {
      const int i = tid + j * kRedThreads;
      if (i < a.N)
        for (int q = 0; q < 12; ++q) s_lw[i * 12 + q] = pr[j][q];
    }
    __syncthreads();
  }
  // gather the drawn poses; apply the next level's prediction to particle k
  auto gather = [&](const double* P) __attribute__((always_inline)) {
    for (int k = tid; k < a.n_out; k += kRedThreads) {
      const int i = idx_lds ? idx_lds[k] : a.idx[k];
      double* out = a.next_pose + (long)k * 12;
      if (i < 0 || i >= a.N) {
        for (int q = 0; q < 12; ++q) out[q] = NAN;
      } else if (a.predict_next) {
        apply_increment(P + (long)i * 12, mo, inc_r ? inc : a.inc + (long)k * 12, out);
      } else {
        for (int q = 0; q < 12; ++q) out[q] = P[(long)i * 12 + q];
      }
    }
  };
  if (stage) gather(s_lw);
  else gather(a.pose);
}

hipError_t launch_level_finish(const LevelFinishArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_level_finish, dim3(1), dim3(kRedThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace fl
