// Learned proposal network: inference with proposal-guided fine placement,
// training (forward + analytic backward with per-wave gradient partials, then
// a fixed-order reduction and Adam), and ray format conversion.
//
// Network: x = [gamma_6(o), gamma_6(d)] (78), h1 = relu(W1 x + b1) (64),
// h2 = relu(W2 h1 + b2) (64), z = W3 h2 + b3 (32), p = softmax(z); parameters
// in the flat order W1, b1, W2, b2, W3, b3 (row-major).  Inference runs on the
// matrix cores, 32 rays per wave (layout below).  Training has one wave per
// ray at a time with hidden unit j on lane j; the vector a layer reads is
// broadcast lane by lane with v_readlane, so no LDS traffic is needed for
// activations.
#include "bf16_tiles.h"
#include "common.h"
#include "kernels.h"

namespace fl {

constexpr int PB = 32, PH = 64, PIN = 78, PENC = 39;
constexpr int P_W1 = 0, P_B1 = P_W1 + PH * PIN, P_W2 = P_B1 + PH, P_B2 = P_W2 + PH * PH;
constexpr int P_W3 = P_B2 + PH, P_B3 = P_W3 + PB * PH, P_N = P_B3 + PB;
static_assert(P_N == kProposalParams, "proposal layout");

__device__ __forceinline__ float bcast(float v, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

// encoding entry k (0..77) of a ray: gamma_6(o) then gamma_6(d), canonical order
__device__ __forceinline__ float prop_feature(const float4 o, const float4 d, int k) {
  const bool dir = k >= PENC;
  const int e = dir ? k - PENC : k;
  const float4 v = dir ? d : o;
  if (e < 3) return e == 0 ? v.x : (e == 1 ? v.y : v.z);
  const int q = e - 3, l = q / 6, r = q % 6, c = r % 3;
  const float x = c == 0 ? v.x : (c == 1 ? v.y : v.z);
  float s, co;
  sincospif(ldexpf(x, l), &s, &co);
  return r < 3 ? s : co;
}

// softmax over lanes 0..31 (lanes 32..63 return garbage); z on lanes 0..31
__device__ __forceinline__ float softmax32(float z, int lane) {
  float m = lane < PB ? z : -INFINITY;
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float e = lane < PB ? expf(z - m) : 0.0f;
  float s = e;
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return e / s;
}

// ---------------------------------------------------------------------------
// inference + placement on the matrix cores (v_mfma_f32_32x32x2_f32, float32
// products and sums).  A wave takes a tile of 32 rays: the layers are computed
// transposed, out^T = W in^T, with the rays as the 32 columns.  In an
// instruction lane l = 32 h + n supplies column n and k-row h of the input; the
// accumulator holds, in lane (n, h) and register v, output row
// 8 (v / 4) + 4 h + v % 4 of column n.  Register v of accumulator tile b is
// then used directly as the input of k-step 16 b + v of the next layer, with
// the matching weights: the contraction index is permuted, not the data.
// Layer 1's k-step kb pairs feature kb of gamma_6(o) (half 0) with feature kb
// of gamma_6(d) (half 1).  The weights, in that operand order, and the biases
// are staged in LDS once per workgroup.
constexpr int kPropWaves = 4;
constexpr int PK1 = PENC;   // 39 k-steps of layer 1
constexpr int PW1 = 2 * PK1 * 64, PW2 = 2 * 32 * 64, PW3 = 32 * 64;

__device__ __forceinline__ void prop_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kPropWaves) void k_proposal_fine(const ProposalArgs a) {
  __shared__ float s_w[PW1 + PW2 + PW3];
  __shared__ float s_b[PH + PH + PB];
  __shared__ float s_c[kPropWaves][32][33];   // per ray: inclusive prefix of the bin masses
  const float* __restrict__ P = a.params;
  for (int e = threadIdx.x; e < PW1 + PW2 + PW3; e += blockDim.x) {
    const int ln = e & 63, n = ln & 31, h = ln >> 5, blk = e >> 6;
    float v;
    if (blk < 2 * PK1) {                   // layer 1: block mt * 39 + kb
      const int mt = blk / PK1, kb = blk - mt * PK1;
      v = P[P_W1 + (mt * 32 + n) * PIN + (h ? PENC + kb : kb)];
    } else if (blk < 2 * PK1 + 64) {      // layer 2: block mt * 32 + s, s = 16 b + r
      const int q = blk - 2 * PK1, mt = q >> 5, st = q & 31;
      v = P[P_W2 + (mt * 32 + n) * PH + 32 * (st >> 4) + tile_row(st & 15, h)];
    } else {                               // layer 3: block s
      const int st = blk - 2 * PK1 - 64;
      v = P[P_W3 + n * PH + 32 * (st >> 4) + tile_row(st & 15, h)];
    }
    s_w[e] = v;
  }
  for (int e = threadIdx.x; e < PH + PH + PB; e += blockDim.x)
    s_b[e] = e < PH ? P[P_B1 + e] : (e < 2 * PH ? P[P_B2 + e - PH] : P[P_B3 + e - 2 * PH]);
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 31, h = lane >> 5;
  const float* w1 = s_w;
  const float* w2 = s_w + PW1;
  const float* w3 = s_w + PW1 + PW2;
  float (*c_ray)[33] = s_c[wv];
  const int tiles = (a.n_rays + 31) / 32;
  for (int tile = blockIdx.x * kPropWaves + wv; tile < tiles; tile += gridDim.x * kPropWaves) {
    const int ray = tile * 32 + n;
    const bool valid = ray < a.n_rays;
    const float4 v = (h ? a.ray_d : a.ray_o)[valid ? ray : a.n_rays - 1];
    // gamma_6 of o (half 0) or d (half 1), canonical order
    float x[PK1];
    x[0] = v.x; x[1] = v.y; x[2] = v.z;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const float vc[3] = {v.x, v.y, v.z};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float sn, cs;
        sincospif(ldexpf(vc[c], l), &sn, &cs);
        x[3 + 6 * l + c] = sn;
        x[3 + 6 * l + 3 + c] = cs;
      }
    }
    // layer 1: 64 hidden rows in two tiles
    pf32x16 h1[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h1[mt][r] = s_b[32 * mt + tile_row(r, h)];
#pragma unroll
    for (int kb = 0; kb < PK1; ++kb)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        h1[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(w1[(mt * PK1 + kb) * 64 + lane], x[kb], h1[mt], 0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h1[mt][r] = fmaxf(h1[mt][r], 0.0f);
    // layer 2
    pf32x16 h2[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h2[mt][r] = s_b[PH + 32 * mt + tile_row(r, h)];
#pragma unroll
    for (int st = 0; st < 32; ++st)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        h2[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(w2[(mt * 32 + st) * 64 + lane], h1[st >> 4][st & 15], h2[mt],
                                                      0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h2[mt][r] = fmaxf(h2[mt][r], 0.0f);
    // layer 3: 32 logits; two accumulators over alternating k-steps (summed
    // once at the end) so that consecutive instructions are independent
    pf32x16 z0, z1;
#pragma unroll
    for (int r = 0; r < 16; ++r) { z0[r] = s_b[2 * PH + tile_row(r, h)]; z1[r] = 0.0f; }
#pragma unroll
    for (int st = 0; st < 32; st += 2) {
      z0 = __builtin_amdgcn_mfma_f32_32x32x2f32(w3[st * 64 + lane], h2[st >> 4][st & 15], z0, 0, 0, 0);
      z1 = __builtin_amdgcn_mfma_f32_32x32x2f32(w3[(st + 1) * 64 + lane], h2[(st + 1) >> 4][(st + 1) & 15], z1, 0,
                                                0, 0);
    }
    // softmax over the 32 logits of column n (16 in each lane half)
    float m = -INFINITY;
#pragma unroll
    for (int r = 0; r < 16; ++r) { z0[r] += z1[r]; m = fmaxf(m, z0[r]); }
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    float sum = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) { z0[r] = expf(z0[r] - m); sum += z0[r]; }
    sum += __shfl_xor(sum, 32, 64);
    const float inv_sum = 1.0f / sum;
#pragma unroll
    for (int r = 0; r < 16; ++r) z0[r] *= inv_sum;
    if (a.hist && valid) {
      float4* hp = reinterpret_cast<float4*>(a.hist + (long)ray * PB);
#pragma unroll
      for (int q = 0; q < 4; ++q) hp[2 * q + h] = make_float4(z0[4 * q], z0[4 * q + 1], z0[4 * q + 2], z0[4 * q + 3]);
    }
    if (a.Sf <= 0) continue;
    // pdf 0.99 p + 0.01 / 32 on 32 equal bins: masses to LDS, then the
    // inclusive prefix of each ray's bins in bin order (lane half 0)
#pragma unroll
    for (int r = 0; r < 16; ++r) c_ray[n][tile_row(r, h)] = 0.99f * z0[r] + 0.01f / PB;
    prop_wave_sync();
    if (h == 0) {
      float c = 0.0f;
      for (int b = 0; b < PB; ++b) { c += c_ray[n][b]; c_ray[n][b] = c; }
    }
    prop_wave_sync();
    const float total = c_ray[n][PB - 1];
    const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
    const float width = (a.far_ - a.near_) / PB;
    // samples 4 q .. 4 q + 3 of the ray share one draw; quads alternate
    // between the lane halves
    for (int q = h; valid && 4 * q < a.Sf; q += 2) {
      u32x4 rnd = {0u, 0u, 0u, 0u};
      if (a.jitter) rnd = draw(a.seed, a.iter, kStreamJitFine, i, j, q);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mm = 4 * q + e;
        if (mm >= a.Sf) break;
        const float xi = a.jitter ? unit24(pick(rnd, e)) : 0.5f;
        const float target = ((float)mm + xi) / (float)a.Sf * total;
        // largest bin b with exclusive prefix c[b - 1] <= target (fixed 5 steps)
        int b = 0;
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
          if (c_ray[n][b + step - 1] <= target) b += step;
        const float c0 = b > 0 ? c_ray[n][b - 1] : 0.0f;
        float frac = (target - c0) / (c_ray[n][b] - c0);
        frac = fminf(fmaxf(frac, 0.0f), 1.0f);
        a.t_fine[(long)ray * a.Sf + mm] = fminf(a.near_ + ((float)b + frac) * width, a.near_ + (b + 1) * width);
      }
    }
    prop_wave_sync();   // the next tile overwrites c_ray
  }
}

hipError_t launch_proposal_fine(const ProposalArgs& a, hipStream_t st) {
  if (a.n_rays <= 0) return hipSuccess;
  const long tiles = ((long)a.n_rays + 31) / 32;
  const long want = (tiles + kPropWaves - 1) / kPropWaves;
  const long blocks = want < 2048 ? want : 2048;
  hipLaunchKernelGGL(k_proposal_fine, dim3((unsigned)blocks), dim3(64 * kPropWaves), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training: one wave per group of rays; weights read from LDS; gradient rows
// accumulated in registers (lane j owns row j of W1, W2 and, for j < 32, W3);
// each wave writes its partial gradient and loss.
constexpr int kTrainWaves = 4;

__global__ __launch_bounds__(256) void k_prop_grad(const TrainArgs a) {
  __shared__ float w[P_N];
  for (int i = threadIdx.x; i < P_N; i += blockDim.x) w[i] = a.params[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kTrainWaves + (threadIdx.x >> 6);
  if (wave >= a.n_waves) return;   // the partial buffers hold n_waves rows (no barrier follows)
  const int l3 = lane < PB ? lane : 0;
  float g1[PIN], g2[PH], g3[PH];
#pragma unroll
  for (int k = 0; k < PIN; ++k) g1[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < PH; ++k) { g2[k] = 0.0f; g3[k] = 0.0f; }
  float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
  const float scale = 2.0f / (float)a.batch;
  for (int q = 0; q < a.rays_per_wave; ++q) {
    const int rb = wave * a.rays_per_wave + q;          // position in the batch
    if (rb >= a.batch) break;
    const long ray = ((long)a.first + rb) % a.n_rays;
    const float4 o = a.ray_o[ray], d = a.ray_d[ray];
    // forward
    const float x0 = prop_feature(o, d, lane);
    const float x1v = lane + 64 < PIN ? prop_feature(o, d, lane + 64) : 0.0f;
    float s1 = w[P_B1 + lane];
#pragma unroll
    for (int k = 0; k < PIN; ++k) s1 = fmaf(w[P_W1 + lane * PIN + k], k < 64 ? bcast(x0, k) : bcast(x1v, k - 64), s1);
    const float h1 = fmaxf(s1, 0.0f);
    float s2 = w[P_B2 + lane];
#pragma unroll
    for (int k = 0; k < PH; ++k) s2 = fmaf(w[P_W2 + lane * PH + k], bcast(h1, k), s2);
    const float h2 = fmaxf(s2, 0.0f);
    float z = w[P_B3 + l3];
#pragma unroll
    for (int k = 0; k < PH; ++k) z = fmaf(w[P_W3 + l3 * PH + k], bcast(h2, k), z);
    const float p = softmax32(z, lane);
    // loss and dL/dz (softmax Jacobian)
    const float tgt = lane < PB ? a.target[ray * PB + lane] : 0.0f;
    const float diff = lane < PB ? p - tgt : 0.0f;
    float sq = diff * diff;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    lsum += sq;
    const float gp = scale * diff;
    float pg = lane < PB ? p * gp : 0.0f;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) pg += __shfl_xor(pg, off, 64);
    const float gz = lane < PB ? p * (gp - pg) : 0.0f;
    // dL/dh2[lane] = sum_j W3[j][lane] gz_j, then ReLU mask
    float gh2 = 0.0f;
#pragma unroll
    for (int jj = 0; jj < PB; ++jj) gh2 = fmaf(w[P_W3 + jj * PH + lane], bcast(gz, jj), gh2);
    const float ga2 = s2 > 0.0f ? gh2 : 0.0f;
    float gh1 = 0.0f;
#pragma unroll
    for (int jj = 0; jj < PH; ++jj) gh1 = fmaf(w[P_W2 + jj * PH + lane], bcast(ga2, jj), gh1);
    const float ga1 = s1 > 0.0f ? gh1 : 0.0f;
    // weight-gradient rows: dW1[lane][k] += ga1 x_k, dW2[lane][k] += ga2 h1_k,
    // dW3[lane][k] += gz h2_k
#pragma unroll
    for (int k = 0; k < PIN; ++k) g1[k] = fmaf(ga1, k < 64 ? bcast(x0, k) : bcast(x1v, k - 64), g1[k]);
#pragma unroll
    for (int k = 0; k < PH; ++k) g2[k] = fmaf(ga2, bcast(h1, k), g2[k]);
#pragma unroll
    for (int k = 0; k < PH; ++k) g3[k] = fmaf(gz, bcast(h2, k), g3[k]);
    gb1 += ga1;
    gb2 += ga2;
    gb3 += gz;
  }
  // per-wave partials in parameter order
  float* out = a.partial + (long)wave * P_N;
#pragma unroll
  for (int k = 0; k < PIN; ++k) out[P_W1 + lane * PIN + k] = g1[k];
#pragma unroll
  for (int k = 0; k < PH; ++k) out[P_W2 + lane * PH + k] = g2[k];
  if (lane < PB) {
#pragma unroll
    for (int k = 0; k < PH; ++k) out[P_W3 + lane * PH + k] = g3[k];
    out[P_B3 + lane] = gb3;
  }
  out[P_B1 + lane] = gb1;
  out[P_B2 + lane] = gb2;
  if (lane == 0) a.loss_partial[wave] = lsum;
}

// sum of the per-wave partials in wave order; then either write the gradient
// or take one Adam step (t = step, counted from 1)
__global__ __launch_bounds__(256) void k_prop_reduce(const TrainArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && a.loss_out) {
    float l = 0.0f;
    for (int v = 0; v < a.n_waves; ++v) l += a.loss_partial[v];
    a.loss_out[a.loss_index] = l / (float)a.batch;
  }
  if (e >= P_N) return;
  // eight interleaved running sums (waves v = 8 u + k into sum k), added in
  // the order k = 0..7: the loads of eight waves are in flight at once
  float g8[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  int v = 0;
  for (; v + 8 <= a.n_waves; v += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) g8[k] += a.partial[(long)(v + k) * P_N + e];
  }
  for (int k = 0; v + k < a.n_waves; ++k) g8[k] += a.partial[(long)(v + k) * P_N + e];
  float g = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) g += g8[k];
  if (a.grad_out) a.grad_out[e] = g;
  if (a.adam) {
    const float m = a.beta1 * a.m[e] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[e] + (1.0f - a.beta2) * g * g;
    a.m[e] = m;
    a.v[e] = v;
    const float mhat = m / (1.0f - powf(a.beta1, (float)a.step));
    const float vhat = v / (1.0f - powf(a.beta2, (float)a.step));
    a.params_rw[e] -= a.lr * mhat / (sqrtf(vhat) + a.eps);
  }
}

hipError_t launch_prop_grad(const TrainArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_prop_grad, dim3((a.n_waves + kTrainWaves - 1) / kTrainWaves), dim3(64 * kTrainWaves), 0,
                     st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prop_reduce, dim3((P_N + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training in bfloat16 on the matrix cores (v_mfma_f32_32x32x16_bf16, float32
// accumulation): a wave takes tiles of 32 rays.  Forward and the backward pass
// through the layers run transposed, out^T = W in^T, with the rays as the 32
// columns: in an instruction lane l = 32 h + n supplies column n and the eight
// k-rows 8 h .. 8 h + 7 of the k-block, and the accumulator holds, in lane
// (n, h) and register v, output row 8 (v / 4) + 4 h + v % 4 of column n.
// Registers v = 0..7 and 8..15 of an output tile, rounded to bf16, are the
// next product's operands of its k-blocks 2 mt and 2 mt + 1, so a chained
// k-block kb carries in half h and slot q the row 16 kb + 8 (q / 4) + 4 h +
// q % 4 (the weights are staged in that order).  Layer 1 reads the encoding
// in natural order (k-row 16 kb + 8 h + q), padded to 80 with x_78 = 1 (the
// bias column of dW1) and x_79 = 0.  The weight gradients contract over the
// rays: each tile's activations and output gradients go through the wave's
// LDS as bf16 [row][ray] tables, whose rows give the 8-ray operand slots,
// and dW = G H^T accumulates in registers over the wave's tiles (one wave per
// SIMD, 512 registers).  db2 and db3 are summed on the vector ALU.  Each wave
// writes its partial gradient in parameter order, as the float32 kernel.
constexpr int kTrainBWaves = 4;
// 32-ray tiles per wave (measured on MI355X for 8192-ray steps: 1, 2 and 4
// tiles took 62, 53 and 60 us per step)
constexpr int kTrainBTiles = 2;
constexpr int PX = 80;                              // padded encoding
constexpr int PKX = PX / 16;                        // 5 k-blocks of layer 1
constexpr int TROW = kTabRow;                       // LDS table row stride (bf16)
// weight fragments (1 KB blocks) in LDS
constexpr int FB_W1 = 0, FB_W2 = FB_W1 + 2 * PKX, FB_W3 = FB_W2 + 2 * 4, FB_W3T = FB_W3 + 4, FB_W2T = FB_W3T + 2 * 2,
              FB_N = FB_W2T + 2 * 4;
// per-wave tables (bf16 rows of TROW): gz 32, h2 64, ga2 64, h1 64, ga1 64, x 96
constexpr int TB_GZ = 0, TB_H2 = TB_GZ + 32, TB_GA2 = TB_H2 + 64, TB_H1 = TB_GA2 + 64, TB_GA1 = TB_H1 + 64,
              TB_X = TB_GA1 + 64, TB_ROWS = TB_X + 96;

__device__ __forceinline__ float warp_f32(float v, int k) { return __shfl_xor(v, k, 64); }

__global__ __launch_bounds__(64 * kTrainBWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_prop_grad_bf16(
    const TrainArgs a) {
  __shared__ uint4 s_w[FB_N * 64];
  __shared__ __align__(16) __bf16 s_t[kTrainBWaves][TB_ROWS * TROW];
  __shared__ float s_b[PH + PH + PB];
  const float* __restrict__ P = a.params;
  // weight fragments in the operand order of each product
  for (int e = threadIdx.x; e < FB_N * 64; e += blockDim.x) {
    const int blk = e >> 6, ln = e & 63, i = ln & 31, h = ln >> 5;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float x = 0.0f;
      if (blk < FB_W2) {                      // W1: block mt * 5 + kb, natural k order
        const int mt = blk / PKX, kb = blk - mt * PKX, k = 16 * kb + 8 * h + q;
        x = k < PIN ? P[P_W1 + (32 * mt + i) * PIN + k] : 0.0f;
      } else if (blk < FB_W3) {               // W2: block mt * 4 + kb, chained k order
        const int b = blk - FB_W2, mt = b >> 2, kb = b & 3;
        x = P[P_W2 + (32 * mt + i) * PH + chain_row(kb, h, q)];
      } else if (blk < FB_W3T) {              // W3: block kb
        const int kb = blk - FB_W3;
        x = P[P_W3 + i * PH + chain_row(kb, h, q)];
      } else if (blk < FB_W2T) {              // W3^T: block mt * 2 + kb (rows hidden, k bins)
        const int b = blk - FB_W3T, mt = b >> 1, kb = b & 1;
        x = P[P_W3 + chain_row(kb, h, q) * PH + 32 * mt + i];
      } else {                                // W2^T: block mt * 4 + kb (rows h1 units, k h2 units)
        const int b = blk - FB_W2T, mt = b >> 2, kb = b & 3;
        x = P[P_W2 + chain_row(kb, h, q) * PH + 32 * mt + i];
      }
      v[q] = x;
    }
    uint4 u;
    u.x = pack2_bf16(v[0], v[1]); u.y = pack2_bf16(v[2], v[3]);
    u.z = pack2_bf16(v[4], v[5]); u.w = pack2_bf16(v[6], v[7]);
    s_w[e] = u;
  }
  for (int e = threadIdx.x; e < PH + PH + PB; e += blockDim.x)
    s_b[e] = e < PH ? P[P_B1 + e] : (e < 2 * PH ? P[P_B2 + e - PH] : P[P_B3 + e - 2 * PH]);
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 31, h = lane >> 5;
  const int wave = blockIdx.x * kTrainBWaves + wv;
  if (wave >= a.n_waves) return;   // no barrier follows
  __bf16* tab = s_t[wv];
  const float scale = 2.0f / (float)a.batch;
  pf32x16 dw1[2][3], dw2[2][2], dw3[2];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int nt = 0; nt < 3; ++nt) dw1[mt][nt][r] = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) dw2[mt][nt][r] = 0.0f;
      dw3[mt][r] = 0.0f;
    }
  }
  float db2[2][16], db3[16], lsum = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) { db2[0][r] = db2[1][r] = 0.0f; db3[r] = 0.0f; }
  for (int tt = 0; tt < kTrainBTiles; ++tt) {
    const int rb = (wave * kTrainBTiles + tt) * 32 + n;   // position in the batch
    const bool valid = rb < a.batch;
    const long ray = ((long)a.first + (valid ? rb : 0)) % a.n_rays;
    const float4 o = a.ray_o[ray], d = a.ray_d[ray];
    // encoding entries 16 kb + 8 h + q of this ray; the same entries into the x table
    pbf16x8 xb[PKX];
    {
      float sn[2][3][6], cs[2][3][6];
      const float oc[2][3] = {{o.x, o.y, o.z}, {d.x, d.y, d.z}};
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int l = 0; l < 6; ++l) sincospif(ldexpf(oc[s2][c], l), &sn[s2][c][l], &cs[s2][c][l]);
#pragma unroll
      for (int kb = 0; kb < PKX; ++kb) {
        float xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float v0 = 0.0f, v1 = 0.0f;       // entry for half 0 and half 1
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int k = 16 * kb + 8 * hh + q;
            float x;
            if (k == PIN) x = 1.0f;
            else if (k > PIN) x = 0.0f;
            else {
              const int s2 = k >= PENC, e = s2 ? k - PENC : k;
              if (e < 3) x = oc[s2][e];
              else {
                const int qq = e - 3, l = qq / 6, rr = qq % 6, c = rr % 3;
                x = rr < 3 ? sn[s2][c][l] : cs[s2][c][l];
              }
            }
            if (hh == 0) v0 = x; else v1 = x;
          }
          xv[q] = valid ? (h ? v1 : v0) : 0.0f;
        }
        uint4 u;
        u.x = pack2_bf16(xv[0], xv[1]); u.y = pack2_bf16(xv[2], xv[3]);
        u.z = pack2_bf16(xv[4], xv[5]); u.w = pack2_bf16(xv[6], xv[7]);
        xb[kb] = __builtin_bit_cast(pbf16x8, u);
#pragma unroll
        for (int q = 0; q < 8; ++q) tab[(TB_X + 16 * kb + 8 * h + q) * TROW + n] = xb[kb][q];
      }
#pragma unroll
      for (int r = PX; r < 96; ++r)
        if (h == 0) tab[(TB_X + r) * TROW + n] = (__bf16)0.0f;
    }
    // forward
    pf32x16 s1[2], s2v[2], z;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s1[mt][r] = s_b[32 * mt + tile_row(r, h)];
#pragma unroll
      for (int kb = 0; kb < PKX; ++kb)
        s1[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, s_w[(FB_W1 + mt * PKX + kb) * 64 + lane]),
                                                         xb[kb], s1[mt], 0, 0, 0);
    }
    pf32x16 h1[2];
    pbf16x8 h1b[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) h1[mt][r] = fmaxf(s1[mt][r], 0.0f);
      tile_operands_bf16(h1[mt], h1b[2 * mt], h1b[2 * mt + 1]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s2v[mt][r] = s_b[PH + 32 * mt + tile_row(r, h)];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        s2v[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, s_w[(FB_W2 + mt * 4 + kb) * 64 + lane]),
                                                          h1b[kb], s2v[mt], 0, 0, 0);
    }
    pf32x16 h2[2];
    pbf16x8 h2b[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) h2[mt][r] = fmaxf(s2v[mt][r], 0.0f);
      tile_operands_bf16(h2[mt], h2b[2 * mt], h2b[2 * mt + 1]);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = s_b[2 * PH + tile_row(r, h)];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, s_w[(FB_W3 + kb) * 64 + lane]), h2b[kb], z,
                                                  0, 0, 0);
    // softmax over the 32 bins of column n, loss and dL/dz
    float m = -INFINITY;
#pragma unroll
    for (int r = 0; r < 16; ++r) m = fmaxf(m, z[r]);
    m = fmaxf(m, warp_f32(m, 32));
    float sum = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) { z[r] = expf(z[r] - m); sum += z[r]; }
    sum += warp_f32(sum, 32);
    const float inv = 1.0f / sum;
    float tg[16];
    {
      const float4* tp = reinterpret_cast<const float4*>(a.target + ray * PB);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 t4 = tp[2 * g + h];
        tg[4 * g] = t4.x; tg[4 * g + 1] = t4.y; tg[4 * g + 2] = t4.z; tg[4 * g + 3] = t4.w;
      }
    }
    float pg = 0.0f, sq = 0.0f;
    pf32x16 gz;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float p = z[r] * inv;
      const float diff = p - tg[r];
      sq += diff * diff;
      gz[r] = scale * diff;          // dL/dp
      z[r] = p;
      pg += p * gz[r];
    }
    pg += warp_f32(pg, 32);
#pragma unroll
    for (int r = 0; r < 16; ++r) gz[r] = valid ? z[r] * (gz[r] - pg) : 0.0f;
    if (valid) lsum += sq;
    // backward through the layers
    pbf16x8 gzb[2];
    tile_operands_bf16(gz, gzb[0], gzb[1]);
    pf32x16 ga2[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) ga2[mt][r] = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
        ga2[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, s_w[(FB_W3T + mt * 2 + kb) * 64 + lane]),
                                                          gzb[kb], ga2[mt], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) ga2[mt][r] = s2v[mt][r] > 0.0f ? ga2[mt][r] : 0.0f;
    }
    pbf16x8 ga2b[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) tile_operands_bf16(ga2[mt], ga2b[2 * mt], ga2b[2 * mt + 1]);
    pf32x16 ga1[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) ga1[mt][r] = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        ga1[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, s_w[(FB_W2T + mt * 4 + kb) * 64 + lane]),
                                                          ga2b[kb], ga1[mt], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) ga1[mt][r] = s1[mt][r] > 0.0f ? ga1[mt][r] : 0.0f;
    }
    // bias gradients of layers 2 and 3 on the vector ALU (this lane's column)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      db3[r] += gz[r];
      db2[0][r] += ga2[0][r];
      db2[1][r] += ga2[1][r];
    }
    // the tile's tables, then dW = G H^T over the tile's 32 rays
    tile_to_table(gz, tab, TB_GZ, n, h);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      tile_to_table(h2[mt], tab, TB_H2 + 32 * mt, n, h);
      tile_to_table(ga2[mt], tab, TB_GA2 + 32 * mt, n, h);
      tile_to_table(h1[mt], tab, TB_H1 + 32 * mt, n, h);
      tile_to_table(ga1[mt], tab, TB_GA1 + 32 * mt, n, h);
    }
    prop_wave_sync();
    const int i = n;   // operand row of this lane
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const pbf16x8 agz = table_operand(tab, TB_GZ + i, kb, h);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        dw3[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(agz, table_operand(tab, TB_H2 + 32 * nt + i, kb, h), dw3[nt],
                                                          0, 0, 0);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const pbf16x8 aga2 = table_operand(tab, TB_GA2 + 32 * mt + i, kb, h);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
          dw2[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aga2, table_operand(tab, TB_H1 + 32 * nt + i, kb, h),
                                                                dw2[mt][nt], 0, 0, 0);
        const pbf16x8 aga1 = table_operand(tab, TB_GA1 + 32 * mt + i, kb, h);
#pragma unroll
        for (int nt = 0; nt < 3; ++nt)
          dw1[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aga1, table_operand(tab, TB_X + 32 * nt + i, kb, h),
                                                                dw1[mt][nt], 0, 0, 0);
      }
    }
    prop_wave_sync();   // the next tile overwrites the tables
  }
  // bias sums over the 32 columns of each half, fixed butterfly order
#pragma unroll
  for (int r = 0; r < 16; ++r) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      db3[r] += __shfl_xor(db3[r], o, 32);
      db2[0][r] += __shfl_xor(db2[0][r], o, 32);
      db2[1][r] += __shfl_xor(db2[1][r], o, 32);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  // partial gradient in parameter order: accumulator (row 8 (v / 4) + 4 h +
  // v % 4, column n) of tile (mt, nt) is dW[32 mt + row][32 nt + n]
  float* out = a.partial + (long)wave * P_N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = tile_row(r, h);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int u = 32 * mt + row;
#pragma unroll
      for (int nt = 0; nt < 3; ++nt) {
        const int k = 32 * nt + n;
        if (k < PIN) out[P_W1 + u * PIN + k] = dw1[mt][nt][r];
        else if (k == PIN) out[P_B1 + u] = dw1[mt][nt][r];
      }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) out[P_W2 + u * PH + 32 * nt + n] = dw2[mt][nt][r];
      if (n == 0) out[P_B2 + u] = db2[mt][r];
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) out[P_W3 + row * PH + 32 * nt + n] = dw3[nt][r];
    if (n == 0) out[P_B3 + row] = db3[r];
  }
  if (lane == 0) a.loss_partial[wave] = lsum;
}

hipError_t launch_prop_grad_bf16(const TrainArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_prop_grad_bf16, dim3((a.n_waves + kTrainBWaves - 1) / kTrainBWaves), dim3(64 * kTrainBWaves),
                     0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prop_reduce, dim3((P_N + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

int prop_rays_per_wave_bf16() { return 32 * kTrainBTiles; }

// ---------------------------------------------------------------------------
__global__ void k_rays_to_f4(const float* o3, const float* d3, int n, float4* o4, float4* d4) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  o4[r] = make_float4(o3[3 * r], o3[3 * r + 1], o3[3 * r + 2], 0.0f);
  d4[r] = make_float4(d3[3 * r], d3[3 * r + 1], d3[3 * r + 2], 0.0f);
}
__global__ void k_rays_from_f4(const float4* o4, const float4* d4, int n, float* o3, float* d3) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float4 o = o4[r], d = d4[r];
  o3[3 * r] = o.x; o3[3 * r + 1] = o.y; o3[3 * r + 2] = o.z;
  d3[3 * r] = d.x; d3[3 * r + 1] = d.y; d3[3 * r + 2] = d.z;
}

hipError_t launch_rays_to_f4(const float* o3, const float* d3, int n, float4* o4, float4* d4, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rays_to_f4, dim3((n + 255) / 256), dim3(256), 0, st, o3, d3, n, o4, d4);
  return hipGetLastError();
}
hipError_t launch_rays_from_f4(const float4* o4, const float4* d4, int n, float* o3, float* d3, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rays_from_f4, dim3((n + 255) / 256), dim3(256), 0, st, o4, d4, n, o3, d3);
  return hipGetLastError();
}

}  // namespace fl
