// Training of the 4x64 map with the photometric loss of Eq. 2 (mean over the
// rays of a batch of |C_hat(r) - C(r)|^2, C_hat the coarse render of Eq. 1
// with stratified samples keyed (ray, 0)): gradient by the chain rule through
// the quadrature and the network, per-wave partial gradients, a fixed-order
// reduction, and Adam on float32 master weights.
//
// One wave handles a ray at a time.  Forward: the S samples in turn, hidden
// unit j on lane j, the vector a layer reads broadcast lane by lane
// (v_readlane), weights in LDS with a padded row stride so that reading a row
// (forward) and a column (backward) are both free of bank conflicts; sample k
// keeps sigma_k and c_k on lane k.  Compositing: one wave scan over the
// samples gives w_k, T_k, C_hat and, with the suffix sums of w_m c_m,
//   dL/dc_k = w_k gC,   dL/dsigma_k = delta_k gC . (T_{k+1} c_k - sum_{m>k} w_m c_m),
// gC = 2 (C_hat - C) / batch.  Backward: each sample's forward is recomputed
// and its gradient rows accumulate in registers (lane j owns row j of every
// hidden weight matrix; two passes, see k_map_grad).  Canonical parameter order as the map description:
// W0 (64 x 39), b0, W1, b1, W2, b2, W3, b3 (64 x 64 each), w_s (1 x 64), b_s,
// W_c (3 x 79), b_c.
#include "bf16_tiles.h"
#include "common.h"
#include "kernels.h"

namespace fl {

namespace tm {
constexpr int H = 64, IX = 39, ID = 15, IC = H + ID;
constexpr int W0 = 0, B0 = W0 + H * IX, W1 = B0 + H, B1 = W1 + H * H, W2 = B1 + H, B2 = W2 + H * H;
constexpr int W3 = B2 + H, B3 = W3 + H * H, WS = B3 + H, BS = WS + H, WC = BS + 1, BC = WC + 3 * IC, N = BC + 3;
static_assert(N == kSmallMapParams, "4x64 map layout");
constexpr int RS = H + 1;                               // padded row stride of the 64 x 64 matrices in LDS
}  // namespace tm


__device__ __forceinline__ float tm_bcast(float v, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

__device__ __forceinline__ float tm_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// inclusive scan over the 64 lanes
__device__ __forceinline__ float tm_scan(float v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// entry f of gamma_L(p), canonical order (p, sin 2^0 pi p, cos 2^0 pi p, ...)
__device__ __forceinline__ float tm_feature(float p0, float p1, float p2, int f) {
  if (f < 3) return f == 0 ? p0 : (f == 1 ? p1 : p2);
  const int q = f - 3, l = q / 6, r = q % 6, c = r % 3;
  const float x = c == 0 ? p0 : (c == 1 ? p1 : p2);
  float s, co;
  sincospif(ldexpf(x, l), &s, &co);
  return r < 3 ? s : co;
}

// the map in LDS: W0 (row stride 39, odd), W1..W3 with row stride 65, then
// the biases and heads
struct TmLds {
  float w0[tm::H * tm::IX];
  float wh[3][tm::H * tm::RS];
  float b[4][tm::H];
  float ws[tm::H];
  float wc[3 * tm::IC];
  float bc[3];
  float bs;
};

__device__ __forceinline__ float lwh(const TmLds& L, int m, int j, int k) { return L.wh[m][j * tm::RS + k]; }

// one sample's forward pass; lane j holds unit j of every layer
struct TmFwd {
  float h0, h1, h2, h3;
  float gx;                      // gamma(x) entry `lane` (lanes < 39)
  float zs, zc[3];               // head inputs (uniform)
};

__device__ __forceinline__ TmFwd tm_forward(const TmLds& L, const float4 o, const float4 d, const float t,
                                            const float gd, const int lane) {
  TmFwd r;
  const float x0 = fmaf(t, d.x, o.x), x1 = fmaf(t, d.y, o.y), x2 = fmaf(t, d.z, o.z);
  r.gx = lane < tm::IX ? tm_feature(x0, x1, x2, lane) : 0.0f;
  float s = L.b[0][lane];
  for (int f = 0; f < tm::IX; ++f) s = fmaf(L.w0[lane * tm::IX + f], tm_bcast(r.gx, f), s);
  r.h0 = fmaxf(s, 0.0f);
  s = L.b[1][lane];
  for (int k = 0; k < tm::H; ++k) s = fmaf(lwh(L, 0, lane, k), tm_bcast(r.h0, k), s);
  r.h1 = fmaxf(s, 0.0f);
  s = L.b[2][lane];
  for (int k = 0; k < tm::H; ++k) s = fmaf(lwh(L, 1, lane, k), tm_bcast(r.h1, k), s);
  r.h2 = fmaxf(s, 0.0f);
  s = L.b[3][lane];
  for (int k = 0; k < tm::H; ++k) s = fmaf(lwh(L, 2, lane, k), tm_bcast(r.h2, k), s);
  r.h3 = fmaxf(s, 0.0f);
  r.zs = tm_wave_sum(L.ws[lane] * r.h3) + L.bs;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v = L.wc[c * tm::IC + lane] * r.h3;
    if (lane < tm::ID) v = fmaf(L.wc[c * tm::IC + tm::H + lane], gd, v);
    r.zc[c] = tm_wave_sum(v) + L.bc[c];
  }
  return r;
}

__device__ __forceinline__ float tm_softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float tm_sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

constexpr int kTmWaves = 4;

// The gradient rows of all four hidden matrices do not fit in one wave's
// registers, so the work runs in two passes over the same rays (each
// recomputes the forward pass and the compositing): pass 0 accumulates the
// heads, W3, b3, W2, b2 and the loss; pass 1 W1, b1, W0, b0.
template <int PASS>
__global__ __launch_bounds__(64 * kTmWaves) void k_map_grad(const MapTrainArgs a) {
  __shared__ TmLds L;
  for (int i = threadIdx.x; i < tm::H * tm::IX; i += blockDim.x) L.w0[i] = a.params[tm::W0 + i];
  for (int i = threadIdx.x; i < 3 * tm::H * tm::H; i += blockDim.x) {
    const int m = i / (tm::H * tm::H), r = (i / tm::H) % tm::H, k = i % tm::H;
    L.wh[m][r * tm::RS + k] = a.params[(m == 0 ? tm::W1 : (m == 1 ? tm::W2 : tm::W3)) + r * tm::H + k];
  }
  for (int i = threadIdx.x; i < tm::H; i += blockDim.x) {
    L.b[0][i] = a.params[tm::B0 + i];
    L.b[1][i] = a.params[tm::B1 + i];
    L.b[2][i] = a.params[tm::B2 + i];
    L.b[3][i] = a.params[tm::B3 + i];
    L.ws[i] = a.params[tm::WS + i];
  }
  for (int i = threadIdx.x; i < 3 * tm::IC; i += blockDim.x) L.wc[i] = a.params[tm::WC + i];
  if (threadIdx.x < 3) L.bc[threadIdx.x] = a.params[tm::BC + threadIdx.x];
  if (threadIdx.x == 0) L.bs = a.params[tm::BS];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kTmWaves + (threadIdx.x >> 6);
  if (wave >= a.n_waves) return;   // the partial buffers hold n_waves rows (no barrier follows)
  const int S = a.S;
  const float scale = 2.0f / (float)a.batch;

  // pass 0: gA = W3 rows, gB = W2 rows; pass 1: gA = W1 rows, gB = W0 rows
  constexpr int NB = PASS == 0 ? tm::H : tm::IX;
  float gA[tm::H], gB[NB];
#pragma unroll
  for (int k = 0; k < tm::H; ++k) gA[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < NB; ++k) gB[k] = 0.0f;
  float gbA = 0.0f, gbB = 0.0f, gws = 0.0f, gbs = 0.0f;
  float gWc[3] = {0.0f, 0.0f, 0.0f}, gWd[3] = {0.0f, 0.0f, 0.0f}, gbc[3] = {0.0f, 0.0f, 0.0f};
  float lsum = 0.0f;

  for (int q = 0; q < a.rays_per_wave; ++q) {
    const int rb = wave * a.rays_per_wave + q;           // position in the batch
    if (rb >= a.batch) break;
    const long ray = ((long)a.first + rb) % a.n_rays;
    const float4 o = a.ray_o[ray], d = a.ray_d[ray];
    const uint32_t key = (uint32_t)ray;
    // lane k: stratified depth of sample k (streams keyed (ray, 0))
    float t_l = 0.0f;
    if (lane < S) {
      float xi = 0.0f;
      if (a.jitter) xi = unit24(pick(draw(a.seed, a.iter, kStreamJitCoarse, key, 0, lane >> 2), lane & 3));
      t_l = a.near_ + ((float)lane + xi) * a.dt;
    }
    const float gd = lane < tm::ID ? tm_feature(d.x, d.y, d.z, lane) : 0.0f;
    // forward over the samples; lane k keeps sigma_k, c_k
    float sig_l = 0.0f, c_l[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < S; ++k) {
      const TmFwd f = tm_forward(L, o, d, tm_bcast(t_l, k), gd, lane);
      if (lane == k) {
        sig_l = tm_softplus(f.zs);
#pragma unroll
        for (int c = 0; c < 3; ++c) c_l[c] = tm_sigmoid(f.zc[c]);
      }
    }
    // quadrature of Eq. 1 over lanes 0..S-1
    const bool on = lane < S;
    const float t_next = __shfl_down(t_l, 1, 64);
    const float delta = on ? (lane + 1 < S ? t_next - t_l : a.far_ - t_l) : 0.0f;
    const float tau = on ? sig_l * delta : 0.0f;
    const float incl = tm_scan(tau, lane);
    const float T_k = expf(-(incl - tau));
    const float T_k1 = expf(-incl);
    const float wk = on ? T_k * (-expm1f(-tau)) : 0.0f;
    float gC[3], wc[3], sfx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      wc[c] = wk * c_l[c];
      const float tot = tm_wave_sum(wc[c]);
      sfx[c] = tot - tm_scan(wc[c], lane);
      const float err = tot - a.target[ray * 3 + c];
      lsum += err * err;
      gC[c] = scale * err;
    }
    float dsig = 0.0f, dc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dsig = fmaf(gC[c], T_k1 * c_l[c] - sfx[c], dsig);
      dc[c] = wk * gC[c];
    }
    dsig *= delta;
    // backward, one sample at a time (forward recomputed)
    for (int k = 0; k < S; ++k) {
      const TmFwd f = tm_forward(L, o, d, tm_bcast(t_l, k), gd, lane);
      const float dzs = tm_bcast(dsig, k) * tm_sigmoid(f.zs);
      float dzc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float cc = tm_sigmoid(f.zc[c]);
        dzc[c] = tm_bcast(dc[c], k) * cc * (1.0f - cc);
      }
      float da = dzs * L.ws[lane];
#pragma unroll
      for (int c = 0; c < 3; ++c) da = fmaf(dzc[c], L.wc[c * tm::IC + lane], da);
      if constexpr (PASS == 0) {
        // heads
        gws = fmaf(dzs, f.h3, gws);
        gbs += dzs;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gWc[c] = fmaf(dzc[c], f.h3, gWc[c]);
          gWd[c] = fmaf(dzc[c], gd, gWd[c]);
          gbc[c] += dzc[c];
        }
      }
      // layer 3 (input h2)
      float dz = f.h3 > 0.0f ? da : 0.0f;
      if constexpr (PASS == 0) {
        gbA += dz;
#pragma unroll
        for (int k2 = 0; k2 < tm::H; ++k2) gA[k2] = fmaf(dz, tm_bcast(f.h2, k2), gA[k2]);
      }
      da = 0.0f;
      for (int j = 0; j < tm::H; ++j) da = fmaf(lwh(L, 2, j, lane), tm_bcast(dz, j), da);
      // layer 2 (input h1)
      dz = f.h2 > 0.0f ? da : 0.0f;
      if constexpr (PASS == 0) {
        gbB += dz;
#pragma unroll
        for (int k2 = 0; k2 < tm::H; ++k2) gB[k2] = fmaf(dz, tm_bcast(f.h1, k2), gB[k2]);
        continue;
      }
      da = 0.0f;
      for (int j = 0; j < tm::H; ++j) da = fmaf(lwh(L, 1, j, lane), tm_bcast(dz, j), da);
      // layer 1 (input h0)
      dz = f.h1 > 0.0f ? da : 0.0f;
      gbA += dz;
#pragma unroll
      for (int k2 = 0; k2 < tm::H; ++k2) gA[k2] = fmaf(dz, tm_bcast(f.h0, k2), gA[k2]);
      da = 0.0f;
      for (int j = 0; j < tm::H; ++j) da = fmaf(lwh(L, 0, j, lane), tm_bcast(dz, j), da);
      // layer 0 (input gamma(x))
      dz = f.h0 > 0.0f ? da : 0.0f;
      gbB += dz;
#pragma unroll
      for (int f2 = 0; f2 < NB; ++f2) gB[f2] = fmaf(dz, tm_bcast(f.gx, f2), gB[f2]);
    }
  }
  // per-wave partials in parameter order
  float* out = a.partial + (long)wave * tm::N;
  if constexpr (PASS == 0) {
#pragma unroll
    for (int k = 0; k < tm::H; ++k) {
      out[tm::W3 + lane * tm::H + k] = gA[k];
      out[tm::W2 + lane * tm::H + k] = gB[k];
    }
    out[tm::B3 + lane] = gbA;
    out[tm::B2 + lane] = gbB;
    out[tm::WS + lane] = gws;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[tm::WC + c * tm::IC + lane] = gWc[c];
      if (lane < tm::ID) out[tm::WC + c * tm::IC + tm::H + lane] = gWd[c];
    }
    if (lane == 0) {
      out[tm::BS] = gbs;
#pragma unroll
      for (int c = 0; c < 3; ++c) out[tm::BC + c] = gbc[c];
      a.loss_partial[wave] = lsum;
    }
  } else {
#pragma unroll
    for (int k = 0; k < tm::H; ++k) out[tm::W1 + lane * tm::H + k] = gA[k];
#pragma unroll
    for (int k = 0; k < NB; ++k) out[tm::W0 + lane * tm::IX + k] = gB[k];
    out[tm::B1 + lane] = gbA;
    out[tm::B0 + lane] = gbB;
  }
}

// ---------------------------------------------------------------------------
// The same gradient in bfloat16 on the matrix cores (v_mfma_f32_32x32x16_bf16,
// float32 accumulation) for 32 samples per ray: a wave takes one ray at a
// time as a tile of 32 sample columns (lane (n, h) holds sample n; layouts
// of bf16_tiles.h).  Forward and the backward pass through the layers run
// transposed, out^T = W in^T: the encoding gamma(x) enters in natural order
// (k-row 16 kb + 8 h + q, padded to 48 with x_39 = 1, the bias column of
// dW0), the hidden activations chained, the head tile's rows are sigma, r,
// g, b (then zeros) over [h3, gamma(d)] with gamma(d) padded to 16 by a 1
// whose weight is zero (and whose column of dW_head is the head biases'
// gradient).  The compositing gradient is the float32 kernel's, on the lanes
// of half 0.  The weight gradients contract over the samples: activations,
// output gradients and the encodings go through per-wave LDS tables
// [row][sample], and dW = G H^T accumulates in registers over the wave's
// rays; db1..db3 come from the same tables against a column of ones, into
// LDS.  Each wave writes its partial gradient in parameter order.
namespace tmb {
constexpr int WAVES = 4;
constexpr int XK = 3;                                    // k-blocks of gamma(x) (48 rows)
// weight fragments (1 KB blocks) in LDS; pass 0 stages the blocks before
// F_W2T, pass 1 all
constexpr int F_W0 = 0, F_W1 = F_W0 + 2 * XK, F_W2 = F_W1 + 8, F_W3 = F_W2 + 8, F_WH = F_W3 + 8,
              F_W3T = F_WH + 5, F_WHT = F_W3T + 8, F_W2T = F_WHT + 2, F_W1T = F_W2T + 8, F_N = F_W1T + 8;
__host__ __device__ constexpr int f_wt(int l) { return l == 3 ? F_W3T : (l == 2 ? F_W2T : F_W1T); }
template <int PASS>
constexpr int frag_blocks() { return PASS == 0 ? F_W2T : F_N; }
// per-wave tables (rows of kTabRow bf16) of a pass; -1: not kept.  Pass 0:
// h1, h2, h3, the output gradient of the current layer, the head gradient
// (4 rows and a zero row), gamma(d) (15 rows, a row of ones, a zero row).
// Pass 1: gamma(x) (48 rows and a zero row), h0, the output gradient.
template <int PASS>
struct Tab;
template <>
struct Tab<0> {
  static constexpr int X = -1, H0 = -1, H1 = 0, H2 = 64, H3 = 128, DZ = 192, G = 256, D = 261, ROWS = 278;
};
template <>
struct Tab<1> {
  static constexpr int X = 0, H0 = 49, H1 = -1, H2 = -1, H3 = -1, DZ = 113, G = -1, D = -1, ROWS = 177;
};
template <int PASS>
__host__ __device__ constexpr int tab_h(int l) {
  return l == 0 ? Tab<PASS>::H0 : (l == 1 ? Tab<PASS>::H1 : (l == 2 ? Tab<PASS>::H2 : Tab<PASS>::H3));
}
}  // namespace tmb

__device__ __forceinline__ pf32x16 tmb_zero() {
  pf32x16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.0f;
  return z;
}

__device__ __forceinline__ pf32x16 tmb_mfma(const uint4& a, const pbf16x8& b, const pf32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, a), b, c, 0, 0, 0);
}

// ReLU'd output gradient of tile mt: da where the layer's activation was
// positive (bit 16 mt + v of the layer's mask)
__device__ __forceinline__ pf32x16 tmb_mask(const pf32x16& da, const uint32_t mask, const int mt) {
  pf32x16 dz;
#pragma unroll
  for (int v = 0; v < 16; ++v) dz[v] = (mask >> (16 * mt + v)) & 1u ? da[v] : 0.0f;
  return dz;
}

template <int PASS>
__global__ __launch_bounds__(64 * tmb::WAVES) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_map_grad_bf16(
    const MapTrainArgs a) {
  using namespace tmb;
  using T = Tab<PASS>;
  constexpr int FN = frag_blocks<PASS>();
  __shared__ uint4 s_w[FN * 64];
  __shared__ __align__(16) __bf16 s_t[WAVES][T::ROWS * kTabRow];
  __shared__ float s_b[4 * tm::H + 4];
  __shared__ float s_db[WAVES][3 * tm::H];
  const float* __restrict__ P = a.params;
  // weight fragments in the operand order of each product: lane (m, h) of
  // block holds A[m][k] for its eight k of k-block kb
  for (int e = threadIdx.x; e < FN * 64; e += blockDim.x) {
    const int blk = e >> 6, ln = e & 63, m = ln & 31, h = ln >> 5;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float x = 0.0f;
      if (blk < F_W1) {                          // W0: block mt * 3 + kb, natural k
        const int mt = blk / XK, kb = blk - mt * XK, k = 16 * kb + 8 * h + q;
        x = k < tm::IX ? P[tm::W0 + (32 * mt + m) * tm::IX + k] : 0.0f;
      } else if (blk < F_WH) {                   // W1..W3: block mt * 4 + kb, chained k
        const int b = blk - F_W1, l = b >> 3, mt = (b >> 2) & 1, kb = b & 3;
        x = P[tm::W1 + l * (tm::H * tm::H + tm::H) + (32 * mt + m) * tm::H + chain_row(kb, h, q)];
      } else if (blk < F_W3T) {                  // head: kb 0..3 chained h3, kb 4 gamma(d) natural
        const int kb = blk - F_WH;
        if (m < 4) {
          if (kb < 4) {
            const int u = chain_row(kb, h, q);
            x = m == 0 ? P[tm::WS + u] : P[tm::WC + (m - 1) * tm::IC + u];
          } else {
            const int k = 8 * h + q;
            x = (m > 0 && k < tm::ID) ? P[tm::WC + (m - 1) * tm::IC + tm::H + k] : 0.0f;
          }
        }
      } else if (blk >= F_WHT && blk < F_W2T) {  // head^T: rows = h3 units, natural k = head rows
        const int mt = blk - F_WHT, k = 8 * h + q, u = 32 * mt + m;
        if (k == 0) x = P[tm::WS + u];
        else if (k < 4) x = P[tm::WC + (k - 1) * tm::IC + u];
      } else {                                   // W3^T, W2^T, W1^T: rows = input units, chained k = output units
        const int l = blk < F_WHT ? 3 : (blk < F_W1T ? 2 : 1);
        const int b = blk - f_wt(l), mt = b >> 2, kb = b & 3;
        x = P[tm::W1 + (l - 1) * (tm::H * tm::H + tm::H) + chain_row(kb, h, q) * tm::H + 32 * mt + m];
      }
      v[q] = x;
    }
    uint4 u;
    u.x = pack2_bf16(v[0], v[1]); u.y = pack2_bf16(v[2], v[3]);
    u.z = pack2_bf16(v[4], v[5]); u.w = pack2_bf16(v[6], v[7]);
    s_w[e] = u;
  }
  for (int e = threadIdx.x; e < 4 * tm::H + 4; e += blockDim.x) {
    float x;
    if (e < 4 * tm::H) {
      const int l = e / tm::H, j = e - l * tm::H;
      x = P[(l == 0 ? tm::B0 : tm::B1 + (l - 1) * (tm::H * tm::H + tm::H)) + j];
    } else {
      const int r = e - 4 * tm::H;
      x = r == 0 ? P[tm::BS] : P[tm::BC + r - 1];
    }
    s_b[e] = x;
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 31, h = lane >> 5;
  __bf16* tab = s_t[wv];
  for (int e = lane; e < 3 * tm::H; e += 64) s_db[wv][e] = 0.0f;
  // constant rows: the zero rows and gamma(d)'s row of ones
  if (h == 0) {
    if constexpr (PASS == 1) {
      tab[(T::X + 48) * kTabRow + n] = (__bf16)0.0f;
    } else {
      tab[(T::G + 4) * kTabRow + n] = (__bf16)0.0f;
      tab[(T::D + 15) * kTabRow + n] = (__bf16)1.0f;
      tab[(T::D + 16) * kTabRow + n] = (__bf16)0.0f;
    }
  }
  __syncthreads();
  const int wave = blockIdx.x * WAVES + wv;
  if (wave >= a.n_waves) return;   // no barrier follows
  const float scale = 2.0f / (float)a.batch;

  pf32x16 dw0[2][2], dw[3][2][2], dwh[3];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      dw0[mt][nt] = tmb_zero();
#pragma unroll
      for (int l = 0; l < 3; ++l) dw[l][mt][nt] = tmb_zero();
    }
#pragma unroll
  for (int nt = 0; nt < 3; ++nt) dwh[nt] = tmb_zero();
  float lsum = 0.0f;
  pbf16x8 ones;
#pragma unroll
  for (int q = 0; q < 8; ++q) ones[q] = (__bf16)1.0f;

  for (int q0 = 0; q0 < a.rays_per_wave; ++q0) {
    const int rb = wave * a.rays_per_wave + q0;   // position in the batch
    if (rb >= a.batch) break;
    const long ray = ((long)a.first + rb) % a.n_rays;
    const float4 o = a.ray_o[ray], d = a.ray_d[ray];
    // sample n of the ray (streams keyed (ray, 0), as the float32 kernel)
    float xi = 0.0f;
    if (a.jitter) xi = unit24(pick(draw(a.seed, a.iter, kStreamJitCoarse, (uint32_t)ray, 0, n >> 2), n & 3));
    const float t = a.near_ + ((float)n + xi) * a.dt;
    // gamma(x) operands (k-row 16 kb + 8 h + q) and their table rows
    pbf16x8 xb[XK];
    {
      const float pc[3] = {fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z)};
      float sn[3][6], cs[3][6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // band 0 by sincospif, band l + 1 from band l by the double-angle
        // identities (each doubling at most doubles the absolute error:
        // within 2^5 float32 roundings at band 5, far inside bf16 rounding)
        sincospif(pc[c], &sn[c][0], &cs[c][0]);
#pragma unroll
        for (int l = 1; l < 6; ++l) {
          const float sa = sn[c][l - 1], ca = cs[c][l - 1];
          sn[c][l] = 2.0f * sa * ca;
          cs[c][l] = (ca - sa) * (ca + sa);
        }
      }
#pragma unroll
      for (int kb = 0; kb < XK; ++kb) {
        float xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float x0 = 0.0f, x1 = 0.0f;
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int k = 16 * kb + 8 * hh + q;
            float x = 0.0f;
            if (k < 3) x = pc[k];
            else if (k < tm::IX) {
              const int qq = k - 3, l = qq / 6, rr = qq % 6, c = rr % 3;
              x = rr < 3 ? sn[c][l] : cs[c][l];
            } else if (k == tm::IX) {
              x = 1.0f;
            }
            if (hh == 0) x0 = x; else x1 = x;
          }
          xv[q] = h ? x1 : x0;
        }
        uint4 u;
        u.x = pack2_bf16(xv[0], xv[1]); u.y = pack2_bf16(xv[2], xv[3]);
        u.z = pack2_bf16(xv[4], xv[5]); u.w = pack2_bf16(xv[6], xv[7]);
        xb[kb] = __builtin_bit_cast(pbf16x8, u);
        if constexpr (PASS == 1)
#pragma unroll
          for (int q = 0; q < 8; ++q) tab[(T::X + 16 * kb + 8 * h + q) * kTabRow + n] = xb[kb][q];
      }
    }
    // gamma(d) operand (natural k-row 8 h + q; k = 15 holds 1) and table
    pbf16x8 gdb;
    {
      float sd[3][2], cd[3][2];
      const float dc[3] = {d.x, d.y, d.z};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sincospif(dc[c], &sd[c][0], &cd[c][0]);
        sd[c][1] = 2.0f * sd[c][0] * cd[c][0];
        cd[c][1] = (cd[c][0] - sd[c][0]) * (cd[c][0] + sd[c][0]);
      }
      float gv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float x0 = 0.0f, x1 = 0.0f;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int k = 8 * hh + q;
          float x;
          if (k < 3) x = dc[k];
          else if (k < tm::ID) {
            const int qq = k - 3, l = qq / 6, rr = qq % 6, c = rr % 3;
            x = rr < 3 ? sd[c][l] : cd[c][l];
          } else {
            x = 1.0f;
          }
          if (hh == 0) x0 = x; else x1 = x;
        }
        gv[q] = h ? x1 : x0;
      }
      uint4 u;
      u.x = pack2_bf16(gv[0], gv[1]); u.y = pack2_bf16(gv[2], gv[3]);
      u.z = pack2_bf16(gv[4], gv[5]); u.w = pack2_bf16(gv[6], gv[7]);
      gdb = __builtin_bit_cast(pbf16x8, u);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (PASS == 0 && 8 * h + q < tm::ID) tab[(T::D + 8 * h + q) * kTabRow + n] = gdb[q];
    }
    // forward (each layer's activations also into its table)
    pbf16x8 hb[4];   // chained operands of the last layer computed
    uint32_t mk[4];  // ReLU masks of h0..h3: bit 16 mt + v
    {
      pf32x16 s0[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int r = 0; r < 16; ++r) s0[mt][r] = s_b[32 * mt + tile_row(r, h)];
#pragma unroll
        for (int kb = 0; kb < XK; ++kb) s0[mt] = tmb_mfma(s_w[(F_W0 + mt * XK + kb) * 64 + lane], xb[kb], s0[mt]);
#pragma unroll
        for (int r = 0; r < 16; ++r) s0[mt][r] = fmaxf(s0[mt][r], 0.0f);
        tile_operands_bf16(s0[mt], hb[2 * mt], hb[2 * mt + 1]);
        if constexpr (T::H0 >= 0) tile_to_table(s0[mt], tab + T::H0 * kTabRow, 32 * mt, n, h);
      }
      mk[0] = 0u;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) mk[0] |= (s0[mt][r] > 0.0f ? 1u : 0u) << (16 * mt + r);
    }
#pragma unroll
    for (int l = 1; l < 4; ++l) {
      pf32x16 sl[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int r = 0; r < 16; ++r) sl[mt][r] = s_b[l * tm::H + 32 * mt + tile_row(r, h)];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          sl[mt] = tmb_mfma(s_w[(F_W1 + (l - 1) * 8 + mt * 4 + kb) * 64 + lane], hb[kb], sl[mt]);
#pragma unroll
        for (int r = 0; r < 16; ++r) sl[mt][r] = fmaxf(sl[mt][r], 0.0f);
        if (tab_h<PASS>(l) >= 0) tile_to_table(sl[mt], tab + tab_h<PASS>(l) * kTabRow, 32 * mt, n, h);
      }
      mk[l] = 0u;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) mk[l] |= (sl[mt][r] > 0.0f ? 1u : 0u) << (16 * mt + r);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) tile_operands_bf16(sl[mt], hb[2 * mt], hb[2 * mt + 1]);
    }
    pf32x16 z;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = tile_row(r, h);
      z[r] = row < 4 ? s_b[4 * tm::H + row] : 0.0f;
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) z = tmb_mfma(s_w[(F_WH + kb) * 64 + lane], hb[kb], z);
    z = tmb_mfma(s_w[(F_WH + 4) * 64 + lane], gdb, z);
    // compositing (Eq. 1) and its gradient on the lanes of half 0: sample n
    const bool on = h == 0;
    const float zs = z[0], zc[3] = {z[1], z[2], z[3]};
    const float sig = on ? tm_softplus(zs) : 0.0f;
    float cl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) cl[c] = tm_sigmoid(zc[c]);
    const float t_next = __shfl_down(t, 1, 32);
    const float delta = n + 1 < 32 ? t_next - t : a.far_ - t;
    const float tau = sig * delta;
    float incl = tau;
#pragma unroll
    for (int o2 = 1; o2 < 32; o2 <<= 1) {
      const float u = __shfl_up(incl, o2, 32);
      if (n >= o2) incl += u;
    }
    const float T_k = expf(-(incl - tau)), T_k1 = expf(-incl);
    const float wk = on ? T_k * (-expm1f(-tau)) : 0.0f;
    float gC[3], sfx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float wc = wk * cl[c];
      float sc = wc, tot = wc;
#pragma unroll
      for (int o2 = 1; o2 < 32; o2 <<= 1) {
        const float u = __shfl_up(sc, o2, 32);
        if (n >= o2) sc += u;
        tot += __shfl_xor(tot, o2, 32);
      }
      sfx[c] = tot - sc;
      const float err = tot - a.target[ray * 3 + c];
      lsum += err * err;
      gC[c] = scale * err;
    }
    float dsig = 0.0f, dzc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dsig = fmaf(gC[c], T_k1 * cl[c] - sfx[c], dsig);
      dzc[c] = on ? wk * gC[c] * cl[c] * (1.0f - cl[c]) : 0.0f;
    }
    const float dzs = on ? dsig * delta * tm_sigmoid(zs) : 0.0f;
    // head gradient: operand (natural k-rows 0..3 in half 0) and table rows
    pbf16x8 gb;
    {
      uint4 u;
      u.x = pack2_bf16(dzs, dzc[0]);
      u.y = pack2_bf16(dzc[1], dzc[2]);
      u.z = 0u;
      u.w = 0u;
      gb = __builtin_bit_cast(pbf16x8, u);
      if (PASS == 0 && on)
#pragma unroll
        for (int r = 0; r < 4; ++r) tab[(T::G + r) * kTabRow + n] = gb[r];
    }
    // backward through the layers: da3 = W_head^T g, then dz_l and dW_l
    pf32x16 dz[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
      dz[mt] = tmb_mask(tmb_mfma(s_w[(F_WHT + mt) * 64 + lane], gb, tmb_zero()), mk[3], mt);
#pragma unroll
    for (int l = 3; l >= 0; --l) {
      // pass 0 accumulates W3, W2 (and the heads), pass 1 W1, W0
      const bool mine = PASS == 0 ? l >= 2 : l <= 1;
      if (mine) {
      // dz_l into the table (after the last layer's reads of it)
      __builtin_amdgcn_wave_barrier();
      asm volatile("" ::: "memory");
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) tile_to_table(dz[mt], tab + T::DZ * kTabRow, 32 * mt, n, h);
      __builtin_amdgcn_wave_barrier();
      asm volatile("" ::: "memory");
      // dW_l += dz_l h_{l-1}^T over the 32 samples; db_l against ones
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        pbf16x8 ga[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) ga[kb] = table_operand(tab + T::DZ * kTabRow, 32 * mt + n, kb, h);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int kb = 0; kb < 2; ++kb) {
            if (l == 0) {
              const int row = 32 * nt + n < 48 ? 32 * nt + n : 48;
              dw0[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  ga[kb], table_operand(tab + T::X * kTabRow, row, kb, h), dw0[mt][nt], 0, 0, 0);
            } else {
              dw[l - 1][mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  ga[kb], table_operand(tab + tab_h<PASS>(l - 1) * kTabRow, 32 * nt + n, kb, h),
                  dw[l - 1][mt][nt], 0, 0, 0);
            }
          }
        if (l > 0) {
          pf32x16 db = tmb_zero();
#pragma unroll
          for (int kb = 0; kb < 2; ++kb) db = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga[kb], ones, db, 0, 0, 0);
          if (n == 0)
#pragma unroll
            for (int v = 0; v < 16; ++v) s_db[wv][(l - 1) * tm::H + 32 * mt + tile_row(v, h)] += db[v];
        }
      }
      }
      if (l == 0 || (PASS == 0 && l == 2)) break;
      // da_{l-1} = W_l^T dz_l, masked by h_{l-1} > 0
      pbf16x8 dzb[4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) tile_operands_bf16(dz[mt], dzb[2 * mt], dzb[2 * mt + 1]);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        pf32x16 da = tmb_zero();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) da = tmb_mfma(s_w[(f_wt(l) + mt * 4 + kb) * 64 + lane], dzb[kb], da);
        dz[mt] = tmb_mask(da, mk[l - 1], mt);
      }
    }
    // head weights: dW_head += g [h3, gamma(d)]^T (row m of g: min(m, 4), a zero row)
    if (PASS == 0) {
      pbf16x8 ga[2];
      const int grow = n < 4 ? n : 4;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) ga[kb] = table_operand(tab + T::G * kTabRow, grow, kb, h);
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
          dwh[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ga[kb], table_operand(tab + T::H3 * kTabRow, 32 * nt + n, kb, h), dwh[nt], 0, 0, 0);
        dwh[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            ga[kb], table_operand(tab + T::D * kTabRow, n < 16 ? n : 16, kb, h), dwh[2], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  }
  // per-wave partials in parameter order (each pass its own entries)
  float* out = a.partial + (long)wave * tm::N;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int j = 32 * mt + tile_row(v, h);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int k = 32 * nt + n;
        if (PASS == 1) {
          if (k < tm::IX) out[tm::W0 + j * tm::IX + k] = dw0[mt][nt][v];
          else if (k == tm::IX) out[tm::B0 + j] = dw0[mt][nt][v];
          out[tm::W1 + j * tm::H + k] = dw[0][mt][nt][v];
        } else {
#pragma unroll
          for (int l = 1; l < 3; ++l) out[tm::W1 + l * (tm::H * tm::H + tm::H) + j * tm::H + k] = dw[l][mt][nt][v];
        }
      }
    }
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  for (int e = lane; e < 3 * tm::H; e += 64) {
    const int l = e / tm::H, j = e - l * tm::H;
    if (PASS == 0 ? l >= 1 : l == 0) out[tm::B1 + l * (tm::H * tm::H + tm::H) + j] = s_db[wv][e];
  }
  if (PASS == 1) return;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = tile_row(v, h);
    if (r >= 4) continue;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int u = 32 * nt + n;
      if (r == 0) out[tm::WS + u] = dwh[nt][v];
      else out[tm::WC + (r - 1) * tm::IC + u] = dwh[nt][v];
    }
    if (n < tm::ID) {
      if (r > 0) out[tm::WC + (r - 1) * tm::IC + tm::H + n] = dwh[2][v];
    } else if (n == tm::ID) {
      if (r == 0) out[tm::BS] = dwh[2][v];
      else out[tm::BC + r - 1] = dwh[2][v];
    }
  }
  if (lane == 0) a.loss_partial[wave] = lsum;
}

// sum of the per-wave partials; then the gradient, or one Adam step (t =
// step, counted from 1).  A workgroup takes kRedP parameters; its kRedG
// thread groups sum waves g, g + kRedG, ... and the groups' sums are added
// in group order (a fixed order: the result does not depend on the launch).
// The last workgroup sums the loss the same way.
constexpr int kRedP = 32, kRedG = 8;

__global__ __launch_bounds__(kRedP * kRedG) void k_map_reduce(const MapTrainArgs a) {
  __shared__ float s_part[kRedG * kRedP];
  const int p = threadIdx.x & (kRedP - 1), g = threadIdx.x / kRedP;
  if ((int)blockIdx.x == (int)gridDim.x - 1) {
    if (!a.loss_out) return;   // whole workgroup, before any barrier
    float l = 0.0f;
    for (int v = threadIdx.x; v < a.n_waves; v += kRedP * kRedG) l += a.loss_partial[v];
    s_part[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.0f;
      for (int k = 0; k < kRedP * kRedG; ++k) t += s_part[k];
      a.loss_out[a.loss_index] = t / (float)a.batch;
    }
    return;
  }
  const int e = blockIdx.x * kRedP + p;
  float acc = 0.0f;
  if (e < tm::N) {
#pragma unroll 4
    for (int v = g; v < a.n_waves; v += kRedG) acc += a.partial[(long)v * tm::N + e];
  }
  s_part[g * kRedP + p] = acc;
  __syncthreads();
  if (g != 0 || e >= tm::N) return;
  float gsum = 0.0f;
#pragma unroll
  for (int k = 0; k < kRedG; ++k) gsum += s_part[k * kRedP + p];
  if (a.grad_out) a.grad_out[e] = gsum;
  if (a.adam) {
    const float m = a.beta1 * a.m[e] + (1.0f - a.beta1) * gsum;
    const float v = a.beta2 * a.v[e] + (1.0f - a.beta2) * gsum * gsum;
    a.m[e] = m;
    a.v[e] = v;
    const float mhat = m / (1.0f - powf(a.beta1, (float)a.step));
    const float vhat = v / (1.0f - powf(a.beta2, (float)a.step));
    a.params_rw[e] -= a.lr * mhat / (sqrtf(vhat) + a.eps);
  }
}

hipError_t launch_map_grad(const MapTrainArgs& a, hipStream_t st) {
  if (a.S < 1 || a.S > 64 || a.n_waves < 1) return hipErrorInvalidValue;
  hipError_t e;
  if (a.bf16) {
    if (a.S != 32) return hipErrorInvalidValue;
    const dim3 grid((a.n_waves + tmb::WAVES - 1) / tmb::WAVES);
    hipLaunchKernelGGL(k_map_grad_bf16<0>, grid, dim3(64 * tmb::WAVES), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_map_grad_bf16<1>, grid, dim3(64 * tmb::WAVES), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    const dim3 grid((a.n_waves + kTmWaves - 1) / kTmWaves);
    hipLaunchKernelGGL(k_map_grad<0>, grid, dim3(64 * kTmWaves), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_map_grad<1>, grid, dim3(64 * kTmWaves), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_map_reduce, dim3((tm::N + kRedP - 1) / kRedP + 1), dim3(kRedP * kRedG), 0, st, a);
  return hipGetLastError();
}

}  // namespace fl
