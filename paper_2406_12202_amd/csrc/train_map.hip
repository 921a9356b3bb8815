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

// sum of the per-wave partials in wave order; then the gradient, or one Adam
// step (t = step, counted from 1)
__global__ __launch_bounds__(256) void k_map_reduce(const MapTrainArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && a.loss_out) {
    float l = 0.0f;
    for (int v = 0; v < a.n_waves; ++v) l += a.loss_partial[v];
    a.loss_out[a.loss_index] = l / (float)a.batch;
  }
  if (e >= tm::N) return;
  float g = 0.0f;
  for (int v = 0; v < a.n_waves; ++v) g += a.partial[(long)v * tm::N + e];
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

hipError_t launch_map_grad(const MapTrainArgs& a, hipStream_t st) {
  if (a.S < 1 || a.S > 64 || a.n_waves < 1) return hipErrorInvalidValue;
  const dim3 grid((a.n_waves + kTmWaves - 1) / kTmWaves);
  hipLaunchKernelGGL(k_map_grad<0>, grid, dim3(64 * kTmWaves), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_map_grad<1>, grid, dim3(64 * kTmWaves), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_map_reduce, dim3((tm::N + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace fl
