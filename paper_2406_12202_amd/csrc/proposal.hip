// Learned proposal network: inference with proposal-guided fine placement,
// training (forward + analytic backward with per-wave gradient partials, then
// a fixed-order reduction and Adam), and ray format conversion.
//
// Network: x = [gamma_6(o), gamma_6(d)] (78), h1 = relu(W1 x + b1) (64),
// h2 = relu(W2 h1 + b2) (64), z = W3 h2 + b3 (32), p = softmax(z); parameters
// in the flat order W1, b1, W2, b2, W3, b3 (row-major).  One wave handles one
// ray at a time with hidden unit j on lane j; the vector a layer reads is
// broadcast lane by lane with v_readlane, so no LDS traffic is needed for
// activations.
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
// inference + placement: one wave per ray, weight rows in registers
__global__ __launch_bounds__(256) void k_proposal_fine(const ProposalArgs a) {
  const int lane = threadIdx.x & 63;
  const float* __restrict__ P = a.params;
  float w1[PIN], w2[PH], w3[PH];
#pragma unroll
  for (int k = 0; k < PIN; ++k) w1[k] = P[P_W1 + lane * PIN + k];
#pragma unroll
  for (int k = 0; k < PH; ++k) w2[k] = P[P_W2 + lane * PH + k];
  const int l3 = lane < PB ? lane : 0;
#pragma unroll
  for (int k = 0; k < PH; ++k) w3[k] = P[P_W3 + l3 * PH + k];
  const float b1 = P[P_B1 + lane], b2 = P[P_B2 + lane], b3 = P[P_B3 + l3];
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int ray = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); ray < a.n_rays; ray += waves) {
    const float4 o = a.ray_o[ray], d = a.ray_d[ray];
    const float x0 = prop_feature(o, d, lane);
    const float x1v = lane + 64 < PIN ? prop_feature(o, d, lane + 64) : 0.0f;
    float s1 = b1;
#pragma unroll
    for (int k = 0; k < PIN; ++k) s1 = fmaf(w1[k], k < 64 ? bcast(x0, k) : bcast(x1v, k - 64), s1);
    const float h1 = fmaxf(s1, 0.0f);
    float s2 = b2;
#pragma unroll
    for (int k = 0; k < PH; ++k) s2 = fmaf(w2[k], bcast(h1, k), s2);
    const float h2 = fmaxf(s2, 0.0f);
    float z = b3;
#pragma unroll
    for (int k = 0; k < PH; ++k) z = fmaf(w3[k], bcast(h2, k), z);
    const float p = softmax32(z, lane);
    if (a.hist && lane < PB) a.hist[(long)ray * PB + lane] = p;
    if (a.Sf <= 0) continue;
    // pdf 0.99 p + 0.01 / 32 on 32 equal bins; inclusive prefix over lanes 0..31
    const float mass = lane < PB ? 0.99f * p + 0.01f / PB : 0.0f;
    float c = mass;
#pragma unroll
    for (int off = 1; off < PB; off <<= 1) {
      const float u = __shfl_up(c, off, 64);
      if ((lane & 31) >= off) c += u;
    }
    const float total = __shfl(c, PB - 1, 64);
    const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
    const float width = (a.far_ - a.near_) / PB;
    // uniform control flow: every lane runs every round so that the
    // cross-lane reads below always address active lanes
    for (int m0 = 0; m0 < a.Sf; m0 += 64) {
      const int m = m0 + lane;
      const int mm = m < a.Sf ? m : a.Sf - 1;
      float xi = 0.5f;
      if (a.jitter) xi = unit24(pick(draw(a.seed, a.iter, kStreamJitFine, i, j, mm >> 2), mm & 3));
      const float target = ((float)mm + xi) / (float)a.Sf * total;
      // largest bin b with exclusive prefix c[b - 1] <= target (fixed 5 steps)
      int b = 0;
#pragma unroll
      for (int step = 16; step > 0; step >>= 1) {
        const float ce = __shfl(c, b + step - 1, 64);
        if (ce <= target) b += step;
      }
      const float cb = __shfl(c, b > 0 ? b - 1 : 0, 64);
      const float c0 = b > 0 ? cb : 0.0f;
      const float mb = __shfl(mass, b, 64);
      float frac = (target - c0) / mb;
      frac = fminf(fmaxf(frac, 0.0f), 1.0f);
      if (m < a.Sf)
        a.t_fine[(long)ray * a.Sf + m] = fminf(a.near_ + ((float)b + frac) * width, a.near_ + (b + 1) * width);
    }
  }
}

hipError_t launch_proposal_fine(const ProposalArgs& a, hipStream_t st) {
  if (a.n_rays <= 0) return hipSuccess;
  const int waves = (a.n_rays + 3) / 4 < 2048 ? (a.n_rays + 3) / 4 : 2048;
  hipLaunchKernelGGL(k_proposal_fine, dim3((waves + 3) / 4), dim3(256), 0, st, a);
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
  float g = 0.0f;
  for (int v = 0; v < a.n_waves; ++v) g += a.partial[(long)v * P_N + e];
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
