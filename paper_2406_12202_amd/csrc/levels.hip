// Coarse-to-fine update of the small map (4x64, bf16 MFMA, 32 stratified
// samples per ray): per level one persistent fused ray kernel and one
// single-workgroup level kernel.
//
// k_level_rays keeps the whole packed map (30 KB of bf16 chunks, biases,
// heads) resident in LDS and walks the level's rays with a grid-stride loop
// over waves: for each ray (one 32-sample column tile) it generates the pixel
// ray of the particle's predicted pose, the box-averaged observation, the
// stratified samples and their encodings, evaluates the map, composites along
// the ray with a wave scan of log transmittance, finds Eq. 5's depths, and
// writes the ray's (C, A) and (F, E).  Every ray is computed by one wave with
// the same instruction sequence as the unfused kernels (raygen, k_mlp_bf16,
// k_composite), so the results do not depend on the tile configuration.
//
// k_level_finish reduces each particle's rays in fixed order to S_i, l_i and
// the mean uncertainty, applies the 1-sigma rejection, normalises, reads out
// the pose, resamples to the next level's particle count, gathers the drawn
// poses and applies the next level's prediction.
#include "filter_dev.h"
#include "maplayout_bf16.h"
#include "mfma_util.h"

namespace fl {

using LS = SmallMapB;
constexpr int kLevelSpr = 32;   // samples per ray on this path

__global__ void k_set_key(LevelKey* key, const LevelKey v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *key = v;
}

hipError_t launch_set_key(LevelKey* key, const LevelKey& v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_key, dim3(1), dim3(64), 0, st, key, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_level_predict(const LevelKey* key, const double* pose_in, double* pose_out,
                                                       int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  predict_pose(pose_in + (long)i * 12, pose_out + (long)i * 12, key->motion, key->sigma_t, key->sigma_r, key->seed,
               key->iter, i);
}

hipError_t launch_level_predict(const LevelKey* key, const double* pose_in, double* pose_out, int N, hipStream_t st) {
  hipLaunchKernelGGL(k_level_predict, dim3((N + 255) / 256), dim3(256), 0, st, key, pose_in, pose_out, N);
  return hipGetLastError();
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

template <int NTL, int WAVES>
struct LevelCfg {
  static constexpr int THREADS = 64 * WAVES;
  static constexpr long LDS = LS::BLOCKS * 1024 + LS::BIASES * 4 + LS::HEADS * 4 +
                              (long)WAVES * NTL * (LS::KBX + LS::KBD) * 1024;
};

template <int NTL, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_level_rays(const LevelRayArgs a) {
  using C = LevelCfg<NTL, WAVES>;
  __shared__ uint4 s_w[LS::BLOCKS * 64];
  __shared__ float4 s_bias[LS::BIASES / 4];
  __shared__ float s_heads[LS::HEADS];
  __shared__ uint4 s_gx[WAVES][NTL * LS::KBX * 64];
  __shared__ uint4 s_gd[WAVES][NTL * LS::KBD * 64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 31, h = lane >> 5;
  {
    const uint4* wb = reinterpret_cast<const uint4*>(a.wblocks);
    for (int i = threadIdx.x; i < LS::BLOCKS * 64; i += C::THREADS) s_w[i] = wb[i];
    for (int i = threadIdx.x; i < LS::BIASES / 4; i += C::THREADS)
      s_bias[i] = reinterpret_cast<const float4*>(a.bias)[i];
    for (int i = threadIdx.x; i < LS::HEADS; i += C::THREADS) s_heads[i] = a.heads[i];
  }
  __syncthreads();
  const uint64_t seed = a.key->seed, iter = a.key->iter + (uint64_t)a.level;
  const float* bias = reinterpret_cast<const float*>(s_bias);
  const long n_rays = (long)a.N * a.B;
  const long n_tiles = (n_rays + NTL - 1) / NTL;
  const long n_waves = (long)gridDim.x * WAVES;
  for (long tile = (long)blockIdx.x * WAVES + wv; tile < n_tiles; tile += n_waves) {
    long ray[NTL];
    bool act[NTL];
    float t[NTL], obs[NTL][3];
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      const long r0 = tile * NTL + nt;
      act[nt] = r0 < n_rays;
      const long r = act[nt] ? r0 : n_rays - 1;
      ray[nt] = r;
      const int i = (int)(r / a.B), j = (int)(r - (r / a.B) * a.B);
      // ray of query pixel p_j (as k_raygen)
      const uint32_t w = draw(seed, iter, kStreamPix, (uint32_t)j, 0, 0).x;
      const uint64_t npix = (uint64_t)a.Wl * (uint64_t)a.Hl;
      const uint64_t p = ((uint64_t)w * npix) >> 32;
      const int u = (int)(p % (uint64_t)a.Wl), v = (int)(p / (uint64_t)a.Wl);
      const double* P = a.pose + (long)i * 12;
      const double dc0 = ((double)u + 0.5 - a.cx) / a.fx;
      const double dc1 = -((double)v + 0.5 - a.cy) / a.fy;
      const double dc2 = -1.0;
      double d0 = P[0] * dc0 + P[1] * dc1 + P[2] * dc2;
      double d1 = P[4] * dc0 + P[5] * dc1 + P[6] * dc2;
      double d2 = P[8] * dc0 + P[9] * dc1 + P[10] * dc2;
      const double inv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      d0 *= inv; d1 *= inv; d2 *= inv;
      const float4 o = make_float4((float)P[3], (float)P[7], (float)P[11], 0.0f);
      const float4 d = make_float4((float)d0, (float)d1, (float)d2, 0.0f);
      // downscale(I_t, R_t) at the query pixel
      double c0 = 0.0, c1 = 0.0, c2 = 0.0;
      for (int yy = 0; yy < a.s; ++yy) {
        const float* row = a.image + ((long)(v * a.s + yy) * a.W_full + (long)u * a.s) * 3;
        for (int xx = 0; xx < a.s; ++xx) {
          c0 += row[3 * xx + 0]; c1 += row[3 * xx + 1]; c2 += row[3 * xx + 2];
        }
      }
      const double sc = 1.0 / ((double)a.s * a.s);
      obs[nt][0] = (float)(c0 * sc); obs[nt][1] = (float)(c1 * sc); obs[nt][2] = (float)(c2 * sc);
      // stratified sample k = n of this ray (as the coarse pass of k_mlp_bf16)
      const int k = n;
      float xi = 0.0f;
      if (a.jitter) xi = unit24(pick(draw(seed, iter, kStreamJitCoarse, i, j, k >> 2), k & 3));
      t[nt] = a.near_ + ((float)k + xi) * a.dt;
      bf16x8 gx[LS::KBX], gd[LS::KBD];
      posenc_b<LS::LX>(fmaf(t[nt], d.x, o.x), fmaf(t[nt], d.y, o.y), fmaf(t[nt], d.z, o.z), h, gx);
      posenc_b<LS::LD>(d.x, d.y, d.z, h, gd);
#pragma unroll
      for (int kb = 0; kb < LS::KBX; ++kb) s_gx[wv][(nt * LS::KBX + kb) * 64 + lane] = __builtin_bit_cast(uint4, gx[kb]);
#pragma unroll
      for (int kb = 0; kb < LS::KBD; ++kb) s_gd[wv][(nt * LS::KBD + kb) * 64 + lane] = __builtin_bit_cast(uint4, gd[kb]);
    }
    // the map (layer order and arithmetic of k_mlp_bf16 for this shape)
    bf16x8 xa[NTL][LS::KBH], xb[NTL][LS::KBH];
    dense_res<NTL, LS::MT, LS::KBX, LS::KBH, true, LS::KBH>(s_w + LS::block_base(0) * 64, bias + LS::bias_base(0) + h * 16,
                                                           true, xb, s_gx[wv], xa, lane);
#pragma unroll
    for (int l = 1; l < LS::D; ++l) {
      dense_res<NTL, LS::MT, LS::KBH, LS::KBH, false, LS::KBH>(s_w + LS::block_base(l) * 64,
                                                              bias + LS::bias_base(l) + h * 16, true, xa, nullptr,
                                                              xb, lane);
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
        for (int q = 0; q < LS::KBH; ++q) xa[nt][q] = xb[nt][q];
    }
    const float* hs = s_heads + LS::SIG_OFF;
    const float* hr = s_heads + LS::RGB_OFF;
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      float z = dot_b<LS::KBH>(hs + h * LS::KBH * 8, xa[nt]);
      z += __shfl_xor(z, 32, 64);
      const float sg = softplus_b(z + hs[16 * LS::KBH]);
      float rgb[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float* w = hr + (c * 2 + h) * LS::KBG * 8;
        bf16x8 gd[LS::KBD];
#pragma unroll
        for (int kb = 0; kb < LS::KBD; ++kb)
          gd[kb] = __builtin_bit_cast(bf16x8, s_gd[wv][(nt * LS::KBD + kb) * 64 + lane]);
        float zc = dot_b<LS::KBH>(w, xa[nt]) + dot_b<LS::KBD>(w + LS::KBH * 8, gd);
        zc += __shfl_xor(zc, 32, 64);
        rgb[c] = sigmoid_b(zc + hr[48 * LS::KBG + c]);
      }
      // compositing along the ray (as k_composite with one sample per lane):
      // lanes 0..31 hold samples 0..31, lanes 32..63 contribute nothing
      const bool mine = h == 0;
      const float tk = t[nt];
      float tn = __shfl_down(tk, 1, 64);
      if (n + 1 >= kLevelSpr) tn = a.far_;
      float lsum = 0.0f;
      if (mine) lsum += sg * (tn - tk);
      const float incl = wave_incl_scan(lsum, lane);
      float run = -(incl - lsum);
      float cr = 0.0f, cg = 0.0f, cb = 0.0f, accw = 0.0f, lt = 0.0f;
      int ktr = 1 << 30, kop = 1 << 30;
      if (mine) {
        const float tau = sg * (tn - tk);
        const float w = expf(run) * -expm1f(-tau);
        lt = run;
        cr = fmaf(w, rgb[0], cr); cg = fmaf(w, rgb[1], cg); cb = fmaf(w, rgb[2], cb);
        accw += w;
        run -= tau;
        if (run <= a.log_trans) ktr = n;
        if (run < a.log_opq) kop = n;
      }
      cr = wave_sum(cr); cg = wave_sum(cg); cb = wave_sum(cb); accw = wave_sum(accw);
      ktr = wave_min_int(ktr);
      kop = wave_min_int(kop);
      float F = a.tau;
      if (ktr < kLevelSpr) {
        const float t_tr = __shfl(tk, ktr, 64), l_tr = __shfl(lt, ktr, 64), s_tr = __shfl(sg, ktr, 64);
        const int ko = kop < kLevelSpr ? kop : 0;
        const float t_op = __shfl(tk, ko, 64), l_op = __shfl(lt, ko, 64), s_op = __shfl(sg, ko, 64);
        const float zt = t_tr + (l_tr - a.log_trans) / s_tr;
        const float zo = (kop < kLevelSpr) ? t_op + (l_op - a.log_opq) / s_op : a.far_;
        F = fmaxf(zo - zt, a.tau);
      }
      const float er = obs[nt][0] - cr, eg = obs[nt][1] - cg, eb = obs[nt][2] - cb;
      const float E = er * er + eg * eg + eb * eb;
      if (act[nt] && lane == 0) {
        a.ray_rgba[ray[nt]] = make_float4(cr, cg, cb, accw);
        a.ray_fe[ray[nt]] = make_float2(F, E);
      }
    }
  }
}

template <int NTL, int WAVES>
hipError_t launch_level_rays_t(const LevelRayArgs& a, int blocks, hipStream_t st) {
  static_assert(LevelCfg<NTL, WAVES>::LDS <= 160 * 1024, "LDS budget");
  hipLaunchKernelGGL((k_level_rays<NTL, WAVES>), dim3(blocks), dim3(64 * WAVES), 0, st, a);
  return hipGetLastError();
}

bool level_rays_config_ok(int ntl, int waves) {
  return (ntl == 1 && (waves == 4 || waves == 8 || waves == 16)) || (ntl == 2 && (waves == 4 || waves == 8));
}

hipError_t launch_level_rays(const LevelRayArgs& a, int ntl, int waves, int blocks, hipStream_t st) {
  if ((long)a.N * a.B <= 0) return hipSuccess;
  if (blocks < 1) return hipErrorInvalidValue;
  if (ntl == 1 && waves == 4) return launch_level_rays_t<1, 4>(a, blocks, st);
  if (ntl == 1 && waves == 8) return launch_level_rays_t<1, 8>(a, blocks, st);
  if (ntl == 1 && waves == 16) return launch_level_rays_t<1, 16>(a, blocks, st);
  if (ntl == 2 && waves == 4) return launch_level_rays_t<2, 4>(a, blocks, st);
  if (ntl == 2 && waves == 8) return launch_level_rays_t<2, 8>(a, blocks, st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRedThreads) void k_level_finish(const LevelFinishArgs a) {
  __shared__ double s_d[kEstThreads * 13];   // >= kRedThreads doubles; reused by every phase
  __shared__ u64 s_u[kRedThreads];
  __shared__ double s_stat[2];
  const int tid = threadIdx.x;
  const uint64_t seed = a.key->seed, iter = a.key->iter + (uint64_t)a.level;
  // per-particle score (fixed order over the rays, as k_composite) and mean F;
  // the float64 mean F waits in weight[] for the rejection statistics
  for (int i = tid; i < a.N; i += kRedThreads) {
    double S_i = 0.0, Fs = 0.0;
    for (int j = 0; j < a.B; ++j) {
      const float2 fe = a.ray_fe[(long)i * a.B + j];
      S_i += (double)(fe.y * fe.x);
      Fs += (double)fe.x;
    }
    const double Sfl = (S_i > 1e-12 || isnan(S_i)) ? S_i : 1e-12;   // NaN stays NaN
    a.loglik[i] = 4.0 * (log((double)a.B) - log(Sfl));
    a.uncert[i] = (float)(Fs / a.B);
    a.weight[i] = Fs / a.B;
  }
  __threadfence_block();
  __syncthreads();
  if (a.reject) {
    // mean and population standard deviation of the mean F over particles
    // with finite mean F and finite l; particles above mean + std get -inf
    double cnt = 0.0, sum = 0.0;
    for (int i = tid; i < a.N; i += kRedThreads) {
      const double U = a.weight[i];
      if (isfinite(U) && isfinite(a.loglik[i])) { cnt += 1.0; sum += U; }
    }
    s_d[tid] = sum;
    s_u[tid] = (u64)cnt;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
      if (tid < o) { s_d[tid] += s_d[tid + o]; s_u[tid] += s_u[tid + o]; }
      __syncthreads();
    }
    if (tid == 0) s_stat[0] = s_u[0] > 0 ? s_d[0] / (double)s_u[0] : 0.0;
    __syncthreads();
    const double mu = s_stat[0];
    const double n_ok = (double)s_u[0];
    __syncthreads();
    double ss = 0.0;
    for (int i = tid; i < a.N; i += kRedThreads) {
      const double U = a.weight[i];
      if (isfinite(U) && isfinite(a.loglik[i])) ss += (U - mu) * (U - mu);
    }
    s_d[tid] = ss;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
      if (tid < o) s_d[tid] += s_d[tid + o];
      __syncthreads();
    }
    if (tid == 0) s_stat[1] = n_ok > 0.0 ? sqrt(s_d[0] / n_ok) : 0.0;
    __syncthreads();
    const double thr = mu + s_stat[1];
    for (int i = tid; i < a.N; i += kRedThreads) {
      const double U = a.weight[i];
      const bool ok = isfinite(U) && isfinite(a.loglik[i]);
      if (!ok || U > thr) a.loglik[i] = -INFINITY;
    }
    __threadfence_block();
    __syncthreads();
  }
  normalize_block(a.loglik, a.weight, a.N, a.flags, s_d);
  if (a.est) pose_estimate_block(a.pose, a.weight, a.N, a.est, a.flags, reinterpret_cast<double(*)[13]>(s_d));
  resample_block(a.weight, a.N, a.n_out, seed, iter, a.prefix, a.idx, a.flags, s_d, s_u);
  // gather the drawn poses; apply the next level's prediction to particle k
  for (int k = tid; k < a.n_out; k += kRedThreads) {
    const int i = a.idx[k];
    double* out = a.next_pose + (long)k * 12;
    if (i < 0 || i >= a.N) {
      for (int q = 0; q < 12; ++q) out[q] = NAN;
    } else if (a.predict_next) {
      predict_pose(a.pose + (long)i * 12, out, a.key->motion, a.key->sigma_t, a.key->sigma_r, seed, iter + 1, k);
    } else {
      for (int q = 0; q < 12; ++q) out[q] = a.pose[(long)i * 12 + q];
    }
  }
}

hipError_t launch_level_finish(const LevelFinishArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_level_finish, dim3(1), dim3(kRedThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace fl
