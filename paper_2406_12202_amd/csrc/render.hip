// Ray generation, hierarchical fine-sample placement and the per-ray
// compositing scan with the uncertainty F and the per-particle score.
#include "common.h"
#include "compositing.h"
#include "kernels.h"

namespace fl {

// ---------------------------------------------------------------------------
// ray generation: query pixel p_j at level R, its box-averaged observation and
// the camera ray of particle i through it (Eq. 4's r(p, x) with intrinsics R K;
// OpenGL camera, pixel centres at +1/2).  One thread per ray, float32 (the
// pose rounded once; camera_ray); the box average sums the s x s block row by
// row in float32.
__global__ __launch_bounds__(256) void k_raygen(const RaygenArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.N * a.B) return;
  const int i = r / a.B, j = r - (r / a.B) * a.B;
  const uint64_t npix = (uint64_t)a.Wl * (uint64_t)a.Hl;
  const uint64_t p = a.all_pixels ? (uint64_t)j
                                  : (((uint64_t)draw(a.seed, a.iter, kStreamPix, (uint32_t)j, 0, 0).x * npix) >> 32);
  const int u = (int)(p % (uint64_t)a.Wl), v = (int)(p / (uint64_t)a.Wl);
  float o[3], d[3];
  camera_ray(a.pose + (long)i * 12, u, v, a.fx, a.fy, a.cx, a.cy, o, d);
  a.ray_o[r] = make_float4(o[0], o[1], o[2], 0.0f);
  a.ray_d[r] = make_float4(d[0], d[1], d[2], 0.0f);
  if (!a.image) return;
  // downscale(I_t, R_t): mean of the s x s block behind level pixel (u, v)
  float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
  for (int yy = 0; yy < a.s; ++yy) {
    const float* row = a.image + ((long)(v * a.s + yy) * a.W_full + (long)u * a.s) * 3;
    for (int xx = 0; xx < a.s; ++xx) {
      c0 += row[3 * xx + 0]; c1 += row[3 * xx + 1]; c2 += row[3 * xx + 2];
    }
  }
  const float sc = 1.0f / (float)(a.s * a.s);   // a power of two: exact
  a.obs[r] = make_float4(c0 * sc, c1 * sc, c2 * sc, 0.0f);
}

hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st) {
  const int n = a.N * a.B;
  hipLaunchKernelGGL(k_raygen, dim3((n + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// hierarchical placement: one wave per ray.  Coarse transmittance by a wave
// scan of tau_k = sigma_k delta_k in log space, pdf mass w_k + 1e-5 delta_k,
// inverse CDF at u_m = (m + xi'_m) / Sf.  Up to 4 coarse samples per lane.
constexpr int kMaxCpl = 4;   // Sc <= 256

__global__ __launch_bounds__(256) void k_fine(const FineArgs a) {
  __shared__ float s_cdf[4][kMaxCpl * 64 + 1];
  __shared__ float s_t[4][kMaxCpl * 64];
  __shared__ float s_dl[4][kMaxCpl * 64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ray = blockIdx.x * 4 + wv;
  const bool active = ray < a.n_rays;
  const int Sc = a.Sc;
  const int cpl = (Sc + 63) / 64;
  float t[kMaxCpl], sg[kMaxCpl];
#pragma unroll
  for (int e = 0; e < kMaxCpl; ++e) {
    const int k = lane * cpl + e;
    const bool in = active && e < cpl && k < Sc;
    t[e] = in ? a.t_coarse[(long)ray * Sc + k] : a.far_;
    sg[e] = in ? a.out_coarse[(long)ray * Sc + k].x : 0.0f;
  }
  const float t_next_lane = __shfl_down(t[0], 1, 64);
  float dl[kMaxCpl], tau[kMaxCpl];
  float lsum = 0.0f;
#pragma unroll
  for (int e = 0; e < kMaxCpl; ++e) {
    const int k = lane * cpl + e;
    float tn;
    if (e + 1 < cpl) tn = t[e + 1 < kMaxCpl ? e + 1 : e];
    else tn = t_next_lane;
    if (k + 1 >= Sc) tn = a.far_;
    dl[e] = (e < cpl && k < Sc) ? tn - t[e] : 0.0f;
    tau[e] = sg[e] * dl[e];
    lsum += tau[e];
  }
  const float excl = wave_incl_scan(lsum, lane) - lsum;
  float mass[kMaxCpl];
  float run = -excl, msum = 0.0f;
#pragma unroll
  for (int e = 0; e < kMaxCpl; ++e) {
    const float w = expf(run) * -expm1f(-tau[e]);
    run -= tau[e];
    const int k = lane * cpl + e;
    mass[e] = (e < cpl && k < Sc) ? w + 1e-5f * dl[e] : 0.0f;
    msum += mass[e];
  }
  const float mincl = wave_incl_scan(msum, lane);
  const float total = __shfl(mincl, 63, 64);
  float c = mincl - msum;
#pragma unroll
  for (int e = 0; e < kMaxCpl; ++e) {
    const int k = lane * cpl + e;
    if (e < cpl && k < Sc) {
      if (k == 0) s_cdf[wv][0] = 0.0f;
      c += mass[e];
      s_cdf[wv][k + 1] = c;
      s_t[wv][k] = t[e];
      s_dl[wv][k] = dl[e];
    }
  }
  __syncthreads();
  if (!active) return;
  for (int m = lane; m < a.Sf; m += 64) {
    const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
    float xi = 0.5f;
    if (a.jitter) xi = unit24(pick(draw(a.seed, a.iter, kStreamJitFine, i, j, m >> 2), m & 3));
    const float target = ((float)m + xi) / (float)a.Sf * total;
    // largest k in [0, Sc-1] with cdf[k] <= target
    int lo = 0, hi = Sc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_cdf[wv][mid] <= target) lo = mid; else hi = mid - 1;
    }
    const float c0 = s_cdf[wv][lo], c1 = s_cdf[wv][lo + 1];
    const float t0 = s_t[wv][lo], d0 = s_dl[wv][lo];
    float frac = (c1 > c0) ? (target - c0) / (c1 - c0) : 0.0f;
    frac = fminf(fmaxf(frac, 0.0f), 1.0f);
    a.t_fine[(long)ray * a.Sf + m] = fminf(fmaf(frac, d0, t0), t0 + d0);
  }
}

hipError_t launch_fine(const FineArgs& a, hipStream_t st) {
  if (a.n_rays <= 0 || a.Sf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fine, dim3((a.n_rays + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compositing (Eq. 1), Eq. 5 depths and F per ray, then the Eq. 6 score per
// particle.  One wave per ray over the whole grid (kCompWaves rays per
// workgroup, independent of each other).  The coarse and fine sample lists
// (each sorted) are merged by rank in the wave's LDS (ties: coarse first);
// each lane then owns a contiguous run of merged samples; transmittance is a
// wave scan of tau in log space.  A wave's LDS is sized from S = Sc + Sf at
// launch (32 S bytes), so short lists leave room for many rays in flight.
constexpr int kCompWaves = 4;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kCompWaves) void k_composite(const CompositeArgs a) {
  extern __shared__ float4 s_dyn[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int Sc = a.Sc, Sf = a.Sf, S = Sc + Sf;
  float4* s_rgb = s_dyn + (long)wv * 2 * S;    // merged colour (rgb, pad)
  float* s_tm = (float*)(s_rgb + S);           // merged t
  float* s_sg = s_tm + S;                      // merged sigma
  float* s_lt = s_sg + S;                      // log T at each merged sample
  float* s_tc = s_lt + S;                      // coarse t (sorted) for ranking
  float* s_tf = s_tc + Sc;                     // fine t (sorted)
  const long ray = (long)blockIdx.x * kCompWaves + wv;
  if (ray >= a.n_rays) return;                 // whole waves leave; no block barriers follow
  const int cpl = (S + 63) / 64;
  // gather (depths and map outputs in flight together), then merge
  constexpr int kPer = 4;              // Sc, Sf <= 256 = 4 x 64
  float tc[kPer], tf[kPer];
  float4 qc[kPer], qf[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int k = lane + 64 * e;
    if (k < Sc) { tc[e] = a.t_coarse[ray * Sc + k]; qc[e] = a.out_coarse[ray * Sc + k]; }
    if (k < Sf) { tf[e] = a.t_fine[ray * Sf + k]; qf[e] = a.out_fine[ray * Sf + k]; }
  }
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int k = lane + 64 * e;
    if (k < Sc) s_tc[k] = tc[e];
    if (k < Sf) s_tf[k] = tf[e];
  }
  wave_lds_sync();
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int k = lane + 64 * e;
    if (k < Sc) {
      int lo = 0, hi = Sf;               // count of fine < t
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_tf[mid] < tc[e]) lo = mid + 1; else hi = mid; }
      const int pos = k + lo;
      s_tm[pos] = tc[e]; s_sg[pos] = qc[e].x; s_rgb[pos] = make_float4(qc[e].y, qc[e].z, qc[e].w, 0.0f);
    }
    if (k < Sf) {
      int lo = 0, hi = Sc;               // count of coarse <= t
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_tc[mid] <= tf[e]) lo = mid + 1; else hi = mid; }
      const int pos = k + lo;
      s_tm[pos] = tf[e]; s_sg[pos] = qf[e].x; s_rgb[pos] = make_float4(qf[e].y, qf[e].z, qf[e].w, 0.0f);
    }
  }
  wave_lds_sync();
  // per-lane run [lane * cpl, lane * cpl + cpl)
  const int k0 = lane * cpl;
  float lsum = 0.0f;
  for (int e = 0; e < cpl; ++e) {
    const int k = k0 + e;
    if (k < S) {
      const float tn = (k + 1 < S) ? s_tm[k + 1] : a.far_;
      lsum += s_sg[k] * (tn - s_tm[k]);
    }
  }
  const float incl = wave_incl_scan(lsum, lane);
  const float log_t_end = -__shfl(incl, 63, 64);
  float run = -(incl - lsum);
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, acc = 0.0f;
  int ktr = 1 << 30, kop = 1 << 30;
  for (int e = 0; e < cpl; ++e) {
    const int k = k0 + e;
    if (k < S) {
      const float tn = (k + 1 < S) ? s_tm[k + 1] : a.far_;
      const float tau = s_sg[k] * (tn - s_tm[k]);
      const float w = transmittance(run) * opacity(tau);
      s_lt[k] = run;
      const float4 c = s_rgb[k];
      cr = fmaf(w, c.x, cr); cg = fmaf(w, c.y, cg); cb = fmaf(w, c.z, cb);
      acc += w;
      run -= tau;
      if (run <= a.log_trans && k < ktr) ktr = k;
      if (run < a.log_opq && k < kop) kop = k;
    }
  }
  cr = wave_sum(cr); cg = wave_sum(cg); cb = wave_sum(cb); acc = wave_sum(acc);
  ktr = wave_min_int(ktr);
  kop = wave_min_int(kop);
  wave_lds_sync();
  if (a.hist && lane < 32) {
    // teacher histogram: bin b collects the weights of samples with depth in
    // [e_b, e_{b+1}); they are consecutive in the sorted list, and their sum
    // telescopes to T(first in bin) - T(first in next bin)
    const float width = (a.far_ - a.near_) / 32.0f;
    int kb[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float edge = a.near_ + (float)(lane + e) * width;
      int lo = 0, hi = S;                // first merged index with t >= edge
      if (lane + e == 32) lo = S;
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_tm[mid] < edge) lo = mid + 1; else hi = mid; }
      kb[e] = lo;
    }
    const float t0 = kb[0] < S ? expf(s_lt[kb[0]]) : expf(log_t_end);
    const float t1 = kb[1] < S ? expf(s_lt[kb[1]]) : expf(log_t_end);
    const float den = -expm1f(log_t_end);
    a.hist[ray * 32 + lane] = acc < 1e-3f ? 1.0f / 32.0f : (t0 - t1) / den;
  }
  if (lane == 0) {
    float F = a.empty_F;
    if (ktr < S) {
      const float zt = crossing_depth(s_tm[ktr], s_lt[ktr], a.log_trans, s_sg[ktr]);
      const float zo = (kop < S) ? crossing_depth(s_tm[kop], s_lt[kop], a.log_opq, s_sg[kop]) : a.far_;
      F = fmaxf(zo - zt, a.tau);
    }
    float E = 0.0f;
    if (a.obs) {
      const float4 ob = a.obs[ray];
      const float er = ob.x - cr, eg = ob.y - cg, eb = ob.z - cb;
      E = er * er + eg * eg + eb * eb;
    }
    a.ray_rgba[ray] = make_float4(cr, cg, cb, acc);
    a.ray_fe[ray] = make_float2(F, E);
  }
}

// Eq. 6 per particle from the per-ray (F, E): G = particle_group(B) lanes per
// particle, the fixed summation order of particle_sums.
__global__ __launch_bounds__(256) void k_particle_scores(const CompositeArgs a) {
  const int G = particle_group(a.B);
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = threadIdx.x & (G - 1);
  const long i = tid / G;
  if (i >= a.N) return;   // whole groups leave together
  double S_i, Fs;
  particle_sums([&](int j, float& ef, float& f) {
    const float2 fe = a.ray_fe[i * a.B + j];
    ef = fe.y * fe.x;
    f = fe.x;
  }, a.B, G, g, S_i, Fs);
  if (g == 0) {
    const double Sfl = (S_i > 1e-12 || isnan(S_i)) ? S_i : 1e-12;   // NaN stays NaN
    a.loglik[i] = 4.0 * (log((double)a.B) - log(Sfl));
    if (a.uncert) a.uncert[i] = (float)(Fs / a.B);
  }
}

hipError_t launch_composite(const CompositeArgs& a, hipStream_t st) {
  const int S = a.Sc + a.Sf;
  if (a.Sc < 1 || a.Sc > 256 || a.Sf < 0 || a.Sf > 256) return hipErrorInvalidValue;
  if (a.loglik && (long)a.N * a.B != a.n_rays) return hipErrorInvalidValue;
  if (a.n_rays > 0) {
    const size_t lds = (size_t)kCompWaves * 32 * S;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)((a.n_rays + kCompWaves - 1) / kCompWaves)),
                       dim3(64 * kCompWaves), lds, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!a.loglik || a.N <= 0) return hipSuccess;
  const long threads = (long)a.N * particle_group(a.B);
  hipLaunchKernelGGL(k_particle_scores, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ void k_split(const float4* rgba, const float2* fe, int n, float* rgb, float* op, float* F,
                        float* E) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float4 c = rgba[r];
  const float2 q = fe[r];
  if (rgb) { rgb[3 * r] = c.x; rgb[3 * r + 1] = c.y; rgb[3 * r + 2] = c.z; }
  if (op) op[r] = c.w;
  if (F) F[r] = q.x;
  if (E) E[r] = q.y;
}

hipError_t launch_split_ray_outputs(const float4* rgba, const float2* fe, int n, float* rgb,
                                    float* opacity, float* F, float* E, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split, dim3((n + 255) / 256), dim3(256), 0, st, rgba, fe, n, rgb, opacity, F, E);
  return hipGetLastError();
}

}  // namespace fl
