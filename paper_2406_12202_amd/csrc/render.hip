// Ray generation, hierarchical fine-sample placement and the per-ray
// compositing scan with the uncertainty F and the per-particle score.
#include "common.h"
#include "kernels.h"

namespace fl {

// ---------------------------------------------------------------------------
// ray generation: query pixel p_j at level R, its box-averaged observation and
// the camera ray of particle i through it (Eq. 4's r(p, x) with intrinsics R K;
// OpenGL camera, pixel centres at +1/2).  One thread per ray; the rotation is
// applied in float64 and the unit direction rounded once to float32.
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
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int yy = 0; yy < a.s; ++yy) {
    const float* row = a.image + ((long)(v * a.s + yy) * a.W_full + (long)u * a.s) * 3;
    for (int xx = 0; xx < a.s; ++xx) {
      c0 += row[3 * xx + 0]; c1 += row[3 * xx + 1]; c2 += row[3 * xx + 2];
    }
  }
  const double sc = 1.0 / ((double)a.s * a.s);
  a.obs[r] = make_float4((float)(c0 * sc), (float)(c1 * sc), (float)(c2 * sc), 0.0f);
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
// compositing (Eq. 1), Eq. 5 depths, F and the Eq. 6 score.  One workgroup per
// particle, one wave per ray at a time.  The coarse and fine sample lists
// (each sorted) are merged by rank in LDS (ties: coarse first); each lane then
// owns a contiguous run of merged samples; transmittance is a wave scan of
// tau in log space.
constexpr int kMaxS = 512;   // Sc + Sf
constexpr int kCompWaves = 4;

__global__ __launch_bounds__(256) void k_composite(const CompositeArgs a) {
  __shared__ float s_tm[kCompWaves][kMaxS];     // merged t
  __shared__ float s_sg[kCompWaves][kMaxS];     // merged sigma
  __shared__ float s_lt[kCompWaves][kMaxS];     // log T at each merged sample
  __shared__ float4 s_rgb[kCompWaves][kMaxS];   // merged colour (rgb, pad)
  __shared__ float s_tc[kCompWaves][256];       // coarse t (sorted) for ranking
  __shared__ float s_tf[kCompWaves][256];       // fine t (sorted)
  __shared__ float s_ef[1024];
  __shared__ float s_f[1024];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x;
  const int Sc = a.Sc, Sf = a.Sf, S = Sc + Sf;
  const int cpl = (S + 63) / 64;
  // every wave runs the same number of rounds so that block barriers match
  for (int jb = 0; jb < a.B; jb += kCompWaves) {
    const int j = jb + wv;
    const bool act = j < a.B && (long)i * a.B + j < a.n_rays;
    const long ray = (long)i * a.B + (act ? j : 0);
    // gather and merge
    if (act) {
      for (int k = lane; k < Sc; k += 64) s_tc[wv][k] = a.t_coarse[ray * Sc + k];
      for (int m = lane; m < Sf; m += 64) s_tf[wv][m] = a.t_fine[ray * Sf + m];
    }
    __syncthreads();
    for (int k = lane; act && k < Sc; k += 64) {
      const float tk = s_tc[wv][k];
      int lo = 0, hi = Sf;                 // count of fine < tk
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_tf[wv][mid] < tk) lo = mid + 1; else hi = mid; }
      const int pos = k + lo;
      const float4 q = a.out_coarse[ray * Sc + k];
      s_tm[wv][pos] = tk; s_sg[wv][pos] = q.x; s_rgb[wv][pos] = make_float4(q.y, q.z, q.w, 0.0f);
    }
    for (int m = lane; act && m < Sf; m += 64) {
      const float tm = s_tf[wv][m];
      int lo = 0, hi = Sc;                 // count of coarse <= tm
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_tc[wv][mid] <= tm) lo = mid + 1; else hi = mid; }
      const int pos = m + lo;
      const float4 q = a.out_fine[ray * Sf + m];
      s_tm[wv][pos] = tm; s_sg[wv][pos] = q.x; s_rgb[wv][pos] = make_float4(q.y, q.z, q.w, 0.0f);
    }
    __syncthreads();
    // per-lane run [lane * cpl, lane * cpl + cpl)
    const int k0 = lane * cpl;
    float lsum = 0.0f;
    for (int e = 0; e < cpl; ++e) {
      const int k = k0 + e;
      if (act && k < S) {
        const float tn = (k + 1 < S) ? s_tm[wv][k + 1] : a.far_;
        lsum += s_sg[wv][k] * (tn - s_tm[wv][k]);
      }
    }
    const float incl = wave_incl_scan(lsum, lane);
    const float log_t_end = -__shfl(incl, 63, 64);
    float run = -(incl - lsum);
    float cr = 0.0f, cg = 0.0f, cb = 0.0f, acc = 0.0f;
    int ktr = 1 << 30, kop = 1 << 30;
    for (int e = 0; e < cpl; ++e) {
      const int k = k0 + e;
      if (act && k < S) {
        const float tn = (k + 1 < S) ? s_tm[wv][k + 1] : a.far_;
        const float tau = s_sg[wv][k] * (tn - s_tm[wv][k]);
        const float w = expf(run) * -expm1f(-tau);
        s_lt[wv][k] = run;
        const float4 c = s_rgb[wv][k];
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
    __syncthreads();
    if (a.hist && act && lane < 32) {
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
        while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_tm[wv][mid] < edge) lo = mid + 1; else hi = mid; }
        kb[e] = lo;
      }
      const float t0 = kb[0] < S ? expf(s_lt[wv][kb[0]]) : expf(log_t_end);
      const float t1 = kb[1] < S ? expf(s_lt[wv][kb[1]]) : expf(log_t_end);
      const float den = -expm1f(log_t_end);
      a.hist[ray * 32 + lane] = acc < 1e-3f ? 1.0f / 32.0f : (t0 - t1) / den;
    }
    if (act && lane == 0) {
      float F = a.tau;
      if (ktr < S) {
        const float zt = s_tm[wv][ktr] + (s_lt[wv][ktr] - a.log_trans) / s_sg[wv][ktr];
        const float zo = (kop < S) ? s_tm[wv][kop] + (s_lt[wv][kop] - a.log_opq) / s_sg[wv][kop] : a.far_;
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
      s_ef[j] = E * F;
      s_f[j] = F;
    }
    __syncthreads();
  }
  __syncthreads();
  if (wv == 0 && a.loglik) {
    // lanes 0 .. G-1 form the particle's group; the rest add nothing
    const int G = particle_group(a.B);
    double S_i = 0.0, Fs = 0.0;
    particle_sums([&](int j, float& ef, float& f) { ef = s_ef[j]; f = s_f[j]; }, lane < G ? a.B : 0, G, lane,
                  S_i, Fs);
    if (lane == 0) {
      const double Sfl = (S_i > 1e-12 || isnan(S_i)) ? S_i : 1e-12;   // NaN stays NaN
      a.loglik[i] = 4.0 * (log((double)a.B) - log(Sfl));
      if (a.uncert) a.uncert[i] = (float)(Fs / a.B);
    }
  }
}

hipError_t launch_composite(const CompositeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_composite, dim3(a.N), dim3(64 * kCompWaves), 0, st, a);
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
