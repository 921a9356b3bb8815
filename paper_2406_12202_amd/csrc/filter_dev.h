// Particle-filter device functions in float64, shared by the per-step kernels
// (filter.hip) and the fused level kernel of the coarse-to-fine path
// (levels.hip): prediction, weight normalisation, integer-exact systematic
// resampling and the pose read-out.  The block-level functions must be called
// by every thread of the workgroup; they synchronise internally and leave
// their global results visible to the whole workgroup on return.
#pragma once

#include "common.h"
#include "kernels.h"

namespace fl {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// x_t = x_{t-1} O_t Exp(delta), delta = (rho, phi) ~ N(0, diag(sigma_t^2 I,
// sigma_r^2 I)) (Sec. III-A, prediction step); Exp by Rodrigues' formula and
// the left Jacobian, Taylor coefficients for |phi| < 1e-4.  Particle i's
// noise comes from the motion stream keyed (i, 0, 0..1).
// The prediction in two parts: the increment Exp(delta) of particle i (its
// noise and the exponential map; independent of the pose), and its
// application x O Exp(delta).
__device__ __forceinline__ void motion_increment(double sigma_t, double sigma_r, uint64_t seed, uint64_t iter, int i,
                                                 double (&E)[12]) {
  const u32x4 w0 = draw(seed, iter, kStreamMotion, (uint32_t)i, 0, 0);
  const u32x4 w1 = draw(seed, iter, kStreamMotion, (uint32_t)i, 0, 1);
  const uint32_t ws[6] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y};
  double g[6];
  for (int p = 0; p < 3; ++p) {
    const double u1 = unit_open(ws[2 * p]), u2 = unit_open(ws[2 * p + 1]);
    const double r = sqrt(-2.0 * log(u1));
    g[2 * p] = r * cos(2.0 * M_PI * u2);
    g[2 * p + 1] = r * sin(2.0 * M_PI * u2);
  }
  const double rho[3] = {sigma_t * g[0], sigma_t * g[1], sigma_t * g[2]};
  const double ph[3] = {sigma_r * g[3], sigma_r * g[4], sigma_r * g[5]};
  const double th2 = ph[0] * ph[0] + ph[1] * ph[1] + ph[2] * ph[2];
  const double th = sqrt(th2);
  double A, Bc, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    Bc = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    A = sin(th) / th;
    Bc = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[3][3] = {{0.0, -ph[2], ph[1]}, {ph[2], 0.0, -ph[0]}, {-ph[1], ph[0], 0.0}};
  double K2[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) K2[r][c] = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
  for (int r = 0; r < 3; ++r) {
    double tv = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double id = (r == c) ? 1.0 : 0.0;
      E[4 * r + c] = id + A * K[r][c] + Bc * K2[r][c];
      tv += (id + Bc * K[r][c] + C * K2[r][c]) * rho[c];
    }
    E[4 * r + 3] = tv;
  }
}

__device__ __forceinline__ void apply_increment(const double* __restrict__ xin, const double* O, const double* E,
                                                double* __restrict__ xout) {
  double x[12];
  for (int q = 0; q < 12; ++q) x[q] = xin[q];
  // y = x * O, then y * E
  double y[12], z[12];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      y[4 * r + c] = x[4 * r + 0] * O[c] + x[4 * r + 1] * O[4 + c] + x[4 * r + 2] * O[8 + c];
    y[4 * r + 3] = x[4 * r + 0] * O[3] + x[4 * r + 1] * O[7] + x[4 * r + 2] * O[11] + x[4 * r + 3];
  }
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      z[4 * r + c] = y[4 * r + 0] * E[c] + y[4 * r + 1] * E[4 + c] + y[4 * r + 2] * E[8 + c];
    z[4 * r + 3] = y[4 * r + 0] * E[3] + y[4 * r + 1] * E[7] + y[4 * r + 2] * E[11] + y[4 * r + 3];
  }
  for (int q = 0; q < 12; ++q) xout[q] = z[q];
}

__device__ __forceinline__ void predict_pose(const double* __restrict__ xin, double* __restrict__ xout, const double* O,
                                             double sigma_t, double sigma_r, uint64_t seed, uint64_t iter, int i) {
  double E[12];
  motion_increment(sigma_t, sigma_r, seed, iter, i, E);
  apply_increment(xin, O, E, xout);
}

// ---------------------------------------------------------------------------
// Workgroup reductions and scans.  Within a 64-lane wave: the DPP scan of
// common.h (wave_scan), lane 63 ending with the wave total.  The wave totals
// meet in LDS and are combined the same way in every wave.  The order is
// fixed, so the results are deterministic; two barriers per workgroup
// reduction.  Eight waves: for sets of a few hundred to a few thousand
// particles they finish a chain of reductions sooner than sixteen (12.6
// against 13.7 us per coarse-to-fine level kernel on MI355X) or four.
constexpr int kRedThreads = 512;

struct OpAdd {
  __device__ double operator()(const double a, const double b) const { return a + b; }
};
struct OpMax {
  __device__ double operator()(const double a, const double b) const { return fmax(a, b); }
};
struct OpAddU64 {
  __device__ unsigned long long operator()(const unsigned long long a, const unsigned long long b) const {
    return a + b;
  }
};

// s: one value per wave of the workgroup (LDS); every thread gets the result
template <class Op>
__device__ __forceinline__ double block_reduce(double v, const double id, Op op, double* s) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = lane_value(wave_scan(v, id, op), 63);
  if (lane == 0) s[w] = v;
  __syncthreads();
  const double t = lane_value(wave_scan(lane < nw ? s[lane] : id, id, op), 63);
  __syncthreads();
  return t;
}
__device__ __forceinline__ double block_sum(const double v, double* s) { return block_reduce(v, 0.0, OpAdd{}, s); }
// two sums through the same barriers (each exactly as block_sum computes it);
// s: two values per wave
__device__ __forceinline__ double2 block_sum2(double a, double b, double* s) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = lane_value(wave_scan(a, 0.0, OpAdd{}), 63);
  b = lane_value(wave_scan(b, 0.0, OpAdd{}), 63);
  if (lane == 0) {
    s[2 * w] = a;
    s[2 * w + 1] = b;
  }
  __syncthreads();
  const double ta = lane_value(wave_scan(lane < nw ? s[2 * lane] : 0.0, 0.0, OpAdd{}), 63);
  const double tb = lane_value(wave_scan(lane < nw ? s[2 * lane + 1] : 0.0, 0.0, OpAdd{}), 63);
  __syncthreads();
  return make_double2(ta, tb);
}
__device__ __forceinline__ double block_max(const double v, double* s) {
  return block_reduce(v, -INFINITY, OpMax{}, s);
}
__device__ __forceinline__ double wave_sum(const double v) { return lane_value(wave_scan(v, 0.0, OpAdd{}), 63); }

// w_i = exp(l_i - m) / sum_k exp(l_k - m), m = max over finite l (Eq. 3).
// Fixed strided assignment and fixed reduction order: deterministic sums.
// Returns the largest weight: the particle at m has exp(0) = 1, and division
// by the common sum keeps the order, so it is 1 / sum (0 when no l is finite).
__device__ inline double normalize_block(const double* ll, double* w, int N, int* flags, double* s) {
  const int tid = threadIdx.x;
  double m = -INFINITY;
  for (int i = tid; i < N; i += kRedThreads) {
    const double v = ll[i];
    if (isfinite(v)) m = fmax(m, v);
  }
  m = block_max(m, s);
  const bool none = !(m > -INFINITY);
  // exp(l_i - m) kept in w (each thread rereads only its own entries)
  double acc = 0.0;
  for (int i = tid; i < N; i += kRedThreads) {
    const double v = ll[i];
    const double e = (!none && isfinite(v)) ? exp(v - m) : 0.0;
    w[i] = e;
    acc += e;
  }
  const double tot = block_sum(acc, s);
  for (int i = tid; i < N; i += kRedThreads) w[i] = none ? 0.0 : w[i] / tot;
  if (none && tid == 0) atomicOr(flags, 1);
  __threadfence_block();
  __syncthreads();
  return none ? 0.0 : 1.0 / tot;
}

// ---------------------------------------------------------------------------
// systematic resampling with integer thresholds (Alg. 1, draw loop):
// q_i = floor(w_i / w_max 2^40), inclusive prefix P (exact uint64),
// theta_k = floor((k 2^32 + r0) Q / (n_out 2^32)), idx_k = min{i : P_i > theta_k}.
__device__ inline double clean_weight(double w) { return (isfinite(w) && w > 0.0) ? w : 0.0; }

// floor(cur / n) for cur < n 2^32, n < 2^31, and the remainder: a float64
// estimate of the quotient (off by at most one) corrected exactly
__device__ inline u64 divmod_small(const u64 cur, const u64 n, const double inv_n, u64& r) {
  u64 q = (u64)((double)cur * inv_n);
  long long rr = (long long)(cur - q * n);
  while (rr < 0) { --q; rr += (long long)n; }
  while (rr >= (long long)n) { ++q; rr -= (long long)n; }
  r = (u64)rr;
  return q;
}

// floor(a * Q / (n 2^32)) for a < 2^63, Q < 2^64, n < 2^31, as 32-bit limbs;
// inv_n = 1 / n in float64
__device__ inline u64 resample_threshold(u64 a, u64 Q, u64 n, double inv_n) {
  const u64 lo = a * Q;
  const u64 hi = __umul64hi(a, Q);
  const u64 x2 = hi >> 32, x1 = hi & 0xffffffffull, x0 = lo >> 32;   // (hi:lo) >> 32
  u64 r = 0, q = 0;
  const u64 limbs[3] = {x2, x1, x0};
  for (int i = 0; i < 3; ++i) {
    const u64 cur = (r << 32) | limbs[i];
    q = (q << 32) | divmod_small(cur, n, inv_n, r);
  }
  return q;
}

// lower bound min{i : P_i > th} over the inclusive prefix P[0 .. n)
template <class P>
__device__ inline int prefix_search(const P* prefix, const int n, const u64 th) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] > th) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// inclusive prefix of the integer weights kept in LDS up to this many
// entries (the searches then read LDS), in the global array beyond
constexpr int kPrefixLds = 4096;

// idx[k] = -1 for every k and flag 2 when all weights are zero.  s_max: one
// double per wave; s_sum: one u64 per wave; s_prefix: kPrefixLds u64 (LDS).
// wmax_in: the largest cleaned weight when the caller knows it, else < 0;
// idx_lds: an LDS copy of idx (n_out entries) when not null.
__device__ inline void resample_block(const double* weight, int n_in, int n_out, uint64_t seed, uint64_t iter,
                                      u64* prefix, int32_t* idx, int* flags, double* s_max, u64* s_sum,
                                      u64* s_prefix, const double wmax_in = -1.0, int32_t* idx_lds = nullptr) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double wmax = wmax_in;
  if (wmax < 0.0) {
    double m = 0.0;
    for (int i = tid; i < n_in; i += kRedThreads) m = fmax(m, clean_weight(weight[i]));
    wmax = block_max(m, s_max);
  }
  // contiguous chunk per thread: local sums, workgroup inclusive scan (waves
  // by shuffles, then the wave totals), local prefixes
  const int chunk = (n_in + kRedThreads - 1) / kRedThreads;
  const int b0 = min(tid * chunk, n_in), b1 = min(b0 + chunk, n_in);
  // the integer weights q_i wait in the prefix array until the scan is known
  const bool in_lds = n_in <= kPrefixLds;
  u64* P = in_lds ? s_prefix : prefix;
  u64 local = 0;
  if (wmax > 0.0)
    for (int i = b0; i < b1; ++i) {
      const u64 q = (u64)floor(clean_weight(weight[i]) / wmax * 1099511627776.0);
      P[i] = q;
      local += q;
    }
  const u64 incl = wave_scan(local, (u64)0, OpAddU64{});
  if (lane == 63) s_sum[w] = incl;
  __syncthreads();
  u64 before = 0, Q = 0;
  for (int v = 0; v < kRedThreads / 64; ++v) {
    const u64 t = s_sum[v];
    if (v < w) before += t;
    Q += t;
  }
  u64 run = before + incl - local;
  if (wmax > 0.0)
    for (int i = b0; i < b1; ++i) {
      run += P[i];
      P[i] = run;
    }
  __threadfence_block();
  __syncthreads();
  if (Q == 0) {
    for (int k = tid; k < n_out; k += kRedThreads) {
      idx[k] = -1;
      if (idx_lds) idx_lds[k] = -1;
    }
    if (tid == 0) atomicOr(flags, 2);
  } else {
    const u64 r0 = draw(seed, iter, kStreamResample, 0, 0, 0).x;
    const double inv_n = 1.0 / (double)n_out;
    for (int k = tid; k < n_out; k += kRedThreads) {
      const u64 th = resample_threshold(((u64)k << 32) + r0, Q, (u64)n_out, inv_n);
      const int32_t v = in_lds ? prefix_search(s_prefix, n_in, th) : prefix_search(prefix, n_in, th);
      idx[k] = v;
      if (idx_lds) idx_lds[k] = v;
    }
  }
  __threadfence_block();
  __syncthreads();
}

// ---------------------------------------------------------------------------
// pose read-out: weighted mean position and chordal L2 mean rotation
// R = U diag(1, 1, det(U V^T)) V^T for sum_i w_i R_i = U S V^T.
__device__ inline void mat3_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}
__device__ inline double mat3_det(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// smallest-eigenvalue eigenvector of a symmetric 3x3 matrix by cyclic Jacobi rotations
__device__ inline void sym3_min_eigvec(const double* Ain, double* v) {
  double A[9], V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int i = 0; i < 9; ++i) A[i] = Ain[i];
  for (int sweep = 0; sweep < 16; ++sweep) {
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        const double apq = A[3 * p + q];
        if (fabs(apq) < 1e-300) continue;
        const double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {     // A <- J^T A J
          const double akp = A[3 * k + p], akq = A[3 * k + q];
          A[3 * k + p] = c * akp - s * akq;
          A[3 * k + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[3 * p + k], aqk = A[3 * q + k];
          A[3 * p + k] = c * apk - s * aqk;
          A[3 * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {     // V <- V J
          const double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - s * vkq;
          V[3 * k + q] = s * vkp + c * vkq;
        }
      }
  }
  int m = 0;
  if (A[4] < A[3 * m + m]) m = 1;
  if (A[8] < A[3 * m + m]) m = 2;
  for (int k = 0; k < 3; ++k) v[k] = V[3 * k + m];
}

constexpr int kEstThreads = 256;

// threads 0 .. kEstThreads-1 of the workgroup accumulate; s: at least 4 x 13 doubles
__device__ inline void pose_estimate_block(const double* pose, const double* w, int N, double* est, int* flags,
                                           double (*s)[13]) {
  const int tid = threadIdx.x;
  if (tid < kEstThreads) {
    double acc[13];
    for (int q = 0; q < 13; ++q) acc[q] = 0.0;
    for (int i = tid; i < N; i += kEstThreads) {
      const double wi = (isfinite(w[i]) && w[i] > 0.0) ? w[i] : 0.0;
      const double* P = pose + (long)i * 12;
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) acc[3 * r + c] += wi * P[4 * r + c];
        acc[9 + r] += wi * P[4 * r + 3];
      }
      acc[12] += wi;
    }
    for (int q = 0; q < 13; ++q) acc[q] = wave_sum(acc[q]);
    if ((tid & 63) == 0)
      for (int q = 0; q < 13; ++q) s[tid >> 6][q] = acc[q];
  }
  __syncthreads();
  if (tid == 0) {
    static_assert(kEstThreads == 256, "four wave totals");
    for (int q = 0; q < 13; ++q) s[0][q] = (s[0][q] + s[1][q]) + (s[2][q] + s[3][q]);
    const double W = s[0][12];
    bool done = false;
    if (!(W > 0.0)) {
      atomicOr(flags, 1);
      for (int q = 0; q < 12; ++q) est[q] = NAN;
      done = true;
    }
    double M[9], Q[9];
    if (!done) {
      for (int q = 0; q < 9; ++q) Q[q] = M[q] = s[0][q] / W;
      if (!(fabs(mat3_det(Q)) > 1e-300)) {
        atomicOr(flags, 4);
        for (int q = 0; q < 12; ++q) est[q] = NAN;
        done = true;
      }
    }
    if (!done) {
      // orthogonal polar factor of M by Newton's iteration with determinant
      // scaling: Q <- (g Q + Q^{-T} / g) / 2, g = |det Q|^(-1/3)
      for (int it = 0; it < 60; ++it) {
        const double d = mat3_det(Q);
        const double g = rcbrt(fabs(d));
        double C[9];   // cofactor matrix: Q^{-T} = C / det Q
        C[0] = Q[4] * Q[8] - Q[5] * Q[7]; C[1] = Q[5] * Q[6] - Q[3] * Q[8]; C[2] = Q[3] * Q[7] - Q[4] * Q[6];
        C[3] = Q[2] * Q[7] - Q[1] * Q[8]; C[4] = Q[0] * Q[8] - Q[2] * Q[6]; C[5] = Q[1] * Q[6] - Q[0] * Q[7];
        C[6] = Q[1] * Q[5] - Q[2] * Q[4]; C[7] = Q[2] * Q[3] - Q[0] * Q[5]; C[8] = Q[0] * Q[4] - Q[1] * Q[3];
        const double inv = 1.0 / (d * g);
        double diff = 0.0;
        for (int q = 0; q < 9; ++q) {
          const double nq = 0.5 * (g * Q[q] + C[q] * inv);
          diff = fmax(diff, fabs(nq - Q[q]));
          Q[q] = nq;
        }
        if (diff < 1e-15) break;
      }
      double R[9];
      for (int q = 0; q < 9; ++q) R[q] = Q[q];
      if (mat3_det(Q) < 0.0) {
        // reflection: flip the direction of the smallest singular value,
        // R = Q - 2 (Q v) v^T with v the smallest eigenvector of H = Q^T M
        double QT[9], H[9], v[3];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) QT[3 * r + c] = Q[3 * c + r];
        mat3_mul(QT, M, H);
        for (int r = 0; r < 3; ++r)
          for (int c = r + 1; c < 3; ++c) H[3 * r + c] = H[3 * c + r] = 0.5 * (H[3 * r + c] + H[3 * c + r]);
        sym3_min_eigvec(H, v);
        double u[3];
        for (int r = 0; r < 3; ++r) u[r] = Q[3 * r] * v[0] + Q[3 * r + 1] * v[1] + Q[3 * r + 2] * v[2];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) R[3 * r + c] = Q[3 * r + c] - 2.0 * u[r] * v[c];
      }
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) est[4 * r + c] = R[3 * r + c];
        est[4 * r + 3] = s[0][9 + r] / W;
      }
    }
  }
  __threadfence_block();
  __syncthreads();
}

// spread of a weighted particle set: sum_i w_i |t_i - t_bar|^2 / sum_i w_i
// (trace of the weighted covariance of the positions; w <= 0 or non-finite
// counts as 0; NaN without weight); two fixed-order passes over kEstThreads
// threads; s: at least 4 x 4 doubles
__device__ inline void position_variance_block(const double* pose, const double* w, int N, double* var,
                                               double (*s)[4]) {
  const int tid = threadIdx.x;
  if (tid < kEstThreads) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = tid; i < N; i += kEstThreads) {
      const double wi = (isfinite(w[i]) && w[i] > 0.0) ? w[i] : 0.0;
      for (int r = 0; r < 3; ++r) acc[r] += wi * pose[(long)i * 12 + 4 * r + 3];
      acc[3] += wi;
    }
    for (int q = 0; q < 4; ++q) acc[q] = wave_sum(acc[q]);
    if ((tid & 63) == 0)
      for (int q = 0; q < 4; ++q) s[tid >> 6][q] = acc[q];
  }
  __syncthreads();
  double tot[4];
  for (int q = 0; q < 4; ++q) tot[q] = (s[0][q] + s[1][q]) + (s[2][q] + s[3][q]);
  const double W = tot[3];
  const double tb[3] = {tot[0] / W, tot[1] / W, tot[2] / W};
  __syncthreads();
  if (tid < kEstThreads) {
    double v = 0.0;
    for (int i = tid; i < N; i += kEstThreads) {
      const double wi = (isfinite(w[i]) && w[i] > 0.0) ? w[i] : 0.0;
      double d2 = 0.0;
      for (int r = 0; r < 3; ++r) {
        const double d = pose[(long)i * 12 + 4 * r + 3] - tb[r];
        d2 += d * d;
      }
      v += wi * d2;
    }
    v = wave_sum(v);
    if ((tid & 63) == 0) s[tid >> 6][0] = v;
  }
  __syncthreads();
  if (tid == 0) *var = W > 0.0 ? ((s[0][0] + s[1][0]) + (s[2][0] + s[3][0])) / W : NAN;
  __threadfence_block();
  __syncthreads();
}

}  // namespace fl
