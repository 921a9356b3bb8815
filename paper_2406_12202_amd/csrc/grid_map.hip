// Multi-resolution grid map (the map type of Sec. IV-B, restated as a
// multiresolution hash encoding with a tiny MLP): per sample, L levels of
// trilinear blends of two-feature table entries at the 8 cell corners (dense
// index while the level's vertices fit the table, the spatial hash of three
// primes otherwise), then z = W2 relu(W1 f + b1) + b2, sigma = softplus(z_0),
// rgb = sigmoid(W4 relu(W3 [z, gamma(d)] + b3) + b4).  Points outside the
// box [-bound, bound]^3 are empty.
//
// Same sample sets and stratified placement as the MLP kernels (MlpArgs).
// The tables hold half-precision feature pairs (one 32-bit word per entry).
// Three passes over a chunk of at most feat_cap samples:
//   points   each sample's position in the unit cube and whether it lies in
//            the box (the coarse stratified depths are stored here when they
//            are not given);
//   encode   one thread per (sample, level), launched level-major (grid.y is
//            the level, so the blocks in flight read one level's table, 2 MB
//            at 2^19 entries, which stays in every XCD's L2), the 8 corner
//            reads (x-neighbours in one 8-byte read where they share one)
//            and the blend, float32 features to the workspace;
//   mlp      the tiny MLP on the matrix cores, 32 samples per wave.
// Positions and features are computed as by a single pass per sample, so
// results do not depend on the chunking.
#include "common.h"
#include "kernels.h"

namespace fl {

namespace gm {
constexpr int H = 64, GEO = 16;
}  // namespace gm

__device__ __forceinline__ float gm_softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float gm_sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// gamma_LD(d) in canonical order (d, sin 2^0 pi d, cos 2^0 pi d, ...): band 0
// from sincospif, band b + 1 from band b by the double-angle identities (each
// doubling at most doubles the absolute error: a few float32 roundings for
// LD <= 4)
template <int LD>
__device__ __forceinline__ void gm_dir_encoding(const float4 d, float (&gd)[3 + 6 * LD]) {
  const float v[3] = {d.x, d.y, d.z};
  gd[0] = d.x;
  gd[1] = d.y;
  gd[2] = d.z;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float sn, cs;
    sincospif(v[c], &sn, &cs);
#pragma unroll
    for (int l = 0; l < LD; ++l) {
      gd[3 + 6 * l + c] = sn;
      gd[3 + 6 * l + 3 + c] = cs;
      const float s2 = 2.0f * sn * cs, c2 = (cs - sn) * (cs + sn);
      sn = s2;
      cs = c2;
    }
  }
}

// depth of sample sl of the pass's sample set
__device__ __forceinline__ float grid_sample_t(const MlpArgs& a, const bool second, const long sl) {
  return second ? a.t_in2[sl] : (a.t_in ? a.t_in[sl] : a.t_out[sl]);
}

// position of sample s (of both sets) in the box's unit cube, and whether it
// lies inside the box
struct GridPoint {
  float u0, u1, u2;
  bool inside, second;
  long sl;
  int ray;
};

__device__ __forceinline__ GridPoint grid_point(const GridDev& g, const MlpArgs& a, const long s) {
  GridPoint p;
  p.second = s >= a.n_samples;
  p.sl = p.second ? s - a.n_samples : s;
  const int spr = p.second ? a.spr2 : a.spr;
  p.ray = (int)(p.sl / spr);
  const float4 o = a.ray_o[p.ray];
  const float4 d = a.ray_d[p.ray];
  const float t = grid_sample_t(a, p.second, p.sl);
  const float x0 = fmaf(t, d.x, o.x), x1 = fmaf(t, d.y, o.y), x2 = fmaf(t, d.z, o.z);
  const float inv = 1.0f / (2.0f * g.bound);
  float u0 = (x0 + g.bound) * inv, u1 = (x1 + g.bound) * inv, u2 = (x2 + g.bound) * inv;
  p.inside = u0 >= 0.0f && u0 <= 1.0f && u1 >= 0.0f && u1 <= 1.0f && u2 >= 0.0f && u2 <= 1.0f;
  p.u0 = fminf(fmaxf(u0, 0.0f), 1.0f);
  p.u1 = fminf(fmaxf(u1, 0.0f), 1.0f);
  p.u2 = fminf(fmaxf(u2, 0.0f), 1.0f);
  return p;
}

// positions of samples c0 .. c0 + n - 1 in the unit cube (u, inside) for
// the encoding and MLP passes; the coarse stratified depths are computed and
// stored here when they are not given
__global__ __launch_bounds__(256) void k_grid_points(const GridDev g, const MlpArgs a, const long c0, const long n) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const long s = c0 + q;
  if (s < a.n_samples && !a.t_in) {
    const int ray = (int)(s / a.spr);
    const int k = (int)(s - (long)ray * a.spr);
    float xi = 0.0f;
    if (a.jitter) {
      const int i = ray / a.B, j = ray - (ray / a.B) * a.B;
      xi = unit24(pick(draw(a.seed, a.iter, kStreamJitCoarse, i, j, k >> 2), k & 3));
    }
    a.t_out[s] = a.near_ + ((float)k + xi) * a.dt;
  }
  const GridPoint p = grid_point(g, a, s);
  g.pts[q] = make_float4(p.u0, p.u1, p.u2, p.inside ? 1.0f : 0.0f);
}

// corner indices and trilinear weights of one sample at level l
__device__ __forceinline__ void grid_corners(const GridDev& g, const float4 u, const int l, uint32_t (&idx)[8],
                                             float (&wt)[8]) {
  const int N = g.res[l];
  const float p0 = u.x * (float)N, p1 = u.y * (float)N, p2 = u.z * (float)N;
  const int c0i = min((int)floorf(p0), N - 1), c1i = min((int)floorf(p1), N - 1), c2i = min((int)floorf(p2), N - 1);
  const float w0 = p0 - (float)c0i, w1 = p1 - (float)c1i, w2 = p2 - (float)c2i;
  const bool dense = (g.dense_mask >> l) & 1u;
  const uint32_t n1 = (uint32_t)N + 1u;
  const uint32_t tmask = (1u << g.log2_table) - 1u;
  // per-axis terms of the two corner coordinates on each axis, combined per
  // corner by + (dense) or xor (hash); the same integers as forming each
  // corner's index from its own coordinates
  const uint32_t x0 = (uint32_t)c0i, y0 = (uint32_t)c1i, z0 = (uint32_t)c2i;
  uint32_t ty[2], tz[2];
  if (dense) {
    ty[0] = n1 * y0;
    tz[0] = n1 * n1 * z0;
    ty[1] = ty[0] + n1;
    tz[1] = tz[0] + n1 * n1;
  } else {
    ty[0] = y0 * 2654435761u;
    tz[0] = z0 * 805459861u;
    ty[1] = ty[0] + 2654435761u;
    tz[1] = tz[0] + 805459861u;
  }
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const uint32_t tx = x0 + (uint32_t)(corner & 1), yz = (corner >> 1) & 1, zz = (corner >> 2) & 1;
    idx[corner] = dense ? tx + ty[yz] + tz[zz] : (tx ^ ty[yz] ^ tz[zz]) & tmask;
    wt[corner] = ((corner & 1) ? w0 : 1.0f - w0) * (yz ? w1 : 1.0f - w1) * (zz ? w2 : 1.0f - w2);
  }
}

// Samples per thread of the encoding pass: the reads of all of a thread's
// samples are issued before any blend, so that more of them are in flight
// (measured on MI355X, 16 levels of 2^19 entries: two samples per thread
// 2.5% faster than one over the whole map launch, four no better than two).
// At the finer levels the pass is bound by the rate of L2 line requests
// (about six distinct lines per sample and level); the index arithmetic is
// not on the critical path.
#ifndef FL_GRID_SPT
#define FL_GRID_SPT 2
#endif
constexpr int kGridSpt = FL_GRID_SPT;
// raw buffer resource word 3 of the gfx9 family (no format, no swizzle), and
// an offset beyond every level's table (at most 2^24 entries of 4 B)
constexpr int kRawBufferFlags = 0x00020000;
constexpr uint32_t kGridNoRead = 0x80000000u;
typedef uint32_t gu32x2 __attribute__((ext_vector_type(2)));

// samples c0 .. c0 + n - 1, level blockIdx.y; thread samples q0 + 256 i
__global__ __launch_bounds__(256) void k_grid_encode(const GridDev g, const MlpArgs a, const long c0, const long n) {
  const long q0 = (long)blockIdx.x * blockDim.x * kGridSpt + threadIdx.x;
  const int l = blockIdx.y;
  const uint32_t* tab = g.tables + ((long)l << g.log2_table);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(tab), 0, (int)(4u << g.log2_table), kRawBufferFlags);
  // every position first, so that no wait for one of them also waits for
  // table reads issued before it
  float4 u[kGridSpt];
#pragma unroll
  for (int i = 0; i < kGridSpt; ++i) {
    const long q = q0 + (long)i * blockDim.x;
    u[i] = q < n ? g.pts[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  uint32_t e[kGridSpt][8];
  float wt[kGridSpt][8];
#pragma unroll
  for (int i = 0; i < kGridSpt; ++i) {
    const bool live = q0 + (long)i * blockDim.x < n;
    uint32_t idx[8];
    grid_corners(g, u[i], l, idx, wt[i]);
    // the x-neighbours c and c + e_0 share one aligned 8-byte word of the
    // table whenever their indices differ only in bit 0 (even c_0 under the
    // hash, whose x factor is 1; an even dense index): one 64-bit read then
    // serves both, and the odd neighbour's own read (like every read of a
    // thread past the last sample) is given an offset past the buffer's end,
    // which returns 0 without touching memory; no branches, so all reads of
    // the thread are in flight together
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i0 = idx[2 * k], i1 = idx[2 * k + 1];
      const bool paired = i1 == (i0 ^ 1u);
      const gu32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, live ? (i0 & ~1u) * 4u : kGridNoRead, 0, 0);
      const uint32_t lone = __builtin_amdgcn_raw_buffer_load_b32(rs, live && !paired ? i1 * 4u : kGridNoRead, 0, 0);
      e[i][2 * k] = (i0 & 1u) ? w.y : w.x;
      e[i][2 * k + 1] = paired ? ((i1 & 1u) ? w.y : w.x) : lone;
    }
  }
#pragma unroll
  for (int i = 0; i < kGridSpt; ++i) {
    const long q = q0 + (long)i * blockDim.x;
    if (q >= n) break;
    float fa = 0.0f, fb = 0.0f;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
      fa = fmaf(wt[i][corner], (float)__builtin_bit_cast(_Float16, (uint16_t)(e[i][corner] & 0xffffu)), fa);
      fb = fmaf(wt[i][corner], (float)__builtin_bit_cast(_Float16, (uint16_t)(e[i][corner] >> 16)), fb);
    }
    g.feat[(long)l * g.feat_cap + q] = make_float2(fa, fb);
  }
}

// The tiny MLP on the matrix cores (v_mfma_f32_32x32x2_f32): a wave takes a
// tile of 32 samples and computes the layers transposed, out^T = W in^T, with
// the samples as columns.  Lane l = 32 h + n supplies k-row h of column n; the
// accumulator holds, in lane (n, h) and register v, output row
// 8 (v / 4) + 4 h + v % 4 of column n, and register v of accumulator tile b
// is the input of the next layer's k-step 16 b + v (the contraction index is
// permuted, not the data).  Layer 1's k-step kb takes feature
// 2 ((kb >> 1) + h L / 2) + (kb & 1), so a lane reads whole feature pairs of
// half the levels; the 16 outputs of layer 2 fill half a tile (zero rows
// 16..31); layer 3's first 8 k-steps are z, then gamma(d) two entries per
// step; the 3 colour outputs are dot products on the vector ALU.  The weights,
// in operand order, are staged in LDS once per workgroup.
constexpr int kGmWaves = 4;
#ifndef FL_GM_BLOCKS
#define FL_GM_BLOCKS 2048
#endif
__device__ __forceinline__ int gm_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }
typedef float gf32x16 __attribute__((ext_vector_type(16)));

template <int L, int LD>
struct GmShape {
  static constexpr int NF = 2 * L, ID = 3 + 6 * LD, IN3 = gm::GEO + ID, KD = (ID + 1) / 2, K3 = 8 + KD;
  static constexpr int O_B1 = gm::H * NF, O_W2 = O_B1 + gm::H, O_B2 = O_W2 + gm::GEO * gm::H, O_W3 = O_B2 + gm::GEO;
  static constexpr int O_B3 = O_W3 + gm::H * IN3, O_W4 = O_B3 + gm::H, O_B4 = O_W4 + 3 * gm::H;
  // LDS: operand blocks of 64 floats
  static constexpr int A1 = 0, A2 = A1 + 2 * L * 64, A3 = A2 + 32 * 64, BIAS = A3 + 2 * K3 * 64;
  static constexpr int B1 = BIAS, B2 = B1 + 64, B3 = B2 + 32, W4 = B3 + 64, B4 = W4 + 3 * 64, TOTAL = B4 + 4;
};

template <int L, int LD>
__global__ __launch_bounds__(64 * kGmWaves) void k_grid_mlp(const GridDev g, const MlpArgs a, const long c0,
                                                           const long n) {
  using S = GmShape<L, LD>;
  __shared__ float s_w[S::TOTAL];
  const float* __restrict__ w = g.mlp;
  for (int e = threadIdx.x; e < S::A2; e += blockDim.x) {           // layer 1: block mt * L + kb
    const int ln = e & 63, nn = ln & 31, hh = ln >> 5, blk = e >> 6, mt = blk / L, kb = blk - mt * L;
    s_w[e] = w[(mt * 32 + nn) * S::NF + 2 * ((kb >> 1) + hh * (L / 2)) + (kb & 1)];
  }
  for (int e = threadIdx.x; e < 32 * 64; e += blockDim.x) {          // layer 2: block s, rows >= 16 zero
    const int ln = e & 63, nn = ln & 31, hh = ln >> 5, st = e >> 6;
    s_w[S::A2 + e] = nn < gm::GEO ? w[S::O_W2 + nn * gm::H + 32 * (st >> 4) + gm_row(st & 15, hh)] : 0.0f;
  }
  for (int e = threadIdx.x; e < 2 * S::K3 * 64; e += blockDim.x) {   // layer 3: block mt * K3 + s
    const int ln = e & 63, nn = ln & 31, hh = ln >> 5, blk = e >> 6, mt = blk / S::K3, st = blk - mt * S::K3;
    const int col = st < 8 ? gm_row(st, hh) : gm::GEO + 2 * (st - 8) + hh;
    s_w[S::A3 + e] = col < S::IN3 ? w[S::O_W3 + (mt * 32 + nn) * S::IN3 + col] : 0.0f;
  }
  for (int e = threadIdx.x; e < S::TOTAL - S::BIAS; e += blockDim.x) {
    float v = 0.0f;
    if (e < 64) v = w[S::O_B1 + e];
    else if (e < 96) v = e - 64 < gm::GEO ? w[S::O_B2 + e - 64] : 0.0f;
    else if (e < 160) v = w[S::O_B3 + e - 96];
    else if (e < 352) v = w[S::O_W4 + e - 160];
    else if (e < 355) v = w[S::O_B4 + e - 352];
    s_w[S::BIAS + e] = v;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nn = lane & 31, h = lane >> 5;
  const long tiles = (n + 31) / 32;
  for (long tile = (long)blockIdx.x * kGmWaves + wv; tile < tiles; tile += (long)gridDim.x * kGmWaves) {
    // an offset the compiler cannot see through, so that the weight reads
    // stay inside the loop instead of being hoisted into ~200 registers
    int o = 0;
    asm volatile("" : "+v"(o));
    const float* sw = s_w + o;
    const long q = tile * 32 + nn;
    const bool valid = q < n;
    const long qc = valid ? q : n - 1;
    const long smp = c0 + qc;
    const bool second = smp >= a.n_samples;
    const long sl = second ? smp - a.n_samples : smp;
    const int ray = (int)(sl / (second ? a.spr2 : a.spr));
    const bool inside = g.pts[qc].w != 0.0f;
    // features: the pairs of levels h L / 2 .. h L / 2 + L / 2 - 1
    float x[L];
#pragma unroll
    for (int i = 0; i < L / 2; ++i) {
      const float2 v = g.feat[(long)(i + h * (L / 2)) * g.feat_cap + qc];
      x[2 * i] = v.x;
      x[2 * i + 1] = v.y;
    }
    gf32x16 h1[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h1[mt][r] = sw[S::B1 + 32 * mt + gm_row(r, h)];
#pragma unroll
    for (int kb = 0; kb < L; ++kb)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        h1[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(sw[S::A1 + (mt * L + kb) * 64 + lane], x[kb], h1[mt], 0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h1[mt][r] = fmaxf(h1[mt][r], 0.0f);
    // layer 2: z (rows 0..15 in registers 0..7)
    gf32x16 z;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = sw[S::B2 + gm_row(r, h)];
#pragma unroll
    for (int st = 0; st < 32; ++st)
      z = __builtin_amdgcn_mfma_f32_32x32x2f32(sw[S::A2 + st * 64 + lane], h1[st >> 4][st & 15], z, 0, 0, 0);
    // layer 3 over [z, gamma(d)]
    float gd[S::ID];
    gm_dir_encoding<LD>(a.ray_d[ray], gd);
    gf32x16 h3[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) h3[mt][r] = sw[S::B3 + 32 * mt + gm_row(r, h)];
#pragma unroll
    for (int st = 0; st < S::K3; ++st) {
      float bx;
      if (st < 8) {
        bx = z[st];
      } else {
        const int i0 = 2 * (st - 8);
        const float v0 = gd[i0], v1 = i0 + 1 < S::ID ? gd[i0 + 1] : 0.0f;
        bx = h ? v1 : v0;
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        h3[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(sw[S::A3 + (mt * S::K3 + st) * 64 + lane], bx, h3[mt], 0, 0, 0);
    }
    // colour: dot products of the 64 hidden units (32 in each lane half)
    float rc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = 0.0f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc = fmaf(sw[S::W4 + c * 64 + 32 * mt + gm_row(r, h)], fmaxf(h3[mt][r], 0.0f), acc);
      rc[c] = acc + __shfl_xor(acc, 32, 64) + sw[S::B4 + c];
    }
    if (valid && h == 0) {
      float4 res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (inside) res = make_float4(gm_softplus(z[0]), gm_sigmoid(rc[0]), gm_sigmoid(rc[1]), gm_sigmoid(rc[2]));
      (second ? a.out2 : a.out)[sl] = res;
    }
  }
}

template <int L, int LD>
hipError_t launch_grid_t(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  const long n_tot = a.n_samples + a.n_samples2;
  for (long c0 = 0; c0 < n_tot; c0 += g.feat_cap) {
    const long n = n_tot - c0 < g.feat_cap ? n_tot - c0 : g.feat_cap;
    hipLaunchKernelGGL(k_grid_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, a, c0, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nbe = (unsigned)((n + 256 * kGridSpt - 1) / (256 * kGridSpt));
    hipLaunchKernelGGL(k_grid_encode, dim3(nbe, L), dim3(256), 0, st, g, a, c0, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long tiles = (n + 31) / 32, want = (tiles + kGmWaves - 1) / kGmWaves;
    const unsigned nbm = (unsigned)(want < FL_GM_BLOCKS ? want : FL_GM_BLOCKS);
    hipLaunchKernelGGL((k_grid_mlp<L, LD>), dim3(nbm), dim3(64 * kGmWaves), 0, st, g, a, c0, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int L>
hipError_t launch_grid_l(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  switch (g.in_d) {
    case 3 + 6 * 2: return launch_grid_t<L, 2>(g, a, st);
    case 3 + 6 * 4: return launch_grid_t<L, 4>(g, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid_map(const GridDev& g, const MlpArgs& a, hipStream_t st) {
  if (a.n_samples + a.n_samples2 <= 0) return hipSuccess;
  if (!g.feat || !g.pts || g.feat_cap <= 0) return hipErrorInvalidValue;
  switch (g.levels) {
    case 4: return launch_grid_l<4>(g, a, st);
    case 8: return launch_grid_l<8>(g, a, st);
    case 16: return launch_grid_l<16>(g, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fl
