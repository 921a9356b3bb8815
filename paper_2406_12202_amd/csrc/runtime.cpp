// Host runtime of the particle-update library: the C ABI of fastloc.h,
// argument validation, weight packing for the MFMA kernels, workspace
// management, launch sequencing and per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fastloc.h"
#include "kernels.h"
#include "maplayout.h"
#include "maplayout_bf16.h"
#include "maplayout_fp8.h"

using namespace fl;

namespace {

enum KernelId { K_PREDICT, K_RAYGEN, K_MLP_COARSE, K_FINE, K_PROPOSAL, K_MLP_FINE, K_COMPOSITE, K_NORMALIZE,
                K_RESAMPLE, K_SPLIT, K_RAYS, K_TEACHER, K_TRAIN, K_GATHER, K_ESTIMATE, K_CALIB,
                K_LV_PREDICT, K_LV_RAYS, K_LV_SCORES, K_LV_FINISH, K_MLP_BOTH, K_VARIANCE, K_MAP_TRAIN, K_COUNT };
const char* kKernelNames[K_COUNT] = {"predict", "raygen", "mlp_coarse", "fine_placement", "proposal_placement",
                                     "mlp_fine", "composite_score", "normalize", "resample", "ray_outputs",
                                     "ray_format", "teacher_histogram", "proposal_train", "gather_poses",
                                     "pose_estimate", "fp8_calibration", "level_predict",
                                     "level_rays", "level_scores", "level_finish", "mlp_coarse_fine",
                                     "position_variance", "map_train"};

struct Pending { int kid; hipEvent_t a, b; double flop, bytes; };

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

struct loc_ctx {
  int device = 0;
  unsigned long long* noalloc_prefix = nullptr;   // this device's scratch of loc_resample_noalloc
  int empty_span = 0;   // 1: F = far - near for rays that never reach opacity alpha (else tau)
  hipStream_t stream = nullptr;
  loc_map_desc desc{};
  int kind = kMapSmall;
  long macs = 0;
  float* weights = nullptr;       // FP32 packed map
  void* wblocks = nullptr;        // BF16 weight chunks
  float* bias_b = nullptr;        // BF16 path biases
  float* heads_b = nullptr;       // BF16 path heads
  // FP8 path: canonical parameters (kept for packing after calibration),
  // E4M3/BF16 weight units, natural-order heads, per-layer exponents
  std::vector<float> params_host;
  void* wunits = nullptr;
  float* heads_f8 = nullptr;
  // multi-resolution grid map: tables and tiny MLP on the device
  GridDev grid{};
  double bytes_per_sample = 20.0;   // algorithmic bytes of one map evaluation (grid: its table reads)
  uint32_t* grid_tab = nullptr;
  float* grid_mlp = nullptr;
  float2* grid_feat = nullptr;   // encoding workspace of the grid map
  float4* grid_pts = nullptr;    // sample positions of the grid map's chunk
  bool f8_ready = false;
  int f8_ew[12] = {}, f8_ea[12] = {};
  float f8_amax[12] = {};
  // workspace
  DevBuf<float4> ray_o, ray_d, obs, out_c, out_f, rgba;
  DevBuf<float2> fe;
  DevBuf<float> t_c, t_f;
  DevBuf<unsigned long long> prefix;
  // learned proposal
  float* prop = nullptr;          // parameters
  float* prop_m = nullptr;        // Adam moments
  float* prop_v = nullptr;
  int prop_step = 0;
  int fine_mode = 0;              // 0 hierarchical, 1 proposal
  DevBuf<float> prop_partial, prop_loss;
  DevBuf<float4> tr_o, tr_d;      // rays of teacher / training calls
  // coarse-to-fine path: per-level buffers, device-side key, tile choices,
  // captured graph of the level sequence
  struct Level {
    DevBuf<double> pose, loglik, weight, inc;   // inc: the next level's motion increments (n_out x 12)
    DevBuf<float> uncert;
    DevBuf<int32_t> idx;
    DevBuf<float4> rgba;
    DevBuf<float2> fe;
    int N = 0, B = 0, n_out = 0;
    int ntl = 0, waves = 0, blocks = 0;   // 0: default choice
  };
  Level lv[8];
  int n_lv = 0;
  LevelKey* key = nullptr;
  int n_cu = 0;
  bool graph_mode = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphNode_t begin_node = nullptr;   // the graph's k_level_begin (takes each call's key)
  hipGraphExec_t gexec = nullptr;
  std::vector<double> graph_sig;
  // map training (4x64 map): float32 master weights in canonical order,
  // Adam moments, per-wave partial gradients and losses
  DevBuf<float> tm_params, tm_m, tm_v, tm_partial, tm_lpart;
  int tm_step = 0;
  bool tm_ready = false;
  // localisation loop: particle sets (ping-pong), predicted set, scores,
  // drawn indices, device and pinned host copies of (var, est)
  DevBuf<double> lz_x[2], lz_pred, lz_ll, lz_w, lz_ve;
  DevBuf<int32_t> lz_idx;
  double* lz_host = nullptr;
  int* flags = nullptr;
  int last_N = 0, last_B = 0;
  // profiling
  int prof = 0;               // 0 off, 1 every launch, 2 map-evaluation launches only
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  long long launches[K_COUNT] = {};
  double ms[K_COUNT] = {}, flop[K_COUNT] = {}, bytes[K_COUNT] = {};
  std::string err;
};

namespace {

loc_status fail(loc_ctx* c, loc_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIP_TRY(c, expr)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail((c), LOC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <class T>
loc_status ensure(loc_ctx* c, DevBuf<T>& b, size_t n) {
  if (b.n >= n) return LOC_OK;
  if (b.p) {
    hipStreamSynchronize(c->stream);
    hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
  }
  if (hipMalloc(&b.p, sizeof(T) * (n ? n : 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, LOC_E_OOM, "workspace allocation of %zu bytes failed", sizeof(T) * n);
  }
  b.n = n;
  return LOC_OK;
}

hipEvent_t get_event(loc_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// launch `fn` with optional event timing
template <class F>
loc_status timed(loc_ctx* c, int kid, double flop, double bytes, F fn) {
  hipEvent_t a = nullptr, b = nullptr;
  const bool map_kernel = kid == K_MLP_COARSE || kid == K_MLP_FINE || kid == K_MLP_BOTH || kid == K_LV_RAYS;
  const bool rec = c->prof == 1 || (c->prof == 2 && map_kernel);
  if (rec) {
    a = get_event(c);
    b = get_event(c);
    if (a) hipEventRecord(a, c->stream);
  }
  hipError_t e = fn();
  if (e != hipSuccess) return fail(c, LOC_E_HIP, "launch of %s failed: %s", kKernelNames[kid], hipGetErrorString(e));
  if (rec && a && b) {
    hipEventRecord(b, c->stream);
    c->pending.push_back({kid, a, b, flop, bytes});
  }
  return LOC_OK;
}

// ------------------------------------------------------------- weight packing
struct Canon {            // canonical (unpacked) layers, row-major W (out x in) and b
  std::vector<const float*> W, b;
  std::vector<int> nout, nin;
};

bool canon_split(const loc_map_desc& d, Canon& cn) {
  const int in_x = 3 + 6 * d.L_xyz, in_d = 3 + 6 * d.L_dir, Wd = d.width;
  std::vector<std::pair<int, int>> sh;
  for (int l = 0; l < d.n_layers; ++l)
    sh.push_back({Wd, l == 0 ? in_x : (l == d.skip_layer ? Wd + in_x : Wd)});
  sh.push_back({1, Wd});
  if (d.dir_width > 0) {
    sh.push_back({Wd, Wd});
    sh.push_back({d.dir_width, Wd + in_d});
    sh.push_back({3, d.dir_width});
  } else {
    sh.push_back({3, Wd + in_d});
  }
  size_t pos = 0;
  for (auto& s : sh) {
    cn.W.push_back(d.params + pos);
    pos += (size_t)s.first * s.second;
    cn.b.push_back(d.params + pos);
    pos += s.first;
    cn.nout.push_back(s.first);
    cn.nin.push_back(s.second);
  }
  return pos == d.n_params;
}

// one dense block: A fragments then permuted biases (maplayout.h)
// in_feature(kb, h) -> canonical input column or -1
template <class FeatFn>
void pack_dense(float* dst, int mto, int kb_total, const float* W, int nin, const float* b, FeatFn in_feature) {
  for (int mt = 0; mt < mto; ++mt)
    for (int kb = 0; kb < kb_total; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int row = 16 * mt + lane % 16;
        const int col = in_feature(kb, lane / 16);
        const long idx = (((long)mt * (kb_total / 4) + kb / 4) * 64 + lane) * 4 + kb % 4;
        dst[idx] = col >= 0 ? W[(long)row * nin + col] : 0.0f;
      }
  float* bias = dst + (long)mto * kb_total * 64;
  for (int mt = 0; mt < mto; ++mt)
    for (int g = 0; g < 4; ++g)
      for (int r = 0; r < 4; ++r) bias[(mt * 4 + g) * 4 + r] = b[16 * mt + 4 * g + r];
}

template <class S>
std::vector<float> pack_map(const loc_map_desc& d) {
  Canon cn;
  canon_split(d, cn);
  std::vector<float> P(S::TOTAL, 0.0f);
  auto chain = [](int kb, int h) { return chain_feature(kb, h); };
  auto gx = [](int kb, int h) { return posenc_feature(S::LX, kb, h); };
  for (int l = 0; l < S::D; ++l) {
    float* dst = P.data() + S::layer_off(l);
    if (l == 0) {
      pack_dense(dst, S::MT, S::KBX, cn.W[0], cn.nin[0], cn.b[0], gx);
    } else if (l == S::SKIP) {
      pack_dense(dst, S::MT, S::KBH + S::KBX, cn.W[l], cn.nin[l], cn.b[l], [](int kb, int h) {
        if (kb < S::KBH) return chain_feature(kb, h);
        const int f = posenc_feature(S::LX, kb - S::KBH, h);
        return f >= 0 ? S::W + f : -1;
      });
    } else {
      pack_dense(dst, S::MT, S::KBH, cn.W[l], cn.nin[l], cn.b[l], chain);
    }
  }
  const int li = S::D;   // sigma head
  float* sig = P.data() + S::SIG_OFF;
  for (int g = 0; g < 4; ++g)
    for (int kb = 0; kb < S::KBH; ++kb) sig[g * S::KBH + kb] = cn.W[li][chain_feature(kb, g)];
  sig[4 * S::KBH] = cn.b[li][0];
  float* rgb = P.data() + S::RGB_OFF;
  if constexpr (S::DW > 0) {
    pack_dense(P.data() + S::FEAT_OFF, S::MT, S::KBH, cn.W[li + 1], cn.nin[li + 1], cn.b[li + 1], chain);
    pack_dense(P.data() + S::DIR_OFF, S::MTD, S::KBH + S::KBD, cn.W[li + 2], cn.nin[li + 2], cn.b[li + 2],
               [](int kb, int h) {
                 if (kb < S::KBH) return chain_feature(kb, h);
                 const int f = posenc_feature(S::LD, kb - S::KBH, h);
                 return f >= 0 ? S::W + f : -1;
               });
    const float* Wc = cn.W[li + 3];
    for (int c = 0; c < 3; ++c)
      for (int g = 0; g < 4; ++g)
        for (int kb = 0; kb < S::KBG; ++kb) rgb[(4 * c + g) * S::KBG + kb] = Wc[c * S::DW + chain_feature(kb, g)];
    for (int c = 0; c < 3; ++c) rgb[12 * S::KBG + c] = cn.b[li + 3][c];
  } else {
    const float* Wc = cn.W[li + 1];
    const int nin = cn.nin[li + 1];
    for (int c = 0; c < 3; ++c)
      for (int g = 0; g < 4; ++g)
        for (int kb = 0; kb < S::KBG; ++kb) {
          int col;
          if (kb < S::KBH) col = chain_feature(kb, g);
          else {
            const int f = posenc_feature(S::LD, kb - S::KBH, g);
            col = f >= 0 ? S::W + f : -1;
          }
          rgb[(4 * c + g) * S::KBG + kb] = col >= 0 ? Wc[c * nin + col] : 0.0f;
        }
    for (int c = 0; c < 3; ++c) rgb[12 * S::KBG + c] = cn.b[li + 1][c];
  }
  return P;
}

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}

struct PackedB {
  std::vector<uint16_t> blocks;   // BLOCKS x 64 lanes x 8 bf16
  std::vector<float> bias, heads;
};

// BF16 chunks, float32 biases and heads (maplayout_bf16.h)
template <class S>
PackedB pack_map_bf16(const loc_map_desc& d) {
  Canon cn;
  canon_split(d, cn);
  PackedB P;
  P.blocks.assign((size_t)S::BLOCKS * 64 * 8, 0);
  P.bias.assign((size_t)S::BIASES, 0.0f);
  P.heads.assign((size_t)S::HEADS, 0.0f);
  // canonical index of layer l (execution order) in cn: hidden 0..D-1, then
  // sigma head at D, feature at D+1, dir at D+2
  for (int l = 0; l < S::NL; ++l) {
    const int ci = l < S::D ? l : l + 1;
    const float* W = cn.W[ci];
    const int nin = cn.nin[ci];
    const int kb_tot = S::layer_kb(l);
    const int kb1 = (l == 0) ? 0 : S::KBH;    // chained k-blocks before the encoding segment
    const int Lenc = (l == 0 || l < S::D) ? S::LX : S::LD;
    const bool has_enc = (l == 0) || (l == S::SKIP) || (l == S::D + 1);
    for (int mt = 0; mt < S::layer_mt(l); ++mt)
      for (int kb = 0; kb < kb_tot; ++kb)
        for (int lane = 0; lane < 64; ++lane)
          for (int q = 0; q < 8; ++q) {
            const int row = 32 * mt + lane % 32, h = lane / 32;
            int col;
            if (kb < kb1) col = chain_feature_b(kb, h, q);
            else if (has_enc) {
              const int f = posenc_feature_b(Lenc, kb - kb1, h, q);
              col = f >= 0 ? (kb1 ? S::W : 0) + f : -1;
            } else col = -1;
            const long blk = S::block_base(l) + (long)mt * kb_tot + kb;
            P.blocks[(size_t)(blk * 64 + lane) * 8 + q] = col >= 0 ? to_bf16(W[(long)row * nin + col]) : 0;
          }
    for (int mt = 0; mt < S::layer_mt(l); ++mt)
      for (int h = 0; h < 2; ++h)
        for (int v = 0; v < 16; ++v)
          P.bias[S::bias_base(l) + (mt * 2 + h) * 16 + v] = cn.b[ci][32 * mt + 8 * (v / 4) + 4 * h + v % 4];
  }
  {
    // tail tiles (maplayout_bf16.h): row r of a tile, lane half h, slot q.
    // A head weight w is carried as two bf16 numbers, hi = bf16(w) in row r
    // and lo = bf16(w - hi) in row r + 8 (16 significant bits in all); the
    // kernels add the two rows' float32 sums
    const int ci = (int)cn.W.size() - 1;   // colour head
    auto put = [&](long blk0, int kb, int lane, int q, float v) {
      const int row = lane % 32;
      if (row >= 8) return;
      const uint16_t hi = to_bf16(v);
      const uint32_t hb = (uint32_t)hi << 16;
      float hv;
      std::memcpy(&hv, &hb, 4);
      P.blocks[(size_t)((blk0 + kb) * 64 + lane) * 8 + q] = hi;
      P.blocks[(size_t)((blk0 + kb) * 64 + lane + 8) * 8 + q] = to_bf16(v - hv);
    };
    for (int kb = 0; kb < S::SIG_KB; ++kb)
      for (int lane = 0; lane < 64; ++lane)
        for (int q = 0; q < 8; ++q) {
          const int row = lane % 32, h = lane / 32;
          float v = 0.0f;
          if (row == 0 && kb < S::KBH) {
            v = cn.W[S::D][chain_feature_b(kb, h, q)];
          } else if (S::DW == 0 && row >= 1 && row <= 3) {
            const int c = row - 1, nin = cn.nin[ci];
            int col;
            if (kb < S::KBH) col = chain_feature_b(kb, h, q);
            else {
              const int f = posenc_feature_b(S::LD, kb - S::KBH, h, q);
              col = f >= 0 ? S::W + f : -1;
            }
            v = col >= 0 ? cn.W[ci][c * nin + col] : 0.0f;
          }
          put(S::SIG_BLOCK, kb, lane, q, v);
        }
    for (int kb = 0; kb < S::RGB_KB; ++kb)
      for (int lane = 0; lane < 64; ++lane)
        for (int q = 0; q < 8; ++q) {
          const int row = lane % 32, h = lane / 32;
          const float v = row < 3 ? cn.W[ci][row * S::DW + chain_feature_b(kb, h, q)] : 0.0f;
          put(S::RGB_BLOCK, kb, lane, q, v);
        }
    for (int h = 0; h < 2; ++h)
      for (int v = 0; v < 16; ++v) {
        const int row = 8 * (v / 4) + 4 * h + v % 4;
        float bs = 0.0f;
        if (row == 0) bs = cn.b[S::D][0];
        else if (S::DW == 0 && row <= 3) bs = cn.b[ci][row - 1];
        P.bias[S::SIG_BIAS + h * 16 + v] = bs;
        if (S::RGB_KB > 0) P.bias[S::RGB_BIAS + h * 16 + v] = row < 3 ? cn.b[ci][row] : 0.0f;
      }
  }
  float* sig = P.heads.data() + S::SIG_OFF;
  for (int h = 0; h < 2; ++h)
    for (int kb = 0; kb < S::KBH; ++kb)
      for (int q = 0; q < 8; ++q) sig[(h * S::KBH + kb) * 8 + q] = cn.W[S::D][chain_feature_b(kb, h, q)];
  sig[16 * S::KBH] = cn.b[S::D][0];
  float* rgb = P.heads.data() + S::RGB_OFF;
  const int ci = (int)cn.W.size() - 1;
  const float* Wc = cn.W[ci];
  const int nin = cn.nin[ci];
  for (int c = 0; c < 3; ++c)
    for (int h = 0; h < 2; ++h)
      for (int kb = 0; kb < S::KBG; ++kb)
        for (int q = 0; q < 8; ++q) {
          int col;
          if (S::DW > 0 || kb < S::KBH) col = chain_feature_b(kb, h, q);
          else {
            const int f = posenc_feature_b(S::LD, kb - S::KBH, h, q);
            col = f >= 0 ? S::W + f : -1;
          }
          rgb[((c * 2 + h) * S::KBG + kb) * 8 + q] = col >= 0 ? Wc[c * nin + col] : 0.0f;
        }
  for (int c = 0; c < 3; ++c) rgb[48 * S::KBG + c] = cn.b[ci][c];
  return P;
}

hipError_t mlp_launch(loc_ctx* c, const MlpArgs& a) {
  if (c->kind == kMapGrid) return launch_grid_map(c->grid, a, c->stream);
  if (a.n_samples2 > 0 && c->desc.precision == LOC_FP32) return hipErrorInvalidValue;   // one set per FP32 launch
  if (c->desc.precision == LOC_FP8_E4M3) {
    MlpArgs b = a;
    b.wblocks = c->wunits;
    b.heads = c->heads_f8;
    // weight scale 2^-ew[l] times the next layer's input scale 2^ea[l+1]:
    // the accumulators come out in the next layer's E4M3 units
    for (int l = 0; l < 12; ++l) {
      b.f8_sw[l] = 127 - c->f8_ew[l] + (l + 1 < 12 ? c->f8_ea[l + 1] : 0);
      b.f8_sx[l] = 127 - c->f8_ea[l];
    }
    return launch_mlp_fp8(c->kind, b, c->stream);
  }
  return c->desc.precision == LOC_BF16 ? launch_mlp_bf16(c->kind, a, c->stream) : launch_mlp(c->kind, a, c->stream);
}

// OCP E4M3 (FN) encoding, round to nearest even, saturating at 448; the
// format: 1 sign, 4 exponent (bias 7), 3 mantissa bits, subnormals below
// 2^-6, no infinities, 0x7f / 0xff NaN
uint8_t to_e4m3(double v) {
  if (std::isnan(v)) return 0x7f;
  const uint8_t sgn = std::signbit(v) ? 0x80 : 0;
  const double a = std::fabs(v);
  if (a == 0.0) return sgn;
  if (a >= 464.0) return sgn | 0x7e;
  int e = (int)std::floor(std::log2(a));
  if (e < -6) e = -6;
  double m = std::nearbyint(a / std::ldexp(1.0, e - 3));   // quantum 2^(e-3), m in [0, 16]
  if (m >= 16.0) { e += 1; m = 8.0; }
  if (m < 8.0) return sgn | (uint8_t)m;                    // subnormal (e == -6)
  return sgn | (uint8_t)((e + 7) << 3) | (uint8_t)(m - 8.0);
}

// exponent e with amax * 2^e <= 448, 2^e as large as possible
int fp8_exponent(double amax) {
  if (!(amax > 0.0) || !std::isfinite(amax)) return 0;
  int e = (int)std::floor(std::log2(448.0 / amax));
  if (std::ldexp(amax, e) > 448.0) --e;
  return e < -60 ? -60 : (e > 60 ? 60 : e);
}

// E4M3 hidden-weight units and BF16 encoding units (maplayout_fp8.h);
// fills ew[l] for l = 1..NL-1.  The encoding weights of layer l carry the
// next layer's input scale 2^ea[l+1] (exact: a power of two)
template <class S>
std::vector<uint8_t> pack_map_fp8(const loc_map_desc& d, int* ew, const int* ea) {
  Canon cn;
  canon_split(d, cn);
  std::vector<uint8_t> U((size_t)S::UNITS * 1024, 0);
  for (int l = 0; l < S::NL; ++l) {
    const int ci = l < S::D ? l : l + 1;
    const float* W = cn.W[ci];
    const int nin = cn.nin[ci], nout = cn.nout[ci];
    const int n_h = l == 0 ? 0 : S::W;
    const int L = (l == S::D + 1) ? S::LD : S::LX;
    int e = 0;
    if (l > 0) {
      double am = 0.0;
      for (int r = 0; r < nout; ++r)
        for (int k = 0; k < n_h; ++k) am = std::fmax(am, std::fabs((double)W[(long)r * nin + k]));
      e = fp8_exponent(am);
      ew[l] = e;
    }
    const int u8 = S::fp8_units(l), ue = S::enc_units(l);
    for (int mt = 0; mt < S::layer_mt(l); ++mt) {
      const long ub = S::unit_base(l) + (long)mt * S::layer_units(l);
      for (int lane = 0; lane < 64; ++lane) {
        const int row = 32 * mt + lane % 32, h = lane / 32;
        for (int kb = 0; kb < u8 / 2; ++kb)
          for (int j = 0; j < 32; ++j) {
            const int col = chain_feature_f8(kb, h, j);
            const long unit = ub + 2 * kb + j / 16;
            U[(size_t)(unit * 64 + lane) * 16 + j % 16] = to_e4m3(std::ldexp((double)W[(long)row * nin + col], e));
          }
        for (int kb = 0; kb < ue; ++kb)
          for (int q = 0; q < 8; ++q) {
            const int f = posenc_feature_b(L, kb, h, q);
            const uint16_t v = f >= 0 ? to_bf16((float)std::ldexp((double)W[(long)row * nin + n_h + f], ea[l + 1])) : 0;
            const long unit = ub + u8 + kb;
            std::memcpy(&U[(size_t)(unit * 64 + lane) * 16 + 2 * q], &v, 2);
          }
      }
    }
  }
  return U;
}

// natural-order heads of the FP8 path: density (W + bias), colour (3 x DW + 3);
// the density weights divided by 2^e_sig, the factor the last trunk layer's
// accumulators carry
template <class S>
std::vector<float> pack_heads_fp8(const loc_map_desc& d, const int e_sig) {
  Canon cn;
  canon_split(d, cn);
  std::vector<float> H((size_t)S::HEADS, 0.0f);
  for (int k = 0; k < S::W; ++k) H[S::SIG_OFF + k] = std::ldexp(cn.W[S::D][k], -e_sig);
  H[S::SIG_OFF + S::W] = cn.b[S::D][0];
  const int ci = (int)cn.W.size() - 1;
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < S::DW; ++k) H[S::RGB_OFF + c * S::DW + k] = cn.W[ci][c * S::DW + k];
  for (int c = 0; c < 3; ++c) H[S::RGB_OFF + 3 * S::DW + c] = cn.b[ci][c];
  return H;
}

// per execution-order layer: transposed weights (in x out), then the bias
template <class S>
std::vector<float> transpose_layers(const loc_map_desc& d) {
  Canon cn;
  canon_split(d, cn);
  std::vector<float> T;
  for (int l = 0; l < S::NL; ++l) {
    const int ci = l < S::D ? l : l + 1;
    const int nin = cn.nin[ci], nout = cn.nout[ci];
    for (int k = 0; k < nin; ++k)
      for (int r = 0; r < nout; ++r) T.push_back(cn.W[ci][(long)r * nin + k]);
    for (int r = 0; r < nout; ++r) T.push_back(cn.b[ci][r]);
  }
  return T;
}

bool same_shape(const loc_map_desc& d, int W, int D, int skip, int lx, int ld, int dw) {
  const int dskip = d.skip_layer >= 1 ? d.skip_layer : -1;
  return d.width == W && d.n_layers == D && dskip == skip && d.L_xyz == lx && d.L_dir == ld &&
         d.dir_width == dw;
}

}  // namespace

namespace {

// Samples of nr rays (ray r = particle r / B, pixel r % B; rays in
// c->ray_o / c->ray_d): stratified coarse samples, fine placement
// (hierarchical or proposal) and the map at every sample, into c->t_c / c->out_c
// and c->t_f / c->out_f.
loc_status map_samples(loc_ctx* c, long nr, int B, uint64_t seed, uint64_t iter) {
  const loc_map_desc& d = c->desc;
  const int Sc = d.n_coarse, Sf = d.n_fine;
  loc_status s;
  MlpArgs ma{};
  ma.ray_o = c->ray_o.p;
  ma.ray_d = c->ray_d.p;
  ma.t_in = nullptr;
  ma.t_out = c->t_c.p;
  ma.out = c->out_c.p;
  ma.weights = c->weights;
  ma.wblocks = c->wblocks;
  ma.bias = c->bias_b;
  ma.heads = c->heads_b;
  ma.n_samples = nr * Sc;
  ma.spr = Sc;
  ma.B = B;
  ma.near_ = d.near_;
  ma.dt = (d.far_ - d.near_) / (float)Sc;
  ma.jitter = d.jitter;
  ma.seed = seed;
  ma.iter = iter;
  const double fl_sample = 2.0 * (double)c->macs;
  // with proposal-placed fine samples (which do not depend on the coarse
  // render) the MFMA paths evaluate coarse and fine samples in one launch
  const bool merged = Sf > 0 && c->fine_mode == 1 && d.precision != LOC_FP32;
  if (!merged && (s = timed(c, K_MLP_COARSE, fl_sample * ma.n_samples, c->bytes_per_sample * ma.n_samples + 32.0 * nr,
                            [&] { return mlp_launch(c, ma); })))
    return s;

  if (Sf > 0 && c->fine_mode == 1) {
    ProposalArgs pa2{};
    pa2.ray_o = c->ray_o.p;
    pa2.ray_d = c->ray_d.p;
    pa2.params = c->prop;
    pa2.hist = nullptr;
    pa2.t_fine = c->t_f.p;
    pa2.n_rays = (int)nr;
    pa2.Sf = Sf;
    pa2.B = B;
    pa2.near_ = d.near_;
    pa2.far_ = d.far_;
    pa2.jitter = d.jitter;
    pa2.seed = seed;
    pa2.iter = iter;
    if ((s = timed(c, K_PROPOSAL, 2.0 * 11136.0 * nr, 40.0 * nr + 4.0 * nr * Sf,
                   [&] { return launch_proposal_fine(pa2, c->stream); })))
      return s;
  }
  if (Sf > 0) {
    FineArgs fa{};
    fa.t_coarse = c->t_c.p;
    fa.out_coarse = c->out_c.p;
    fa.t_fine = c->t_f.p;
    fa.n_rays = (int)nr;
    fa.Sc = Sc;
    fa.Sf = Sf;
    fa.B = B;
    fa.far_ = d.far_;
    fa.jitter = d.jitter;
    fa.seed = seed;
    fa.iter = iter;
    if (c->fine_mode == 0 &&
        (s = timed(c, K_FINE, 0, nr * (8.0 * Sc + 4.0 * Sf), [&] { return launch_fine(fa, c->stream); })))
      return s;
    if (merged) {
      MlpArgs mb = ma;
      mb.t_in2 = c->t_f.p;
      mb.out2 = c->out_f.p;
      mb.n_samples2 = nr * Sf;
      mb.spr2 = Sf;
      const double n_all = (double)(ma.n_samples + mb.n_samples2);
      if ((s = timed(c, K_MLP_BOTH, fl_sample * n_all, c->bytes_per_sample * n_all + 4.0 * mb.n_samples2 + 32.0 * nr,
                     [&] { return mlp_launch(c, mb); })))
        return s;
    } else {
      MlpArgs mf = ma;
      mf.t_in = c->t_f.p;
      mf.t_out = nullptr;
      mf.out = c->out_f.p;
      mf.n_samples = nr * Sf;
      mf.spr = Sf;
      if ((s = timed(c, K_MLP_FINE, fl_sample * mf.n_samples, c->bytes_per_sample * mf.n_samples + 32.0 * nr,
                     [&] { return mlp_launch(c, mf); })))
        return s;
    }
  }

  return LOC_OK;
}

}  // namespace

extern "C" {

const char* loc_status_str(loc_status s) {
  switch (s) {
    case LOC_OK: return "ok";
    case LOC_E_ARG: return "invalid argument";
    case LOC_E_HIP: return "HIP runtime error";
    case LOC_E_OOM: return "out of device memory";
    case LOC_E_DEGENERATE: return "degenerate weights";
    case LOC_E_UNSUPPORTED: return "unsupported map shape or precision";
    case LOC_E_STATE: return "invalid call order";
  }
  return "unknown status";
}

const char* loc_last_error(const loc_ctx* c) { return c ? c->err.c_str() : ""; }

loc_status loc_init_map(const loc_map_desc* d, void* hip_stream, loc_ctx** out) {
  if (!out) return LOC_E_ARG;
  *out = nullptr;
  if (!d || !d->params) return LOC_E_ARG;
  if (!(d->near_ >= 0.0f && d->far_ > d->near_)) return LOC_E_ARG;
  if (d->n_coarse < 1 || d->n_coarse > 256 || d->n_fine < 0 || d->n_fine > 256) return LOC_E_ARG;
  if (!(d->alpha > 0.0f && d->alpha < 0.5f) || !(d->tau > 0.0f)) return LOC_E_ARG;
  if (d->precision != LOC_FP32 && d->precision != LOC_BF16 && d->precision != LOC_FP8_E4M3) return LOC_E_UNSUPPORTED;
  int kind;
  long macs, total;
  if (same_shape(*d, 64, 4, -1, 6, 2, 0)) { kind = kMapSmall; macs = SmallMap::macs(); total = SmallMap::TOTAL; }
  else if (same_shape(*d, 256, 8, 5, 10, 4, 128)) { kind = kMapNerf; macs = NerfMap::macs(); total = NerfMap::TOTAL; }
  else return LOC_E_UNSUPPORTED;
  if (d->precision == LOC_FP8_E4M3 && kind != kMapNerf) return LOC_E_UNSUPPORTED;
  Canon cn;
  if (!canon_split(*d, cn)) return LOC_E_ARG;
  loc_ctx* c = new (std::nothrow) loc_ctx();
  if (!c) return LOC_E_OOM;
  c->desc = *d;
  c->desc.params = nullptr;
  c->kind = kind;
  c->macs = macs;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return LOC_E_HIP; }
  if (noalloc_scratch(c->device, &c->noalloc_prefix) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return LOC_E_HIP;
  }
  if (hipMalloc(&c->flags, sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    loc_destroy(c);
    return LOC_E_OOM;
  }
  c->params_host.assign(d->params, d->params + d->n_params);
  bool ok = true;
  if (d->precision == LOC_FP32) {
    std::vector<float> P = kind == kMapSmall ? pack_map<SmallMap>(*d) : pack_map<NerfMap>(*d);
    ok = hipMalloc(&c->weights, sizeof(float) * total) == hipSuccess &&
         hipMemcpy(c->weights, P.data(), sizeof(float) * total, hipMemcpyHostToDevice) == hipSuccess;
  } else if (d->precision == LOC_FP8_E4M3) {
    // biases as in the BF16 layout; weights are packed by loc_calibrate_fp8
    PackedB P = pack_map_bf16<NerfMapB>(*d);
    std::vector<float> H = pack_heads_fp8<NerfMapF8>(*d, 0);
    ok = hipMalloc(&c->bias_b, P.bias.size() * 4) == hipSuccess &&
         hipMalloc(&c->heads_f8, H.size() * 4) == hipSuccess &&
         hipMalloc(&c->wunits, (size_t)NerfMapF8::UNITS * 1024) == hipSuccess &&
         hipMemcpy(c->bias_b, P.bias.data(), P.bias.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->heads_f8, H.data(), H.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  } else {
    PackedB P = kind == kMapSmall ? pack_map_bf16<SmallMapB>(*d) : pack_map_bf16<NerfMapB>(*d);
    ok = hipMalloc(&c->wblocks, P.blocks.size() * 2) == hipSuccess &&
         hipMalloc(&c->bias_b, P.bias.size() * 4) == hipSuccess &&
         hipMalloc(&c->heads_b, P.heads.size() * 4) == hipSuccess &&
         hipMemcpy(c->wblocks, P.blocks.data(), P.blocks.size() * 2, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->bias_b, P.bias.data(), P.bias.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->heads_b, P.heads.data(), P.heads.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok || hipMemsetAsync(c->flags, 0, sizeof(int), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    loc_destroy(c);
    return LOC_E_HIP;
  }
  *out = c;
  return LOC_OK;
}

void loc_destroy(loc_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  hipFree(c->weights);
  hipFree(c->wblocks);
  hipFree(c->bias_b);
  hipFree(c->heads_b);
  hipFree(c->wunits);
  hipFree(c->heads_f8);
  hipFree(c->grid_tab);
  hipFree(c->grid_mlp);
  hipFree(c->grid_feat);
  hipFree(c->grid_pts);
  hipFree(c->flags);
  hipFree(c->ray_o.p); hipFree(c->ray_d.p); hipFree(c->obs.p); hipFree(c->out_c.p); hipFree(c->out_f.p);
  hipFree(c->rgba.p); hipFree(c->fe.p); hipFree(c->t_c.p); hipFree(c->t_f.p); hipFree(c->prefix.p);
  hipFree(c->prop); hipFree(c->prop_m); hipFree(c->prop_v); hipFree(c->prop_partial.p); hipFree(c->prop_loss.p);
  hipFree(c->tr_o.p); hipFree(c->tr_d.p);
  for (auto& b : c->lz_x) hipFree(b.p);
  hipFree(c->tm_params.p); hipFree(c->tm_m.p); hipFree(c->tm_v.p); hipFree(c->tm_partial.p); hipFree(c->tm_lpart.p);
  hipFree(c->lz_pred.p); hipFree(c->lz_ll.p); hipFree(c->lz_w.p); hipFree(c->lz_ve.p); hipFree(c->lz_idx.p);
  if (c->lz_host) hipHostFree(c->lz_host);
  for (auto& L : c->lv) {
    hipFree(L.pose.p); hipFree(L.loglik.p); hipFree(L.weight.p); hipFree(L.uncert.p); hipFree(L.idx.p);
    hipFree(L.rgba.p); hipFree(L.fe.p); hipFree(L.inc.p);
  }
  hipFree(c->key);
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->graph) hipGraphDestroy(c->graph);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (auto& p : c->pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
  for (auto e : c->free_events) hipEventDestroy(e);
  delete c;
}

loc_status loc_update_particles(loc_ctx* c, const float* image, const loc_camera* cam, int inv_R, int B, int N,
                                const double* pose_in, const double* motion, double sigma_t, double sigma_r,
                                uint64_t seed, uint64_t iter, double* pose_out, double* loglik_out,
                                double* weight_out, float* uncert_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!image || !cam || !pose_in || !pose_out || !loglik_out || !weight_out)
    return fail(c, LOC_E_ARG, "null pointer argument");
  if (inv_R != 1 && inv_R != 2 && inv_R != 4 && inv_R != 8) return fail(c, LOC_E_ARG, "inv_R must be 1, 2, 4 or 8");
  if (c->fine_mode == 1 && !c->prop) return fail(c, LOC_E_STATE, "proposal mode without proposal parameters");
  if (c->desc.precision == LOC_FP8_E4M3 && !c->f8_ready)
    return fail(c, LOC_E_STATE, "FP8 map used before loc_calibrate_fp8");
  if (cam->W <= 0 || cam->H <= 0 || cam->W % inv_R || cam->H % inv_R)
    return fail(c, LOC_E_ARG, "image %dx%d not divisible by level factor %d", cam->W, cam->H, inv_R);
  if (!(cam->fx > 0 && cam->fy > 0) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(c, LOC_E_ARG, "invalid intrinsics");
  if (B < 1 || B > 1024) return fail(c, LOC_E_ARG, "B must be in [1, 1024]");
  if (N < 1 || (long)N * B > (1L << 30) / 256) return fail(c, LOC_E_ARG, "N out of range");
  if (!(sigma_t >= 0.0) || !(sigma_r >= 0.0)) return fail(c, LOC_E_ARG, "negative noise scale");
  const loc_map_desc& d = c->desc;
  const int Sc = d.n_coarse, Sf = d.n_fine;
  const long nr = (long)N * B;
  loc_status s;
  if ((s = ensure(c, c->ray_o, nr)) || (s = ensure(c, c->ray_d, nr)) || (s = ensure(c, c->obs, nr)) ||
      (s = ensure(c, c->rgba, nr)) || (s = ensure(c, c->fe, nr)) || (s = ensure(c, c->t_c, nr * Sc)) ||
      (s = ensure(c, c->out_c, nr * Sc)))
    return s;
  if (Sf > 0 && ((s = ensure(c, c->t_f, nr * Sf)) || (s = ensure(c, c->out_f, nr * Sf)))) return s;
  {
    hipError_t pe = hipGetLastError();
    if (pe != hipSuccess) return fail(c, LOC_E_HIP, "pending HIP error: %s", hipGetErrorString(pe));
  }

  PredictArgs pa{};
  pa.pose_in = pose_in;
  pa.pose_out = pose_out;
  for (int q = 0; q < 12; ++q) pa.motion.m[q] = motion ? motion[q] : ((q % 5 == 0) ? 1.0 : 0.0);
  pa.sigma_t = sigma_t;
  pa.sigma_r = sigma_r;
  pa.N = N;
  pa.seed = seed;
  pa.iter = iter;
  if ((s = timed(c, K_PREDICT, 0, 192.0 * N, [&] { return launch_predict(pa, c->stream); }))) return s;

  RaygenArgs ra{};
  ra.pose = pose_out;
  ra.image = image;
  ra.W_full = cam->W;
  ra.s = inv_R;
  ra.Wl = cam->W / inv_R;
  ra.Hl = cam->H / inv_R;
  ra.fx = cam->fx / inv_R;
  ra.fy = cam->fy / inv_R;
  ra.cx = cam->cx / inv_R;
  ra.cy = cam->cy / inv_R;
  ra.N = N;
  ra.B = B;
  ra.seed = seed;
  ra.iter = iter;
  ra.ray_o = c->ray_o.p;
  ra.ray_d = c->ray_d.p;
  ra.obs = c->obs.p;
  if ((s = timed(c, K_RAYGEN, 0, nr * (48.0 + 12.0 * inv_R * inv_R) + 96.0 * N,
                 [&] { return launch_raygen(ra, c->stream); })))
    return s;

  if ((s = map_samples(c, nr, B, seed, iter))) return s;

  CompositeArgs ca{};
  ca.t_coarse = c->t_c.p;
  ca.out_coarse = c->out_c.p;
  ca.t_fine = Sf > 0 ? c->t_f.p : nullptr;
  ca.out_fine = Sf > 0 ? c->out_f.p : nullptr;
  ca.obs = c->obs.p;
  ca.N = N;
  ca.B = B;
  ca.Sc = Sc;
  ca.Sf = Sf;
  ca.far_ = d.far_;
  ca.log_trans = (float)std::log1p(-(double)d.alpha);
  ca.log_opq = (float)std::log((double)d.alpha);
  ca.tau = d.tau;
  ca.empty_F = c->empty_span ? d.far_ - d.near_ : d.tau;
  ca.ray_rgba = c->rgba.p;
  ca.ray_fe = c->fe.p;
  ca.loglik = loglik_out;
  ca.uncert = uncert_out;
  ca.hist = nullptr;
  ca.n_rays = (int)nr;
  ca.near_ = d.near_;
  if ((s = timed(c, K_COMPOSITE, 0, nr * (20.0 * (Sc + Sf) + 16.0 + 24.0) + 12.0 * N,
                 [&] { return launch_composite(ca, c->stream); })))
    return s;
  if ((s = timed(c, K_NORMALIZE, 0, 16.0 * N,
                 [&] { return launch_normalize(loglik_out, weight_out, N, c->flags, c->stream); })))
    return s;
  c->last_N = N;
  c->last_B = B;
  return LOC_OK;
}

loc_status loc_resample(loc_ctx* c, const double* weight, int n_in, int n_out, uint64_t seed, uint64_t iter,
                        int32_t* idx_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!weight || !idx_out) return fail(c, LOC_E_ARG, "null pointer argument");
  // n_in < 2^24 keeps Q = sum q_i (each q_i <= 2^40) below 2^64
  if (n_in < 1 || n_in >= (1 << 24) || n_out < 1 || n_out > (1 << 24))
    return fail(c, LOC_E_ARG, "n_in must be in [1, 2^24 - 1] and n_out in [1, 2^24]");
  loc_status s;
  if ((s = ensure(c, c->prefix, (size_t)n_in))) return s;
  return timed(c, K_RESAMPLE, 0, 8.0 * n_in * 2 + 4.0 * n_out, [&] {
    return launch_resample(weight, n_in, n_out, seed, iter, c->prefix.p, idx_out, c->flags, c->stream);
  });
}

static_assert(LOC_NOALLOC_MAX_WEIGHTS == fl::kNoAllocMaxWeights, "scratch size");

loc_status loc_resample_noalloc(loc_ctx* c, const double* weight, int n_in, int n_out, uint64_t seed,
                                uint64_t iter, int32_t* idx_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!weight || !idx_out) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n_in < 1 || n_in > LOC_NOALLOC_MAX_WEIGHTS || n_out < 1 || n_out > (1 << 24))
    return fail(c, LOC_E_ARG, "n_in must be in [1, %d] (the fixed scratch) and n_out in [1, 2^24]",
                LOC_NOALLOC_MAX_WEIGHTS);
  if (!c->noalloc_prefix) return fail(c, LOC_E_STATE, "scratch address not resolved at init");
  const hipError_t e = launch_resample(weight, n_in, n_out, seed, iter, c->noalloc_prefix, idx_out, c->flags,
                                       c->stream);
  if (e != hipSuccess) return fail(c, LOC_E_HIP, "launch of k_resample failed: %s", hipGetErrorString(e));
  return LOC_OK;
}

loc_status loc_ray_outputs(loc_ctx* c, float* rgb, float* opacity, float* F, float* E) {
  if (!c) return LOC_E_ARG;
  if (c->last_N == 0) return fail(c, LOC_E_STATE, "no update has run on this context");
  const int n = c->last_N * c->last_B;
  return timed(c, K_SPLIT, 0, 24.0 * n, [&] {
    return launch_split_ray_outputs(c->rgba.p, c->fe.p, n, rgb, opacity, F, E, c->stream);
  });
}

loc_status loc_sync(loc_ctx* c, int* flags) {
  if (!c) return LOC_E_ARG;
  int h = 0;
  HIP_TRY(c, hipMemcpyAsync(&h, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (flags) *flags = h;
  return LOC_OK;
}

loc_status loc_set_profiling(loc_ctx* c, int enable) {
  if (!c) return LOC_E_ARG;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) { c->free_events.push_back(p.a); c->free_events.push_back(p.b); }
  c->pending.clear();
  for (int k = 0; k < K_COUNT; ++k) { c->launches[k] = 0; c->ms[k] = c->flop[k] = c->bytes[k] = 0.0; }
  if (enable < 0 || enable > 2) return fail(c, LOC_E_ARG, "profiling mode must be 0, 1 or 2");
  c->prof = enable;
  return LOC_OK;
}

loc_status loc_kernel_stats(loc_ctx* c, loc_kernel_stat* out, int max, int* n) {
  if (!c || (max > 0 && !out)) return LOC_E_ARG;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->launches[p.kid] += 1;
    c->ms[p.kid] += ms;
    c->flop[p.kid] += p.flop;
    c->bytes[p.kid] += p.bytes;
    c->free_events.push_back(p.a);
    c->free_events.push_back(p.b);
  }
  c->pending.clear();
  int k_out = 0;
  for (int k = 0; k < K_COUNT; ++k) {
    if (c->launches[k] == 0) continue;
    if (k_out < max) {
      loc_kernel_stat& st = out[k_out];
      std::memset(&st, 0, sizeof st);
      std::strncpy(st.name, kKernelNames[k], sizeof st.name - 1);
      st.launches = c->launches[k];
      st.ms = c->ms[k];
      st.flop = c->flop[k];
      st.bytes = c->bytes[k];
    }
    ++k_out;
  }
  if (n) *n = k_out;
  return LOC_OK;
}


loc_status loc_cast_rays(loc_ctx* c, const loc_camera* cam, int inv_R, int B, int N, const double* pose,
                         uint64_t seed, uint64_t iter, float* ray_o, float* ray_d) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!cam || !pose || !ray_o || !ray_d) return fail(c, LOC_E_ARG, "null pointer argument");
  if (inv_R != 1 && inv_R != 2 && inv_R != 4 && inv_R != 8) return fail(c, LOC_E_ARG, "inv_R must be 1, 2, 4 or 8");
  if (cam->W <= 0 || cam->H <= 0 || cam->W % inv_R || cam->H % inv_R || !(cam->fx > 0 && cam->fy > 0))
    return fail(c, LOC_E_ARG, "invalid camera for level factor %d", inv_R);
  if (B < 1 || B > 1024 || N < 1 || (long)N * B > (1L << 30) / 256) return fail(c, LOC_E_ARG, "N or B out of range");
  const long nr = (long)N * B;
  loc_status s;
  if ((s = ensure(c, c->tr_o, nr)) || (s = ensure(c, c->tr_d, nr))) return s;
  RaygenArgs ra{};
  ra.pose = pose;
  ra.image = nullptr;
  ra.W_full = cam->W;
  ra.s = inv_R;
  ra.Wl = cam->W / inv_R;
  ra.Hl = cam->H / inv_R;
  ra.fx = cam->fx / inv_R;
  ra.fy = cam->fy / inv_R;
  ra.cx = cam->cx / inv_R;
  ra.cy = cam->cy / inv_R;
  ra.N = N;
  ra.B = B;
  ra.seed = seed;
  ra.iter = iter;
  ra.ray_o = c->tr_o.p;
  ra.ray_d = c->tr_d.p;
  ra.obs = nullptr;
  if ((s = timed(c, K_RAYGEN, 0, 32.0 * nr + 96.0 * N, [&] { return launch_raygen(ra, c->stream); }))) return s;
  return timed(c, K_RAYS, 0, 56.0 * nr,
               [&] { return launch_rays_from_f4(c->tr_o.p, c->tr_d.p, (int)nr, ray_o, ray_d, c->stream); });
}

loc_status loc_teacher_histograms(loc_ctx* c, const float* ray_o, const float* ray_d, int n, int n_fine,
                                  uint64_t seed, uint64_t iter, float* hist) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!ray_o || !ray_d || !hist) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n < 1 || n > (1 << 24)) return fail(c, LOC_E_ARG, "n out of range");
  if (n_fine < 0 || n_fine > 256) return fail(c, LOC_E_ARG, "n_fine must be in [0, 256]");
  if (c->desc.precision == LOC_FP8_E4M3 && !c->f8_ready)
    return fail(c, LOC_E_STATE, "FP8 map used before loc_calibrate_fp8");
  const loc_map_desc& d = c->desc;
  const int Sc = d.n_coarse, Sf = n_fine;
  loc_status s;
  if ((s = ensure(c, c->ray_o, n)) || (s = ensure(c, c->ray_d, n)) || (s = ensure(c, c->t_c, (size_t)n * Sc)) ||
      (s = ensure(c, c->out_c, (size_t)n * Sc)) || (s = ensure(c, c->rgba, n)) || (s = ensure(c, c->fe, n)))
    return s;
  if (Sf > 0 && ((s = ensure(c, c->t_f, (size_t)n * Sf)) || (s = ensure(c, c->out_f, (size_t)n * Sf)))) return s;
  if ((s = timed(c, K_RAYS, 0, 56.0 * n,
                 [&] { return launch_rays_to_f4(ray_o, ray_d, n, c->ray_o.p, c->ray_d.p, c->stream); })))
    return s;
  MlpArgs ma{};
  ma.ray_o = c->ray_o.p;
  ma.ray_d = c->ray_d.p;
  ma.t_out = c->t_c.p;
  ma.out = c->out_c.p;
  ma.weights = c->weights;
  ma.wblocks = c->wblocks;
  ma.bias = c->bias_b;
  ma.heads = c->heads_b;
  ma.n_samples = (long)n * Sc;
  ma.spr = Sc;
  ma.B = 1;                      // streams keyed (ray, 0)
  ma.near_ = d.near_;
  ma.dt = (d.far_ - d.near_) / (float)Sc;
  ma.jitter = d.jitter;
  ma.seed = seed;
  ma.iter = iter;
  const double fl_sample = 2.0 * (double)c->macs;
  if ((s = timed(c, K_MLP_COARSE, fl_sample * ma.n_samples, 20.0 * ma.n_samples, [&] { return mlp_launch(c, ma); })))
    return s;
  if (Sf > 0) {
    FineArgs fa{};
    fa.t_coarse = c->t_c.p;
    fa.out_coarse = c->out_c.p;
    fa.t_fine = c->t_f.p;
    fa.n_rays = n;
    fa.Sc = Sc;
    fa.Sf = Sf;
    fa.B = 1;
    fa.far_ = d.far_;
    fa.jitter = d.jitter;
    fa.seed = seed;
    fa.iter = iter;
    if ((s = timed(c, K_FINE, 0, (double)n * (8.0 * Sc + 4.0 * Sf), [&] { return launch_fine(fa, c->stream); })))
      return s;
    MlpArgs mf = ma;
    mf.t_in = c->t_f.p;
    mf.t_out = nullptr;
    mf.out = c->out_f.p;
    mf.n_samples = (long)n * Sf;
    mf.spr = Sf;
    if ((s = timed(c, K_MLP_FINE, fl_sample * mf.n_samples, 20.0 * mf.n_samples, [&] { return mlp_launch(c, mf); })))
      return s;
  }
  CompositeArgs ca{};
  ca.t_coarse = c->t_c.p;
  ca.out_coarse = c->out_c.p;
  ca.t_fine = Sf > 0 ? c->t_f.p : nullptr;
  ca.out_fine = Sf > 0 ? c->out_f.p : nullptr;
  ca.obs = nullptr;
  ca.N = (n + 3) / 4;
  ca.B = 4;
  ca.Sc = Sc;
  ca.Sf = Sf;
  ca.far_ = d.far_;
  ca.log_trans = (float)std::log1p(-(double)d.alpha);
  ca.log_opq = (float)std::log((double)d.alpha);
  ca.tau = d.tau;
  ca.empty_F = c->empty_span ? d.far_ - d.near_ : d.tau;
  ca.ray_rgba = c->rgba.p;
  ca.ray_fe = c->fe.p;
  ca.loglik = nullptr;
  ca.uncert = nullptr;
  ca.hist = hist;
  ca.n_rays = n;
  ca.near_ = d.near_;
  return timed(c, K_TEACHER, 0, (double)n * (20.0 * (Sc + Sf) + 128.0),
               [&] { return launch_composite(ca, c->stream); });
}

loc_status loc_set_proposal(loc_ctx* c, const float* params, size_t n) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!params || n != (size_t)kProposalParams)
    return fail(c, LOC_E_ARG, "proposal parameters: expected %d floats", kProposalParams);
  if (!c->prop) {
    if (hipMalloc(&c->prop, 4 * kProposalParams) != hipSuccess || hipMalloc(&c->prop_m, 4 * kProposalParams) != hipSuccess ||
        hipMalloc(&c->prop_v, 4 * kProposalParams) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, LOC_E_OOM, "proposal allocation failed");
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->prop, params, 4 * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->prop_m, 0, 4 * n, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->prop_v, 0, 4 * n, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->prop_step = 0;
  return LOC_OK;
}

loc_status loc_get_proposal(loc_ctx* c, float* params, size_t n) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!params || n != (size_t)kProposalParams)
    return fail(c, LOC_E_ARG, "proposal parameters: expected %d floats", kProposalParams);
  if (!c->prop) return fail(c, LOC_E_STATE, "no proposal parameters set");
  HIP_TRY(c, hipMemcpyAsync(params, c->prop, 4 * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LOC_OK;
}

loc_status loc_set_fine_mode(loc_ctx* c, int mode) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (mode != 0 && mode != 1) return fail(c, LOC_E_ARG, "fine mode must be 0 (hierarchical) or 1 (proposal)");
  if (mode == 1 && !c->prop) return fail(c, LOC_E_STATE, "no proposal parameters set");
  c->fine_mode = mode;
  return LOC_OK;
}

loc_status loc_proposal_forward(loc_ctx* c, const float* ray_o, const float* ray_d, int n, float* hist) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!ray_o || !ray_d || !hist) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n < 1 || n > (1 << 24)) return fail(c, LOC_E_ARG, "n out of range");
  if (!c->prop) return fail(c, LOC_E_STATE, "no proposal parameters set");
  loc_status s;
  if ((s = ensure(c, c->tr_o, n)) || (s = ensure(c, c->tr_d, n))) return s;
  if ((s = timed(c, K_RAYS, 0, 56.0 * n,
                 [&] { return launch_rays_to_f4(ray_o, ray_d, n, c->tr_o.p, c->tr_d.p, c->stream); })))
    return s;
  ProposalArgs pa{};
  pa.ray_o = c->tr_o.p;
  pa.ray_d = c->tr_d.p;
  pa.params = c->prop;
  pa.hist = hist;
  pa.n_rays = n;
  pa.Sf = 0;
  pa.B = 1;
  return timed(c, K_PROPOSAL, 2.0 * 11136.0 * n, 160.0 * n, [&] { return launch_proposal_fine(pa, c->stream); });
}

namespace {
constexpr int kRaysPerWave = 32;

// the proposal trains in the map's precision: float32 on the vector ALU for a
// float32 context, bf16 operands on the matrix cores otherwise
bool prop_bf16(const loc_ctx* c) { return c->desc.precision != LOC_FP32; }

loc_status prop_prepare(loc_ctx* c, const float* ray_o, const float* ray_d, int n, int batch, TrainArgs& ta) {
  loc_status s;
  const int rpw = prop_bf16(c) ? prop_rays_per_wave_bf16() : kRaysPerWave;
  const int n_waves = (batch + rpw - 1) / rpw;
  if ((s = ensure(c, c->tr_o, n)) || (s = ensure(c, c->tr_d, n)) ||
      (s = ensure(c, c->prop_partial, (size_t)n_waves * kProposalParams)) || (s = ensure(c, c->prop_loss, n_waves)))
    return s;
  if ((s = timed(c, K_RAYS, 0, 56.0 * n,
                 [&] { return launch_rays_to_f4(ray_o, ray_d, n, c->tr_o.p, c->tr_d.p, c->stream); })))
    return s;
  ta = TrainArgs{};
  ta.ray_o = c->tr_o.p;
  ta.ray_d = c->tr_d.p;
  ta.params = c->prop;
  ta.partial = c->prop_partial.p;
  ta.loss_partial = c->prop_loss.p;
  ta.n_rays = n;
  ta.batch = batch;
  ta.rays_per_wave = rpw;
  ta.n_waves = n_waves;
  return LOC_OK;
}

hipError_t launch_prop_step(const loc_ctx* c, const TrainArgs& ta) {
  return prop_bf16(c) ? launch_prop_grad_bf16(ta, c->stream) : launch_prop_grad(ta, c->stream);
}
}  // namespace

loc_status loc_proposal_grad(loc_ctx* c, const float* ray_o, const float* ray_d, const float* target, int n,
                             float* loss_out, float* grad_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!ray_o || !ray_d || !target || !grad_out) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n < 1 || n > (1 << 20)) return fail(c, LOC_E_ARG, "n must be in [1, 2^20]");
  if (!c->prop) return fail(c, LOC_E_STATE, "no proposal parameters set");
  TrainArgs ta;
  loc_status s;
  if ((s = prop_prepare(c, ray_o, ray_d, n, n, ta))) return s;
  ta.target = target;
  ta.first = 0;
  ta.loss_out = loss_out;
  ta.loss_index = 0;
  ta.grad_out = grad_out;
  ta.adam = 0;
  return timed(c, K_TRAIN, 3.0 * 2.0 * 11136.0 * n, 0.0, [&] { return launch_prop_step(c, ta); });
}

loc_status loc_train_proposal(loc_ctx* c, const float* ray_o, const float* ray_d, const float* target, int n,
                              const loc_train_cfg* cfg, float* loss_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!ray_o || !ray_d || !target || !cfg) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n < 1 || n > (1 << 24)) return fail(c, LOC_E_ARG, "n out of range");
  if (cfg->batch < 1 || cfg->batch > (1 << 20) || cfg->steps < 0) return fail(c, LOC_E_ARG, "batch or steps out of range");
  if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f))
    return fail(c, LOC_E_ARG, "invalid Adam hyperparameters");
  if (!c->prop) return fail(c, LOC_E_STATE, "no proposal parameters set");
  TrainArgs ta;
  loc_status s;
  if ((s = prop_prepare(c, ray_o, ray_d, n, cfg->batch, ta))) return s;
  ta.target = target;
  ta.params_rw = c->prop;
  ta.m = c->prop_m;
  ta.v = c->prop_v;
  ta.loss_out = loss_out;
  ta.grad_out = nullptr;
  ta.adam = 1;
  ta.lr = cfg->lr;
  ta.beta1 = cfg->beta1;
  ta.beta2 = cfg->beta2;
  ta.eps = cfg->eps;
  for (int k = 0; k < cfg->steps; ++k) {
    ta.first = (int)(((long)k * cfg->batch) % n);
    ta.loss_index = k;
    ta.step = ++c->prop_step;
    if ((s = timed(c, K_TRAIN, 3.0 * 2.0 * 11136.0 * cfg->batch, 0.0, [&] { return launch_prop_step(c, ta); })))
      return s;
  }
  return LOC_OK;
}


loc_status loc_gather_poses(loc_ctx* c, const double* pose_in, int n_in, const int32_t* idx, int n_out,
                            double* pose_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!pose_in || !idx || !pose_out) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n_in < 1 || n_in > (1 << 24) || n_out < 1 || n_out > (1 << 24))
    return fail(c, LOC_E_ARG, "n_in and n_out must be in [1, 2^24]");
  return timed(c, K_GATHER, 0, 96.0 * 2 * n_out + 4.0 * n_out, [&] {
    return launch_gather_poses(pose_in, idx, n_in, n_out, pose_out, c->stream);
  });
}

loc_status loc_pose_estimate(loc_ctx* c, const double* pose, const double* weight, int N, double* est) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!pose || !weight || !est) return fail(c, LOC_E_ARG, "null pointer argument");
  if (N < 1 || N > (1 << 24)) return fail(c, LOC_E_ARG, "N must be in [1, 2^24]");
  return timed(c, K_ESTIMATE, 0, 104.0 * N, [&] { return launch_pose_estimate(pose, weight, N, est, c->flags, c->stream); });
}


loc_status loc_calibrate_fp8(loc_ctx* c, const float* o, const float* d, int n_rays) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (c->desc.precision != LOC_FP8_E4M3) return fail(c, LOC_E_STATE, "context precision is not FP8");
  if (!o || !d) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n_rays < 1 || n_rays > (1 << 20)) return fail(c, LOC_E_ARG, "n_rays must be in [1, 2^20]");
  using S = NerfMapF8;
  loc_map_desc pd = c->desc;
  pd.params = c->params_host.data();
  std::vector<float> T = transpose_layers<S>(pd);
  float* wt = nullptr;
  unsigned* am = nullptr;
  auto cleanup = [&] { hipFree(wt); hipFree(am); };
  if (hipMalloc(&wt, T.size() * 4) != hipSuccess || hipMalloc(&am, 16 * sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(c, LOC_E_OOM, "calibration buffers");
  }
  CalibArgs ca{};
  ca.o = o;
  ca.d = d;
  ca.n_rays = n_rays;
  ca.spr = c->desc.n_coarse;
  ca.near_ = c->desc.near_;
  ca.dt = (c->desc.far_ - c->desc.near_) / (float)c->desc.n_coarse;
  ca.wt = wt;
  ca.amax = am;
  unsigned h_am[16] = {};
  hipError_t e = hipMemcpyAsync(wt, T.data(), T.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(am, 0, 16 * sizeof(unsigned), c->stream);
  if (e == hipSuccess) {
    loc_status s = timed(c, K_CALIB, 2.0 * (double)c->macs * n_rays * ca.spr, 0.0,
                         [&] { return launch_calibrate_fp8(ca, c->stream); });
    if (s) { hipStreamSynchronize(c->stream); cleanup(); return s; }
    e = hipMemcpyAsync(h_am, am, sizeof h_am, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) return fail(c, LOC_E_HIP, "calibration: %s", hipGetErrorString(e));
  // activation exponent of layer l's input = output range of layer l - 1
  for (int l = 0; l < 12; ++l) { c->f8_ea[l] = 0; c->f8_ew[l] = 0; c->f8_amax[l] = 0.0f; }
  for (int l = 0; l <= S::D; ++l) {
    float v;
    std::memcpy(&v, &h_am[l], 4);
    c->f8_amax[l] = v;
    c->f8_ea[l + 1] = fp8_exponent(v);
  }
  std::vector<uint8_t> U = pack_map_fp8<S>(pd, c->f8_ew, c->f8_ea);
  // biases of layer l times 2^ea[l+1] (the layer's output scale), density head
  // weights over the last trunk layer's factor
  PackedB P = pack_map_bf16<NerfMapB>(pd);
  for (int l = 0; l < S::NL; ++l)
    for (long i = NerfMapB::bias_base(l); i < NerfMapB::bias_base(l) + 32L * NerfMapB::layer_mt(l); ++i)
      P.bias[i] = std::ldexp(P.bias[i], c->f8_ea[l + 1]);
  std::vector<float> H = pack_heads_fp8<S>(pd, c->f8_ea[S::D]);
  e = hipMemcpyAsync(c->wunits, U.data(), U.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->bias_b, P.bias.data(), P.bias.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->heads_f8, H.data(), H.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, LOC_E_HIP, "FP8 weight upload: %s", hipGetErrorString(e));
  c->f8_ready = true;
  return LOC_OK;
}

loc_status loc_fp8_scales(loc_ctx* c, int* ew, int* ea, float* amax, int n) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (c->desc.precision != LOC_FP8_E4M3) return fail(c, LOC_E_STATE, "context precision is not FP8");
  if (!c->f8_ready) return fail(c, LOC_E_STATE, "no calibration has run");
  if (n < NerfMapF8::NL) return fail(c, LOC_E_ARG, "n must be at least %d", NerfMapF8::NL);
  for (int l = 0; l < NerfMapF8::NL; ++l) {
    if (ew) ew[l] = c->f8_ew[l];
    if (ea) ea[l] = c->f8_ea[l];
    if (amax) amax[l] = c->f8_amax[l];
  }
  return LOC_OK;
}


// ------------------------------------------------------------- coarse-to-fine

}  // extern "C"

namespace {

// default tile choice: one 32-sample tile per wave, 8 waves, two workgroups per CU
void level_default_cfg(const loc_ctx* c, long n_rays, int& ntl, int& waves, int& blocks) {
  ntl = 2;
  waves = 4;
  const long batches = (n_rays + 7) / 8;   // rays set up per wave at once
  blocks = (int)std::max(1L, std::min((batches + waves - 1) / waves, 2L * c->n_cu));
}

void level_cfg(const loc_ctx* c, int L, int& ntl, int& waves, int& blocks) {
  const auto& lv = c->lv[L];
  if (lv.ntl > 0) { ntl = lv.ntl; waves = lv.waves; blocks = lv.blocks; return; }
  level_default_cfg(c, (long)lv.N * lv.B, ntl, waves, blocks);
}

struct LevelCall {
  const float* image;
  loc_camera cam;
  int n_levels;
  loc_level levels[8];
  int N;
  const double* pose_in;
  int reject;
  double* pose_out;
  double* est_out;
};

LevelRayArgs level_ray_args(const loc_ctx* c, const LevelCall& q, int L) {
  const loc_map_desc& d = c->desc;
  const int s = q.levels[L].inv_R;
  LevelRayArgs a{};
  a.key = c->key;
  a.level = L;
  a.pose = c->lv[L].pose.p;
  a.image = q.image;
  a.W_full = q.cam.W;
  a.s = s;
  a.Wl = q.cam.W / s;
  a.Hl = q.cam.H / s;
  a.fx = q.cam.fx / s;
  a.fy = q.cam.fy / s;
  a.cx = q.cam.cx / s;
  a.cy = q.cam.cy / s;
  a.N = c->lv[L].N;
  a.B = c->lv[L].B;
  a.wblocks = c->wblocks;
  a.bias = c->bias_b;
  a.heads = c->heads_b;
  a.near_ = d.near_;
  a.dt = (d.far_ - d.near_) / (float)d.n_coarse;
  a.far_ = d.far_;
  a.log_trans = (float)std::log1p(-(double)d.alpha);
  a.log_opq = (float)std::log((double)d.alpha);
  a.tau = d.tau;
  a.empty_F = c->empty_span ? d.far_ - d.near_ : d.tau;
  a.jitter = d.jitter;
  a.ray_rgba = c->lv[L].rgba.p;
  a.ray_fe = c->lv[L].fe.p;
  return a;
}

// the level sequence on stream st; with `prof`, every launch is timed.  The
// first kernel writes the call's key kv (by value) for the later kernels and
// predicts the first level from it; a captured graph gets each later call's
// key on that node (set_level_begin_node)
// where the begin kernel puts the later levels' motion increments
LevelIncs level_incs(const loc_ctx* c, const LevelCall& q) {
  LevelIncs incs{};
  for (int L = 0; L + 1 < q.n_levels; ++L) {
    incs.inc[L] = c->lv[L].inc.p;
    incs.n[L] = c->lv[L].n_out;
  }
  return incs;
}

loc_status enqueue_levels(loc_ctx* c, const LevelCall& q, hipStream_t st, bool prof, const LevelKey& kv) {
  auto run = [&](int kid, double flop, double bytes, auto fn) -> loc_status {
    if (prof) return timed(c, kid, flop, bytes, fn);
    hipError_t e = fn();
    return e == hipSuccess ? LOC_OK : fail(c, LOC_E_HIP, "launch of %s failed: %s", kKernelNames[kid], hipGetErrorString(e));
  };
  loc_status s;
  const LevelIncs incs = level_incs(c, q);
  if ((s = run(K_LV_PREDICT, 0, 192.0 * q.N,
               [&] { return launch_level_begin(c->key, kv, q.pose_in, c->lv[0].pose.p, q.N, incs, st); })))
    return s;
  for (int L = 0; L < q.n_levels; ++L) {
    auto& lv = c->lv[L];
    const LevelRayArgs ra = level_ray_args(c, q, L);
    int ntl, waves, blocks;
    level_cfg(c, L, ntl, waves, blocks);
    const double nr = (double)lv.N * lv.B;
    if ((s = run(K_LV_RAYS, 2.0 * (double)c->macs * nr * 32, nr * (24.0 + 12.0 * ra.s * ra.s), [&] {
           return launch_level_rays(ra, ntl, waves, blocks, st);
         })))
      return s;
    LevelFinishArgs fa{};
    fa.key = c->key;
    fa.level = L;
    fa.ray_fe = lv.fe.p;
    fa.N = lv.N;
    fa.B = lv.B;
    fa.reject = q.reject;
    fa.pose = lv.pose.p;
    fa.loglik = lv.loglik.p;
    fa.uncert = lv.uncert.p;
    fa.weight = lv.weight.p;
    fa.idx = lv.idx.p;
    fa.prefix = c->prefix.p;
    fa.n_out = lv.n_out;
    const bool last = L + 1 == q.n_levels;
    fa.next_pose = last ? q.pose_out : c->lv[L + 1].pose.p;
    fa.predict_next = last ? 0 : 1;
    fa.inc = lv.inc.p;
    fa.est = last ? q.est_out : nullptr;
    fa.flags = c->flags;
    if ((s = run(K_LV_SCORES, 0, nr * 8.0 + lv.N * 20.0, [&] { return launch_level_scores(fa, st); }))) return s;
    if ((s = run(K_LV_FINISH, 0, lv.N * 120.0 + lv.n_out * 100.0, [&] { return launch_level_finish(fa, st); })))
      return s;
  }
  return LOC_OK;
}

std::vector<double> level_signature(const loc_ctx* c, const LevelCall& q) {
  std::vector<double> v = {(double)(uintptr_t)q.image, (double)q.cam.W, (double)q.cam.H, q.cam.fx, q.cam.fy,
                           q.cam.cx, q.cam.cy, (double)q.n_levels, (double)q.N, (double)(uintptr_t)q.pose_in,
                           (double)q.reject, (double)(uintptr_t)q.pose_out, (double)(uintptr_t)q.est_out};
  for (int L = 0; L < q.n_levels; ++L) {
    int ntl, waves, blocks;
    level_cfg(c, L, ntl, waves, blocks);
    for (double x : {(double)q.levels[L].inv_R, (double)q.levels[L].B, (double)q.levels[L].n_out, (double)ntl,
                     (double)waves, (double)blocks, (double)(uintptr_t)c->lv[L].pose.p,
                     (double)(uintptr_t)c->lv[L].inc.p})
      v.push_back(x);
  }
  return v;
}

void drop_graph(loc_ctx* c) {
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->graph) hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->begin_node = nullptr;
  c->graph_sig.clear();
}

// argument checks and workspace of a level call; fills q
loc_status prepare_levels(loc_ctx* c, const float* image, const loc_camera* cam, int n_levels,
                          const loc_level* levels, int N, const double* pose_in, int reject, double* pose_out,
                          double* est_out, LevelCall& q) {
  if (!image || !cam || !levels || !pose_in || !pose_out) return fail(c, LOC_E_ARG, "null pointer argument");
  const loc_map_desc& d = c->desc;
  if (c->kind != kMapSmall || d.precision != LOC_BF16 || d.n_coarse != 32 || d.n_fine != 0)
    return fail(c, LOC_E_UNSUPPORTED, "the level path needs the 4x64 map in BF16 with 32 coarse and 0 fine samples");
  if (n_levels < 1 || n_levels > 8) return fail(c, LOC_E_ARG, "n_levels must be in [1, 8]");
  if (N < 1 || N > (1 << 20)) return fail(c, LOC_E_ARG, "N must be in [1, 2^20]");
  if (!(cam->fx > 0 && cam->fy > 0) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy) || cam->W <= 0 ||
      cam->H <= 0)
    return fail(c, LOC_E_ARG, "invalid camera");
  q.image = image;
  q.cam = *cam;
  q.n_levels = n_levels;
  q.N = N;
  q.pose_in = pose_in;
  q.reject = reject ? 1 : 0;
  q.pose_out = pose_out;
  q.est_out = est_out;
  int n_in = N;
  size_t max_n = 0;
  for (int L = 0; L < n_levels; ++L) {
    const loc_level& v = levels[L];
    if (v.inv_R != 1 && v.inv_R != 2 && v.inv_R != 4 && v.inv_R != 8)
      return fail(c, LOC_E_ARG, "level %d: inv_R must be 1, 2, 4 or 8", L);
    if (cam->W % v.inv_R || cam->H % v.inv_R) return fail(c, LOC_E_ARG, "level %d: image not divisible", L);
    if (v.B < 1 || v.B > 1024) return fail(c, LOC_E_ARG, "level %d: B must be in [1, 1024]", L);
    if (v.n_out < 1 || v.n_out > (1 << 20)) return fail(c, LOC_E_ARG, "level %d: n_out must be in [1, 2^20]", L);
    if ((long)n_in * v.B > (1L << 26)) return fail(c, LOC_E_ARG, "level %d: too many rays", L);
    q.levels[L] = v;
    auto& lv = c->lv[L];
    loc_status s;
    if ((s = ensure(c, lv.pose, (size_t)n_in * 12)) || (s = ensure(c, lv.loglik, n_in)) ||
        (s = ensure(c, lv.weight, n_in)) || (s = ensure(c, lv.uncert, n_in)) || (s = ensure(c, lv.idx, v.n_out)) ||
        (s = ensure(c, lv.rgba, (size_t)n_in * v.B)) || (s = ensure(c, lv.fe, (size_t)n_in * v.B)) ||
        (s = ensure(c, lv.inc, (size_t)v.n_out * 12)))
      return s;
    if (lv.N != n_in || lv.B != v.B || lv.n_out != v.n_out) lv.ntl = lv.waves = lv.blocks = 0;   // retune
    lv.N = n_in;
    lv.B = v.B;
    lv.n_out = v.n_out;
    max_n = std::max(max_n, (size_t)n_in);
    n_in = v.n_out;
  }
  c->n_lv = n_levels;
  loc_status s;
  if ((s = ensure(c, c->prefix, max_n))) return s;
  if (!c->key && hipMalloc(&c->key, sizeof(LevelKey)) != hipSuccess) {
    (void)hipGetLastError();
    c->key = nullptr;
    return fail(c, LOC_E_OOM, "level key");
  }
  if (!c->n_cu) {
    hipDeviceProp_t prop;
    HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
    c->n_cu = prop.multiProcessorCount;
  }
  return LOC_OK;
}

loc_status make_key(loc_ctx* c, const double* motion, double sigma_t, double sigma_r, uint64_t seed, uint64_t iter,
                    LevelKey& kv) {
  if (!(sigma_t >= 0.0) || !(sigma_r >= 0.0)) return fail(c, LOC_E_ARG, "negative noise scale");
  kv = LevelKey{};
  kv.seed = seed;
  kv.iter = iter;
  for (int qd = 0; qd < 12; ++qd) kv.motion[qd] = motion ? motion[qd] : ((qd % 5 == 0) ? 1.0 : 0.0);
  kv.sigma_t = sigma_t;
  kv.sigma_r = sigma_r;
  return LOC_OK;
}

}  // namespace

extern "C" {

loc_status loc_update_levels(loc_ctx* c, const float* image, const loc_camera* cam, int n_levels,
                             const loc_level* levels, int N, const double* pose_in, const double* motion,
                             double sigma_t, double sigma_r, uint64_t seed, uint64_t iter, int reject,
                             double* pose_out, double* est_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  LevelCall q{};
  loc_status s;
  if ((s = prepare_levels(c, image, cam, n_levels, levels, N, pose_in, reject, pose_out, est_out, q))) return s;
  {
    hipError_t pe = hipGetLastError();
    if (pe != hipSuccess) return fail(c, LOC_E_HIP, "pending HIP error: %s", hipGetErrorString(pe));
  }
  LevelKey kv;
  if ((s = make_key(c, motion, sigma_t, sigma_r, seed, iter, kv))) return s;
  if (!c->graph_mode) return enqueue_levels(c, q, c->stream, c->prof != 0, kv);
  // graph mode: the same launches captured once per signature; each replay
  // first hands this call's key to the graph's k_level_begin node
  std::vector<double> sig = level_signature(c, q);
  if (!c->gexec || sig != c->graph_sig) {
    drop_graph(c);
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    loc_status cs = enqueue_levels(c, q, c->cap_stream, false, kv);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (cs) { if (g) hipGraphDestroy(g); return cs; }
    if (e != hipSuccess) return fail(c, LOC_E_HIP, "graph capture: %s", hipGetErrorString(e));
    c->graph = g;
    size_t n_roots = 0;
    e = hipGraphGetRootNodes(c->graph, nullptr, &n_roots);
    if (e == hipSuccess && n_roots == 1) e = hipGraphGetRootNodes(c->graph, &c->begin_node, &n_roots);
    if (e != hipSuccess || n_roots != 1) {
      drop_graph(c);
      return fail(c, LOC_E_HIP, "graph capture: expected one root node, found %zu", n_roots);
    }
    e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_graph(c); return fail(c, LOC_E_HIP, "graph instantiate: %s", hipGetErrorString(e)); }
    c->graph_sig = sig;
  } else {
    hipError_t e = set_level_begin_node(c->gexec, c->begin_node, c->key, kv, q.pose_in, c->lv[0].pose.p, q.N,
                                        level_incs(c, q));
    if (e != hipSuccess) return fail(c, LOC_E_HIP, "graph key update: %s", hipGetErrorString(e));
  }
  HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
  return LOC_OK;
}

loc_status loc_set_empty_ray_uncertainty(loc_ctx* c, int mode) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (mode != 0 && mode != 1) return fail(c, LOC_E_ARG, "mode must be 0 (F = tau) or 1 (F = far - near)");
  if (mode != c->empty_span) drop_graph(c);    // a captured level graph holds the old value
  c->empty_span = mode;
  return LOC_OK;
}

loc_status loc_set_graph_mode(loc_ctx* c, int enable) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  c->graph_mode = enable != 0;
  if (!c->graph_mode) drop_graph(c);
  return LOC_OK;
}

loc_status loc_level_outputs(loc_ctx* c, int level, double* loglik, double* weight, float* uncert, int32_t* idx,
                             double* pose) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (level < 0 || level >= c->n_lv) return fail(c, LOC_E_STATE, "no level %d in the last level call", level);
  const auto& L = c->lv[level];
  if (loglik) HIP_TRY(c, hipMemcpyAsync(loglik, L.loglik.p, 8 * (size_t)L.N, hipMemcpyDeviceToDevice, c->stream));
  if (weight) HIP_TRY(c, hipMemcpyAsync(weight, L.weight.p, 8 * (size_t)L.N, hipMemcpyDeviceToDevice, c->stream));
  if (uncert) HIP_TRY(c, hipMemcpyAsync(uncert, L.uncert.p, 4 * (size_t)L.N, hipMemcpyDeviceToDevice, c->stream));
  if (idx) HIP_TRY(c, hipMemcpyAsync(idx, L.idx.p, 4 * (size_t)L.n_out, hipMemcpyDeviceToDevice, c->stream));
  if (pose) HIP_TRY(c, hipMemcpyAsync(pose, L.pose.p, 96 * (size_t)L.N, hipMemcpyDeviceToDevice, c->stream));
  return LOC_OK;
}

loc_status loc_level_ray_outputs(loc_ctx* c, int level, float* rgb, float* opacity, float* F, float* E) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (level < 0 || level >= c->n_lv) return fail(c, LOC_E_STATE, "no level %d in the last level call", level);
  const auto& L = c->lv[level];
  const int n = L.N * L.B;
  return timed(c, K_SPLIT, 0, 24.0 * n, [&] {
    return launch_split_ray_outputs(L.rgba.p, L.fe.p, n, rgb, opacity, F, E, c->stream);
  });
}


// Autotuner of the fused ray kernel: for every level of the given call, each
// tile configuration (column tiles per wave x waves per workgroup) and grid
// size (1, 2, 4 or 8 workgroups per CU, capped by the work) is timed over
// `reps` launches after one warm-up on the level's real particles (an update
// runs first to produce them), and the fastest is kept for the level.  With a
// cache file, a level whose key (arch, map, N, B, scale) is already recorded
// takes the recorded choice without timing, and new choices are appended as
// one JSON object per line.
loc_status loc_autotune_levels(loc_ctx* c, const float* image, const loc_camera* cam, int n_levels,
                               const loc_level* levels, int N, const double* pose_in, int reps,
                               const char* cache_path, int* chosen) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (reps < 1 || reps > 1000) return fail(c, LOC_E_ARG, "reps must be in [1, 1000]");
  const bool gm = c->graph_mode;
  c->graph_mode = false;
  drop_graph(c);
  if (!levels || n_levels < 1 || n_levels > 8) {
    c->graph_mode = gm;
    return fail(c, LOC_E_ARG, "levels: NULL or n_levels outside [1, 8]");
  }
  const int n_last = levels[n_levels - 1].n_out;
  if (n_last < 1 || n_last > (1 << 20)) {
    c->graph_mode = gm;
    return fail(c, LOC_E_ARG, "last level: n_out must be in [1, 2^20]");
  }
  double* pose_out = nullptr;
  double* est = nullptr;
  if (hipMalloc(&pose_out, (size_t)n_last * 96) != hipSuccess || hipMalloc(&est, 96) != hipSuccess) {
    (void)hipGetLastError();
    hipFree(pose_out);
    c->graph_mode = gm;
    return fail(c, LOC_E_OOM, "autotune buffers");
  }
  LevelCall q{};
  loc_status s = prepare_levels(c, image, cam, n_levels, levels, N, pose_in, 1, pose_out, est, q);
  if (s) {
    hipFree(pose_out);
    hipFree(est);
    c->graph_mode = gm;
    return s;
  }
  for (int L = 0; L < n_levels; ++L) c->lv[L].ntl = c->lv[L].waves = c->lv[L].blocks = 0;
  const int prof = c->prof;
  c->prof = 0;
  LevelKey kv;
  s = make_key(c, nullptr, 0.0, 0.0, 12345, 0, kv);
  if (!s) s = enqueue_levels(c, q, c->stream, false, kv);
  // cached choices
  std::vector<std::string> cache_lines;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof line, f)) cache_lines.push_back(line);
      std::fclose(f);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!s && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    s = fail(c, LOC_E_HIP, "event creation failed");
  static const int kCand[3][2] = {{2, 2}, {2, 4}, {2, 8}};
  for (int L = 0; !s && L < n_levels; ++L) {
    auto& lv = c->lv[L];
    char key[160];
    std::snprintf(key, sizeof key, "gfx950/small-bf16-32/N%d/B%d/s%d", lv.N, lv.B, q.levels[L].inv_R);
    bool found = false;
    for (const auto& ln : cache_lines) {
      char k2[160];
      int ntl, waves, blocks;
      if (std::sscanf(ln.c_str(), "{\"key\": \"%159[^\"]\", \"ntl\": %d, \"waves\": %d, \"blocks\": %d", k2, &ntl,
                      &waves, &blocks) == 4 &&
          std::strcmp(k2, key) == 0 && level_rays_config_ok(ntl, waves) && blocks >= 1) {
        lv.ntl = ntl; lv.waves = waves; lv.blocks = blocks;
        found = true;
      }
    }
    if (found) continue;
    const LevelRayArgs ra = level_ray_args(c, q, L);
    const long n_rays = (long)lv.N * lv.B;
    float best = 1e30f;
    int bn = 1, bw = 8, bb = 1;
    for (const auto& cd : kCand) {
      const long tiles = ((n_rays + 7) / 8 + cd[1] - 1) / cd[1];   // workgroups with work
      int last_blocks = -1;
      for (int mult : {1, 2, 4, 8}) {
        const int blocks = (int)std::max(1L, std::min(tiles, (long)mult * c->n_cu));
        if (blocks == last_blocks) continue;
        last_blocks = blocks;
        hipError_t e = launch_level_rays(ra, cd[0], cd[1], blocks, c->stream);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; e == hipSuccess && r < reps; ++r) e = launch_level_rays(ra, cd[0], cd[1], blocks, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { s = fail(c, LOC_E_HIP, "autotune launch: %s", hipGetErrorString(e)); break; }
        if (ms < best) { best = ms; bn = cd[0]; bw = cd[1]; bb = blocks; }
      }
      if (s) break;
    }
    if (s) break;
    lv.ntl = bn; lv.waves = bw; lv.blocks = bb;
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "{\"key\": \"%s\", \"ntl\": %d, \"waves\": %d, \"blocks\": %d, \"us_per_launch\": %.3f}\n", key,
                     bn, bw, bb, 1000.0 * best / reps);
        std::fclose(f);
      }
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(c->stream);
  hipFree(pose_out);
  hipFree(est);
  c->prof = prof;
  c->graph_mode = gm;
  if (s) return s;
  if (chosen)
    for (int L = 0; L < n_levels; ++L) {
      chosen[3 * L] = c->lv[L].ntl;
      chosen[3 * L + 1] = c->lv[L].waves;
      chosen[3 * L + 2] = c->lv[L].blocks;
    }
  return LOC_OK;
}

loc_status loc_set_level_tiles(loc_ctx* c, int level, int ntl, int waves, int blocks) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (level < 0 || level >= 8) return fail(c, LOC_E_ARG, "level out of range");
  if (!(ntl == 0 && waves == 0 && blocks == 0) && (!level_rays_config_ok(ntl, waves) || blocks < 1))
    return fail(c, LOC_E_ARG, "unsupported tile configuration");
  c->lv[level].ntl = ntl;
  c->lv[level].waves = waves;
  c->lv[level].blocks = blocks;
  return LOC_OK;
}


loc_status loc_position_variance(loc_ctx* c, const double* pose, const double* weight, int N, double* var) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!pose || !weight || !var) return fail(c, LOC_E_ARG, "null pointer argument");
  if (N < 1 || N > (1 << 24)) return fail(c, LOC_E_ARG, "N must be in [1, 2^24]");
  return timed(c, K_VARIANCE, 0, 2.0 * 32.0 * N, [&] { return launch_position_variance(pose, weight, N, var, c->stream); });
}

loc_status loc_render_image(loc_ctx* c, const loc_camera* cam, int inv_R, const double* pose, uint64_t seed,
                            uint64_t iter, float* rgb, float* opacity) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!cam || !pose || !rgb) return fail(c, LOC_E_ARG, "null pointer argument");
  if (inv_R != 1 && inv_R != 2 && inv_R != 4 && inv_R != 8) return fail(c, LOC_E_ARG, "inv_R must be 1, 2, 4 or 8");
  if (cam->W <= 0 || cam->H <= 0 || cam->W % inv_R || cam->H % inv_R || !(cam->fx > 0 && cam->fy > 0) ||
      !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(c, LOC_E_ARG, "invalid camera for level factor %d", inv_R);
  if (c->fine_mode == 1 && !c->prop) return fail(c, LOC_E_STATE, "proposal mode without proposal parameters");
  if (c->desc.precision == LOC_FP8_E4M3 && !c->f8_ready)
    return fail(c, LOC_E_STATE, "FP8 map used before loc_calibrate_fp8");
  const int Wl = cam->W / inv_R, Hl = cam->H / inv_R;
  const long n = (long)Wl * Hl;
  if (n > (1L << 30) / 256) return fail(c, LOC_E_ARG, "image of %ld pixels exceeds 2^22", n);
  const loc_map_desc& d = c->desc;
  const int Sc = d.n_coarse, Sf = d.n_fine;
  loc_status s;
  if ((s = ensure(c, c->ray_o, n)) || (s = ensure(c, c->ray_d, n)) || (s = ensure(c, c->rgba, n)) ||
      (s = ensure(c, c->fe, n)) || (s = ensure(c, c->t_c, n * Sc)) || (s = ensure(c, c->out_c, n * Sc)))
    return s;
  if (Sf > 0 && ((s = ensure(c, c->t_f, n * Sf)) || (s = ensure(c, c->out_f, n * Sf)))) return s;
  RaygenArgs ra{};
  ra.pose = pose;
  ra.image = nullptr;
  ra.W_full = cam->W;
  ra.s = inv_R;
  ra.Wl = Wl;
  ra.Hl = Hl;
  ra.fx = cam->fx / inv_R;
  ra.fy = cam->fy / inv_R;
  ra.cx = cam->cx / inv_R;
  ra.cy = cam->cy / inv_R;
  ra.N = 1;
  ra.B = (int)n;
  ra.seed = seed;
  ra.iter = iter;
  ra.ray_o = c->ray_o.p;
  ra.ray_d = c->ray_d.p;
  ra.obs = nullptr;
  ra.all_pixels = 1;
  if ((s = timed(c, K_RAYGEN, 0, 32.0 * n + 96.0, [&] { return launch_raygen(ra, c->stream); }))) return s;
  if ((s = map_samples(c, n, (int)n, seed, iter))) return s;
  CompositeArgs ca{};
  ca.t_coarse = c->t_c.p;
  ca.out_coarse = c->out_c.p;
  ca.t_fine = Sf > 0 ? c->t_f.p : nullptr;
  ca.out_fine = Sf > 0 ? c->out_f.p : nullptr;
  ca.obs = nullptr;
  ca.N = (int)((n + 3) / 4);     // no scores: particle grouping is immaterial
  ca.B = 4;
  ca.Sc = Sc;
  ca.Sf = Sf;
  ca.far_ = d.far_;
  ca.log_trans = (float)std::log1p(-(double)d.alpha);
  ca.log_opq = (float)std::log((double)d.alpha);
  ca.tau = d.tau;
  ca.empty_F = c->empty_span ? d.far_ - d.near_ : d.tau;
  ca.ray_rgba = c->rgba.p;
  ca.ray_fe = c->fe.p;
  ca.loglik = nullptr;
  ca.uncert = nullptr;
  ca.hist = nullptr;
  ca.n_rays = (int)n;
  ca.near_ = d.near_;
  if ((s = timed(c, K_COMPOSITE, 0, n * (20.0 * (Sc + Sf) + 24.0), [&] { return launch_composite(ca, c->stream); })))
    return s;
  return timed(c, K_SPLIT, 0, 28.0 * n, [&] {
    return launch_split_ray_outputs(c->rgba.p, c->fe.p, (int)n, rgb, opacity, nullptr, nullptr, c->stream);
  });
}

loc_status loc_localize(loc_ctx* c, const float* image, const loc_camera* cam, int n_stages, const loc_stage* stages,
                        int n_iters, int n_in, const double* pose_in, const double* motion, double sigma_t,
                        double sigma_r, uint64_t seed, uint64_t iter, double* pose_out, int* n_out,
                        loc_step_info* info, int* n_done, const loc_trace* trace) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!image || !cam || !stages || !pose_in || !pose_out || !n_out) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n_stages < 1 || n_stages > 8) return fail(c, LOC_E_ARG, "n_stages must be in [1, 8]");
  if (n_iters < 1) return fail(c, LOC_E_ARG, "n_iters must be >= 1");
  int n_max = n_in;
  for (int k = 0; k < n_stages; ++k) {
    const loc_stage& g = stages[k];
    if (g.inv_R != 1 && g.inv_R != 2 && g.inv_R != 4 && g.inv_R != 8)
      return fail(c, LOC_E_ARG, "stage %d: inv_R must be 1, 2, 4 or 8", k);
    if (g.B < 1 || g.B > 1024 || g.N < 1 || g.N >= (1 << 24))
      return fail(c, LOC_E_ARG, "stage %d: B or N out of range", k);
    if (k + 1 < n_stages && std::isnan(g.delta)) return fail(c, LOC_E_ARG, "stage %d: delta is NaN", k);
    if (!(g.noise >= 0.0) || !std::isfinite(g.noise)) return fail(c, LOC_E_ARG, "stage %d: noise factor", k);
    n_max = std::max(n_max, g.N);
  }
  if (n_in < 1 || n_in >= (1 << 24)) return fail(c, LOC_E_ARG, "n_in must be in [1, 2^24 - 1]");
  if (trace && trace->capacity > 0 && (!trace->pose || !trace->weight || !trace->idx))
    return fail(c, LOC_E_ARG, "trace buffers missing");
  loc_status s;
  if ((s = ensure(c, c->lz_x[0], 12L * n_max)) || (s = ensure(c, c->lz_x[1], 12L * n_max)) ||
      (s = ensure(c, c->lz_pred, 12L * n_max)) || (s = ensure(c, c->lz_ll, n_max)) ||
      (s = ensure(c, c->lz_w, n_max)) || (s = ensure(c, c->lz_ve, 13)) || (s = ensure(c, c->lz_idx, n_max)))
    return s;
  if (!c->lz_host && hipHostMalloc((void**)&c->lz_host, 13 * sizeof(double), 0) != hipSuccess) {
    (void)hipGetLastError();
    c->lz_host = nullptr;
    return fail(c, LOC_E_OOM, "pinned host allocation failed");
  }
  HIP_TRY(c, hipMemcpyAsync(c->lz_x[0].p, pose_in, 96L * n_in, hipMemcpyDeviceToDevice, c->stream));
  int cur = 0, n = n_in, st = 0, done = 0;
  bool lost = false;
  long toff = 0, ioff = 0;
  for (int t = 0; t < n_iters; ++t) {
    const auto t0 = std::chrono::steady_clock::now();
    const loc_stage& g = stages[st];
    const uint64_t it = iter + (uint64_t)t;
    if ((s = loc_update_particles(c, image, cam, g.inv_R, g.B, n, c->lz_x[cur].p, motion, g.noise * sigma_t,
                                  g.noise * sigma_r, seed, it, c->lz_pred.p, c->lz_ll.p, c->lz_w.p, nullptr)))
      return s;
    if ((s = loc_position_variance(c, c->lz_pred.p, c->lz_w.p, n, c->lz_ve.p)) ||
        (s = loc_pose_estimate(c, c->lz_pred.p, c->lz_w.p, n, c->lz_ve.p + 1)))
      return s;
    HIP_TRY(c, hipMemcpyAsync(c->lz_host, c->lz_ve.p, 13 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double var = c->lz_host[0];
    const int st_w = st;
    if (st + 1 < n_stages && var < stages[st].delta) ++st;   // NaN never switches
    const int n_next = std::isnan(var) ? 0 : stages[st].N;
    if (n_next > 0) {
      if ((s = loc_resample(c, c->lz_w.p, n, n_next, seed, it, c->lz_idx.p)) ||
          (s = loc_gather_poses(c, c->lz_pred.p, n, c->lz_idx.p, n_next, c->lz_x[cur ^ 1].p)))
        return s;
    }
    if (trace && trace->capacity > 0) {
      if (toff + n > trace->capacity || ioff + n_next > trace->capacity)
        return fail(c, LOC_E_ARG, "trace capacity %ld exceeded at iteration %d", trace->capacity, t);
      HIP_TRY(c, hipMemcpyAsync(trace->pose + 12 * toff, c->lz_pred.p, 96L * n, hipMemcpyDeviceToDevice, c->stream));
      HIP_TRY(c, hipMemcpyAsync(trace->weight + toff, c->lz_w.p, 8L * n, hipMemcpyDeviceToDevice, c->stream));
      if (n_next > 0)
        HIP_TRY(c, hipMemcpyAsync(trace->idx + ioff, c->lz_idx.p, 4L * n_next, hipMemcpyDeviceToDevice, c->stream));
      toff += n;
      ioff += n_next;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (info) {
      loc_step_info& r = info[t];
      r.iter = (long long)it;
      r.stage = st_w;
      r.n = n;
      r.n_next = n_next;
      r.var = var;
      for (int q = 0; q < 12; ++q) r.est[q] = c->lz_host[1 + q];
      r.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    ++done;
    if (n_next == 0) {
      lost = true;
      break;
    }
    cur ^= 1;
    n = n_next;
  }
  if (n_done) *n_done = done;
  if (lost) {
    *n_out = 0;
    return LOC_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(pose_out, c->lz_x[cur].p, 96L * n, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *n_out = n;
  return LOC_OK;
}

}  // extern "C"

// ------------------------------------------------------------- map training
namespace {

constexpr int kMapWavesMax = 1024;   // partial-gradient rows per call, at most
constexpr int kMapWavesBf16 = 1024;  // the same for the bf16 kernel (four waves per CU)

loc_status tm_prepare(loc_ctx* c, const float* ray_o, const float* ray_d, int n, int batch, MapTrainArgs& ta) {
  const loc_map_desc& d = c->desc;
  if (c->kind != kMapSmall || d.n_fine != 0 || d.n_coarse > 64 || c->desc.precision == LOC_FP8_E4M3)
    return fail(c, LOC_E_UNSUPPORTED, "map training covers the 4x64 map with at most 64 coarse and no fine samples");
  // bf16 contexts with 32 samples per ray take the matrix-core kernel: one
  // ray at a time per wave, sized to fill 1024 waves (four per CU) once
  const bool bf16 = d.precision == LOC_BF16 && d.n_coarse == 32;
  const int rpw = bf16 ? (batch + kMapWavesBf16 - 1) / kMapWavesBf16 : (batch + kMapWavesMax - 1) / kMapWavesMax;
  const int n_waves = (batch + rpw - 1) / rpw;
  loc_status s;
  if ((s = ensure(c, c->tr_o, n)) || (s = ensure(c, c->tr_d, n)) || (s = ensure(c, c->tm_params, kSmallMapParams)) ||
      (s = ensure(c, c->tm_m, kSmallMapParams)) || (s = ensure(c, c->tm_v, kSmallMapParams)) ||
      (s = ensure(c, c->tm_partial, (size_t)n_waves * kSmallMapParams)) || (s = ensure(c, c->tm_lpart, n_waves)))
    return s;
  if (!c->tm_ready) {
    if (c->params_host.size() != (size_t)kSmallMapParams) return fail(c, LOC_E_STATE, "map parameters missing");
    HIP_TRY(c, hipMemcpyAsync(c->tm_params.p, c->params_host.data(), 4L * kSmallMapParams, hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipMemsetAsync(c->tm_m.p, 0, 4L * kSmallMapParams, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->tm_v.p, 0, 4L * kSmallMapParams, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->tm_step = 0;
    c->tm_ready = true;
  }
  if ((s = timed(c, K_RAYS, 0, 56.0 * n,
                 [&] { return launch_rays_to_f4(ray_o, ray_d, n, c->tr_o.p, c->tr_d.p, c->stream); })))
    return s;
  ta = MapTrainArgs{};
  ta.ray_o = c->tr_o.p;
  ta.ray_d = c->tr_d.p;
  ta.params = c->tm_params.p;
  ta.partial = c->tm_partial.p;
  ta.loss_partial = c->tm_lpart.p;
  ta.n_rays = n;
  ta.batch = batch;
  ta.rays_per_wave = rpw;
  ta.n_waves = n_waves;
  ta.S = d.n_coarse;
  ta.jitter = d.jitter;
  ta.bf16 = bf16 ? 1 : 0;
  ta.near_ = d.near_;
  ta.far_ = d.far_;
  ta.dt = (d.far_ - d.near_) / (float)d.n_coarse;
  return LOC_OK;
}

// the map packed again for the context's precision from params_host
loc_status tm_repack(loc_ctx* c) {
  loc_map_desc d = c->desc;
  d.params = c->params_host.data();
  d.n_params = c->params_host.size();
  if (d.precision == LOC_FP32) {
    std::vector<float> P = pack_map<SmallMap>(d);
    HIP_TRY(c, hipMemcpyAsync(c->weights, P.data(), 4 * P.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  } else {
    PackedB P = pack_map_bf16<SmallMapB>(d);
    HIP_TRY(c, hipMemcpyAsync(c->wblocks, P.blocks.data(), P.blocks.size() * 2, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->bias_b, P.bias.data(), P.bias.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->heads_b, P.heads.data(), P.heads.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  drop_graph(c);
  return LOC_OK;
}

}  // namespace

extern "C" {

loc_status loc_map_grad(loc_ctx* c, const float* ray_o, const float* ray_d, const float* target, int n, uint64_t seed,
                        uint64_t iter, float* grad_out, float* loss_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!ray_o || !ray_d || !target || !grad_out) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n < 1 || n > (1 << 20)) return fail(c, LOC_E_ARG, "n must be in [1, 2^20]");
  MapTrainArgs ta;
  loc_status s;
  if ((s = tm_prepare(c, ray_o, ray_d, n, n, ta))) return s;
  ta.target = target;
  ta.first = 0;
  ta.seed = seed;
  ta.iter = iter;
  ta.loss_out = loss_out;
  ta.loss_index = 0;
  ta.grad_out = grad_out;
  ta.adam = 0;
  return timed(c, K_MAP_TRAIN, 2.0 * 4.0 * SmallMap::macs() * n * ta.S, 0.0,
               [&] { return launch_map_grad(ta, c->stream); });
}

loc_status loc_train_map(loc_ctx* c, const float* ray_o, const float* ray_d, const float* target, int n,
                         const loc_train_cfg* cfg, uint64_t seed, float* loss_out) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!ray_o || !ray_d || !target || !cfg) return fail(c, LOC_E_ARG, "null pointer argument");
  if (n < 1 || n > (1 << 24)) return fail(c, LOC_E_ARG, "n out of range");
  if (cfg->batch < 1 || cfg->batch > (1 << 20) || cfg->steps < 0) return fail(c, LOC_E_ARG, "batch or steps out of range");
  if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f))
    return fail(c, LOC_E_ARG, "invalid Adam hyperparameters");
  MapTrainArgs ta;
  loc_status s;
  if ((s = tm_prepare(c, ray_o, ray_d, n, cfg->batch, ta))) return s;
  ta.target = target;
  ta.params_rw = c->tm_params.p;
  ta.m = c->tm_m.p;
  ta.v = c->tm_v.p;
  ta.loss_out = loss_out;
  ta.adam = 1;
  ta.lr = cfg->lr;
  ta.beta1 = cfg->beta1;
  ta.beta2 = cfg->beta2;
  ta.eps = cfg->eps;
  ta.seed = seed;
  for (int k = 0; k < cfg->steps; ++k) {
    ta.first = (int)(((long)k * cfg->batch) % n);
    ta.loss_index = k;
    ta.iter = (uint64_t)c->tm_step;
    ta.step = ++c->tm_step;
    if ((s = timed(c, K_MAP_TRAIN, 2.0 * 4.0 * SmallMap::macs() * cfg->batch * ta.S, 0.0,
                   [&] { return launch_map_grad(ta, c->stream); })))
      return s;
  }
  HIP_TRY(c, hipMemcpyAsync(c->params_host.data(), c->tm_params.p, 4L * kSmallMapParams, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return tm_repack(c);
}

loc_status loc_get_map(loc_ctx* c, float* params, size_t n) {
  if (!c) return LOC_E_ARG;
  c->err.clear();
  if (!params || n != c->params_host.size()) return fail(c, LOC_E_ARG, "expected %zu floats", c->params_host.size());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(params, c->params_host.data(), 4 * n);
  return LOC_OK;
}

}  // extern "C"

extern "C" {

loc_status loc_init_grid_map(const loc_grid_desc* g, void* hip_stream, loc_ctx** out) {
  if (!out) return LOC_E_ARG;
  *out = nullptr;
  if (!g || !g->tables || !g->mlp) return LOC_E_ARG;
  if (g->levels != 4 && g->levels != 8 && g->levels != 16) return LOC_E_UNSUPPORTED;
  if (g->L_dir != 2 && g->L_dir != 4) return LOC_E_UNSUPPORTED;
  if (g->log2_table < 10 || g->log2_table > 24 || g->n_min < 2 || g->n_max < g->n_min || g->n_max > (1 << 16) ||
      !(g->bound > 0.0f))
    return LOC_E_ARG;
  if (!(g->near_ >= 0.0f && g->far_ > g->near_)) return LOC_E_ARG;
  if (g->n_coarse < 1 || g->n_coarse > 256 || g->n_fine < 0 || g->n_fine > 256) return LOC_E_ARG;
  if (!(g->alpha > 0.0f && g->alpha < 0.5f) || !(g->tau > 0.0f)) return LOC_E_ARG;
  const int L = g->levels, in_d = 3 + 6 * g->L_dir;
  const long n_mlp = 64L * 2 * L + 64 + 16L * 64 + 16 + 64L * (16 + in_d) + 64 + 3L * 64 + 3;
  if ((long)g->n_mlp != n_mlp) return LOC_E_ARG;
  loc_ctx* c = new (std::nothrow) loc_ctx();
  if (!c) return LOC_E_OOM;
  c->desc = loc_map_desc{};
  c->desc.precision = LOC_FP32;
  c->desc.near_ = g->near_;
  c->desc.far_ = g->far_;
  c->desc.n_coarse = g->n_coarse;
  c->desc.n_fine = g->n_fine;
  c->desc.alpha = g->alpha;
  c->desc.tau = g->tau;
  c->desc.jitter = g->jitter;
  c->kind = kMapGrid;
  c->macs = n_mlp - (64 + 16 + 64 + 3);
  c->bytes_per_sample = 8.0 * 4.0 * L + 20.0;   // 8 corners x one word (two half features) per level, sample out
  c->stream = (hipStream_t)hip_stream;
  {
    hipDeviceProp_t prop;
    if (hipGetDevice(&c->device) == hipSuccess && hipGetDeviceProperties(&prop, c->device) == hipSuccess)
      c->n_cu = prop.multiProcessorCount;
  }
  if (noalloc_scratch(c->device, &c->noalloc_prefix) != hipSuccess) {
    (void)hipGetLastError();
    loc_destroy(c);
    return LOC_E_HIP;
  }
  // resolutions N_l = floor(N_min b^l + 1e-6), b = exp((ln N_max - ln N_min) / (L - 1))
  GridDev& d = c->grid;
  d.levels = L;
  d.log2_table = g->log2_table;
  d.in_d = in_d;
  d.n_mlp = (int)n_mlp;
  d.bound = g->bound;
  d.dense_mask = 0;
  const double b = L > 1 ? std::exp((std::log((double)g->n_max) - std::log((double)g->n_min)) / (L - 1)) : 1.0;
  for (int l = 0; l < L; ++l) {
    const long N = (long)std::floor((double)g->n_min * std::pow(b, l) + 1e-6);
    d.res[l] = (int)N;
    if ((N + 1) * (N + 1) * (N + 1) <= (1L << g->log2_table)) d.dense_mask |= 1u << l;
  }
  // tables rounded to half precision (nearest even), one 32-bit word per entry
  const size_t n_tab = (size_t)L << g->log2_table;
  std::vector<uint32_t> H(n_tab);
  for (size_t i = 0; i < n_tab; ++i) {
    const _Float16 a = (_Float16)g->tables[2 * i], b = (_Float16)g->tables[2 * i + 1];
    H[i] = (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
  // encoding workspace: 2^21 samples per chunk (16 MB per level)
  d.feat_cap = 1L << 21;
  bool ok = hipMalloc(&c->flags, sizeof(int)) == hipSuccess && hipMalloc(&c->grid_tab, n_tab * 4) == hipSuccess &&
            hipMalloc(&c->grid_mlp, n_mlp * 4) == hipSuccess &&
            hipMalloc(&c->grid_feat, (size_t)d.feat_cap * L * sizeof(float2)) == hipSuccess &&
            hipMalloc(&c->grid_pts, (size_t)d.feat_cap * sizeof(float4)) == hipSuccess &&
            hipMemcpy(c->grid_tab, H.data(), n_tab * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->grid_mlp, g->mlp, n_mlp * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemsetAsync(c->flags, 0, sizeof(int), c->stream) == hipSuccess &&
            hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    loc_destroy(c);
    return LOC_E_HIP;
  }
  d.tables = c->grid_tab;
  d.mlp = c->grid_mlp;
  d.feat = c->grid_feat;
  d.pts = c->grid_pts;
  *out = c;
  return LOC_OK;
}

}  // extern "C"
