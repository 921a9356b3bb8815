// Kernel argument blocks and launchers of the particle-update library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

enum MapKind { kMapSmall = 0, kMapNerf = 1, kMapGrid = 2 };

// map evaluation over n_samples = n_rays * spr samples laid out [ray][k]
struct MlpArgs {
  const float4* ray_o;   // per ray origin (xyz, pad)
  const float4* ray_d;   // per ray unit direction (xyz, pad)
  const float* t_in;     // per sample depth, or NULL: stratified coarse samples
  float* t_out;          // coarse depths written when t_in == NULL
  float4* out;           // per sample (sigma, r, g, b)
  const float* weights;  // packed FP32 map (maplayout.h)
  const void* wblocks;   // packed BF16 weight chunks (maplayout_bf16.h)
  const float* bias;     // BF16 path: float32 biases
  const float* heads;    // BF16 path: float32 density / colour heads
  long n_samples;
  int spr;               // samples per ray in this pass
  int B;                 // rays per particle (ray = i * B + j)
  float near_, dt;       // coarse grid: t_k = near + (k + xi) dt
  int jitter;
  uint64_t seed, iter;
  // FP8 path, per layer l in execution order: E8M0 scale bytes of the weight
  // (2^-ew_l) and activation (2^-ea_l) operands, and the factor 2^ea_{l+1}
  // applied to layer l's output before it is rounded to E4M3
  int f8_sw[12], f8_sx[12];
  // optional second sample set evaluated by the same launch (BF16 and FP8
  // kernels): samples n_samples .. n_samples + n_samples2 - 1 are sample
  // s - n_samples of this set, laid out [ray][k] with spr2 per ray, depths
  // from t_in2, outputs to out2
  const float* t_in2;
  float4* out2;
  long n_samples2;
  int spr2;
};
hipError_t launch_mlp(int map_kind, const MlpArgs& a, hipStream_t st);
hipError_t launch_mlp_bf16(int map_kind, const MlpArgs& a, hipStream_t st);
hipError_t launch_mlp_fp8(int map_kind, const MlpArgs& a, hipStream_t st);

// FP8 calibration: float32 evaluation of the 8x256 map at the midpoints of
// spr strata on each ray, recording per layer l (execution order 0..D) the
// largest |output| (after ReLU where the layer has one) into amax[l]
struct CalibArgs {
  const float* o;        // n_rays x 3
  const float* d;        // n_rays x 3
  int n_rays, spr;
  float near_, dt;
  const float* wt;       // per layer, transposed weights (in x out) then bias (out)
  unsigned* amax;        // float bits of non-negative maxima, D + 1 entries
};
hipError_t launch_calibrate_fp8(const CalibArgs& a, hipStream_t st);

struct Pose12 { double m[12]; };

struct PredictArgs {
  const double* pose_in;
  double* pose_out;
  Pose12 motion;         // O_t
  double sigma_t, sigma_r;
  int N;
  uint64_t seed, iter;
};
hipError_t launch_predict(const PredictArgs& a, hipStream_t st);

struct RaygenArgs {
  const double* pose;    // N x 12 predicted poses
  const float* image;    // full-resolution H x W x 3
  int W_full, s;         // full width, level factor
  int Wl, Hl;            // level resolution
  double fx, fy, cx, cy; // level intrinsics R K
  int N, B;
  uint64_t seed, iter;
  float4* ray_o;
  float4* ray_d;
  float4* obs;           // I^R(p_j) per ray (rgb, pad)
  int all_pixels;        // 1: ray j goes through level pixel j (row-major) instead of a drawn pixel
};
hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st);

struct FineArgs {
  const float* t_coarse;   // [ray][Sc]
  const float4* out_coarse;
  float* t_fine;           // [ray][Sf]
  int n_rays, Sc, Sf, B;
  float far_;
  int jitter;
  uint64_t seed, iter;
};
hipError_t launch_fine(const FineArgs& a, hipStream_t st);

struct CompositeArgs {
  const float* t_coarse;
  const float4* out_coarse;
  const float* t_fine;     // NULL when Sf == 0
  const float4* out_fine;
  const float4* obs;
  int N, B, Sc, Sf;
  float far_, log_trans, log_opq, tau;   // log(1 - alpha), log(alpha)
  float empty_F;                         // F of a ray that never reaches opacity alpha
  float4* ray_rgba;        // per ray (C, A)
  float2* ray_fe;          // per ray (F, E)
  double* loglik;          // per particle, or NULL (teacher mode)
  float* uncert;           // per particle mean F, may be NULL
  float* hist;             // per ray 32-bin weight histogram (teacher targets), or NULL
  int n_rays;              // rays present (N * B, or fewer in teacher mode)
  float near_;
};
hipError_t launch_composite(const CompositeArgs& a, hipStream_t st);

constexpr int kProposalParams = 64 * 78 + 64 + 64 * 64 + 64 + 32 * 64 + 32;   // 11296

struct ProposalArgs {
  const float4* ray_o;
  const float4* ray_d;
  const float* params;     // flat proposal parameters (device)
  float* hist;             // per ray 32 probabilities, or NULL
  float* t_fine;           // per ray Sf fine depths (when Sf > 0)
  int n_rays, Sf, B;
  float near_, far_;
  int jitter;
  uint64_t seed, iter;
};
hipError_t launch_proposal_fine(const ProposalArgs& a, hipStream_t st);

struct TrainArgs {
  const float4* ray_o;
  const float4* ray_d;
  const float* target;     // per ray 32
  const float* params;     // read by the gradient kernel
  float* params_rw;        // Adam update target (same buffer), or NULL
  float* m;
  float* v;
  float* partial;          // n_waves x kProposalParams
  float* loss_partial;     // n_waves
  float* loss_out;         // mean loss per call at loss_index, or NULL
  float* grad_out;         // summed gradient, or NULL
  int loss_index;
  int n_rays, first, batch, rays_per_wave, n_waves;
  int adam, step;
  float lr, beta1, beta2, eps;
};
hipError_t launch_prop_grad(const TrainArgs& a, hipStream_t st);
// the same gradient with bf16 operands on the matrix cores (float32
// accumulation), prop_rays_per_wave_bf16() rays per wave
hipError_t launch_prop_grad_bf16(const TrainArgs& a, hipStream_t st);
int prop_rays_per_wave_bf16();
// multi-resolution grid map (levels 4, 8 or 16; direction bands <= 4)
constexpr int kGridMaxLevels = 16;
constexpr int kGridMaxDirBands = 4;
struct GridDev {
  const uint32_t* tables;  // levels x 2^log2_table entries: two half-precision features (low, high)
  const float* mlp;        // tiny MLP, flat canonical order
  int n_mlp;
  int levels, log2_table, in_d;
  uint32_t dense_mask;     // bit l: level l indexes its vertices densely
  int res[kGridMaxLevels];
  float bound;
  float2* feat;            // encoding workspace: levels x feat_cap (f_2l, f_2l+1) per sample
  float4* pts;             // feat_cap sample positions (u in the unit cube, inside flag)
  long feat_cap;           // samples per encoding chunk
};
hipError_t launch_grid_map(const GridDev& g, const MlpArgs& a, hipStream_t st);

// training of the 4x64 map with the photometric loss (Eq. 2)
constexpr int kSmallMapParams = 15345;
struct MapTrainArgs {
  const float4* ray_o;
  const float4* ray_d;
  const float* target;     // per ray 3 (rgb)
  const float* params;     // canonical order, read by the gradient kernel
  float* params_rw;        // Adam update target (same buffer), or NULL
  float* m;
  float* v;
  float* partial;          // n_waves x kSmallMapParams
  float* loss_partial;     // n_waves
  float* loss_out;         // mean loss per call at loss_index, or NULL
  float* grad_out;         // summed gradient, or NULL
  int loss_index;
  int n_rays, first, batch, rays_per_wave, n_waves;
  int adam, step;
  float lr, beta1, beta2, eps;
  int S, jitter;           // coarse samples per ray (<= 64), stratified jitter
  int bf16;                // 1: bfloat16 products on the matrix cores (S = 32), else float32
  uint64_t seed, iter;     // sample streams keyed (ray, 0) at counter iter
  float near_, far_, dt;
};
hipError_t launch_map_grad(const MapTrainArgs& a, hipStream_t st);
hipError_t launch_rays_to_f4(const float* o3, const float* d3, int n, float4* o4, float4* d4, hipStream_t st);
hipError_t launch_rays_from_f4(const float4* o4, const float4* d4, int n, float* o3, float* d3, hipStream_t st);

hipError_t launch_normalize(const double* loglik, double* weight, int N, int* flags, hipStream_t st);

hipError_t launch_resample(const double* weight, int n_in, int n_out, uint64_t seed, uint64_t iter,
                           unsigned long long* prefix, int32_t* idx, int* flags, hipStream_t st);
// the allocation-free resampling call's scratch (kNoAllocMaxWeights uint64
// entries per GPU): its device address on `device`, resolved once per device
constexpr int kNoAllocMaxWeights = 1 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, unsigned long long** out);

hipError_t launch_gather_poses(const double* in, const int32_t* idx, int n_in, int n_out, double* out,
                               hipStream_t st);
hipError_t launch_pose_estimate(const double* pose, const double* w, int N, double* est, int* flags, hipStream_t st);
hipError_t launch_position_variance(const double* pose, const double* w, int N, double* var, hipStream_t st);

hipError_t launch_split_ray_outputs(const float4* rgba, const float2* fe, int n, float* rgb,
                                    float* opacity, float* F, float* E, hipStream_t st);

// ---------------------------------------------------------------------------
// coarse-to-fine path (small map in bf16, 32 stratified samples per ray).
// The per-call values live in a device-side key so that a captured graph of
// the level sequence replays with new seeds, motion and noise.
struct LevelKey {
  uint64_t seed, iter;    // level L uses iteration counter iter + L
  double motion[12];      // O_t (3 x 4)
  double sigma_t, sigma_r;
};

struct LevelRayArgs {
  const LevelKey* key;
  int level;
  const double* pose;     // N x 12 predicted poses of this level
  const float* image;     // full-resolution H x W x 3
  int W_full, s, Wl, Hl;  // level factor s, level resolution
  double fx, fy, cx, cy;  // level intrinsics
  int N, B;
  const void* wblocks;    // BF16 small-map chunks, biases, heads (maplayout_bf16.h)
  const float* bias;
  const float* heads;
  float near_, dt, far_, log_trans, log_opq, tau;
  float empty_F;                         // F of a ray that never reaches opacity alpha
  int jitter;
  float4* ray_rgba;       // per ray (C, A)
  float2* ray_fe;         // per ray (F, E)
};

struct LevelFinishArgs {
  const LevelKey* key;
  int level;
  const float2* ray_fe;   // this level's per-ray (F, E)
  int N, B, reject;
  const double* pose;     // this level's predicted poses
  double* loglik;         // N (after rejection: -inf for rejected particles)
  float* uncert;          // N mean F
  double* weight;         // N
  int32_t* idx;           // n_out resampled indices
  unsigned long long* prefix;  // N scratch
  int n_out;
  double* next_pose;      // n_out x 12
  int predict_next;       // apply the next level's prediction to the drawn poses
  double* inc;            // n_out x 12: the next level's motion increments (written by the begin kernel)
  double* est;            // 12: pose read-out of this level's weighted set, or NULL
  int* flags;
};

// the motion increments of the levels after the first, drawn by the begin
// kernel: level L's n[L] drawn particles get their increment for level L + 1
// in inc[L] (n[L] x 12; n[L] = 0 where no level follows)
constexpr int kMaxLevels = 8;
struct LevelIncs {
  double* inc[kMaxLevels];
  int n[kMaxLevels];
};

hipError_t launch_level_begin(LevelKey* key, const LevelKey& v, const double* pose_in, double* pose_out, int N,
                              const LevelIncs& incs, hipStream_t st);
hipError_t set_level_begin_node(hipGraphExec_t ge, hipGraphNode_t node, LevelKey* key, const LevelKey& v,
                                const double* pose_in, double* pose_out, int N, const LevelIncs& incs);
// tile configuration (column tiles per wave, waves per workgroup), grid size
hipError_t launch_level_rays(const LevelRayArgs& a, int ntl, int waves, int blocks, hipStream_t st);
bool level_rays_config_ok(int ntl, int waves);
hipError_t launch_level_scores(const LevelFinishArgs& a, hipStream_t st);
hipError_t launch_level_finish(const LevelFinishArgs& a, hipStream_t st);

}  // namespace fl
