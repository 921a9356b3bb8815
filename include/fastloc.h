/*
 * fastloc.h -- C ABI of the MI355X (gfx950) particle-update library for
 * Monte Carlo localization on a NeRF map (Fast Loc-NeRF, arXiv 2406.12202).
 *
 * One MCL step (Alg. 1) is two calls:
 *   loc_update_particles  -- the per-particle loop of Alg. 1: prediction
 *                            x_t = x_{t-1} O_t Exp(delta) (Sec. III-A), the
 *                            downscaled observation, rendering of B_t query
 *                            pixels per particle with intrinsics R_t K (Eq. 1),
 *                            the uncertainty F = max(z_opaque - z_trans, tau)
 *                            (Eq. 5 and below Eq. 6) and the particle
 *                            rejection weight of Eq. 6, normalised (Eq. 3);
 *   loc_resample          -- the draw loop of Alg. 1: N_t indices drawn with
 *                            probability proportional to the weights.
 *
 * Conventions for every entry point:
 *  - C linkage; no exception crosses the ABI; every call returns a loc_status.
 *  - Arguments are validated on the host before anything is enqueued; a
 *    rejected call enqueues nothing and returns LOC_E_ARG (detail text in
 *    loc_last_error).
 *  - Array arguments marked DEVICE are device pointers owned by the caller
 *    (for example torch tensor storage) and must stay valid until the work
 *    enqueued on the context's stream has completed.  HOST arguments are read
 *    before the call returns.
 *  - Work is enqueued on the HIP stream given to loc_init_map and the call
 *    returns before it completes.  Failures of enqueued work surface as
 *    LOC_E_HIP from a later call.  Conditions only known on the device
 *    (degenerate weights) are reported by loc_sync through its flags.
 *  - A context may be used by one host thread at a time.  It owns the packed
 *    map weights and a workspace that grows on demand; calls on one context
 *    are serialised by its stream.
 *
 * Random draws (query pixels, stratified jitter, fine jitter, motion noise,
 * resampling offset) come from Philox4x32-10 (Salmon et al., SC'11) with
 *   key     = (seed & 0xffffffff, seed >> 32)
 *   counter = (c0, c1, iter & 0xffffffff, (stream << 24) | group)
 * and streams
 *   1 query pixel j             c0 = j, c1 = 0; p_j = (word0 * W'H') >> 32,
 *                               flat index v * W' + u at the level resolution
 *   2 coarse jitter of sample k of ray (i, j)   c0 = i, c1 = j, group k / 4,
 *                               word k % 4; xi = (word >> 8) * 2^-24
 *   3 fine jitter of sample m of ray (i, j)     as 2 with m
 *   4 motion noise of particle i  c0 = i, c1 = 0, groups 0 and 1 (Box-Muller
 *                               on u = (word + 1/2) 2^-32, pairs (w0,w1),
 *                               (w2,w3), (w4,w5) -> rho = sigma_t (g0,g1,g2),
 *                               phi = sigma_r (g3,g4,g5))
 *   5 resampling offset         c0 = c1 = 0, group 0, word 0 = r0
 * so results are reproducible from (seed, iter) on any device.
 */
#ifndef FASTLOC_H
#define FASTLOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct loc_ctx loc_ctx;

typedef enum {
  LOC_OK = 0,
  LOC_E_ARG = -1,          /* invalid argument (nothing enqueued)              */
  LOC_E_HIP = -2,          /* a HIP runtime call or enqueued kernel failed     */
  LOC_E_OOM = -3,          /* device allocation failed                         */
  LOC_E_DEGENERATE = -4,   /* all weights zero / no finite log-likelihood      */
  LOC_E_UNSUPPORTED = -5,  /* map shape or precision not compiled in           */
  LOC_E_STATE = -6         /* call order violated (e.g. no update before read) */
} loc_status;

typedef enum { LOC_FP32 = 0, LOC_BF16 = 1, LOC_FP8_E4M3 = 2 } loc_precision;

/*
 * The NeRF map M (Sec. III-A: F_NeRF(x, d) -> (c, sigma)) and renderer settings.
 *
 * Map: positional encoding gamma(p) = (p, sin(2^0 pi p), cos(2^0 pi p), ...,
 * sin(2^{L-1} pi p), cos(2^{L-1} pi p)) of widths in_x = 3 + 6 L_xyz and
 * in_d = 3 + 6 L_dir, then n_layers ReLU layers of `width` units.
 * `params` is a HOST float32 array of n_params values in this order
 * (each W row-major out x in, then its bias):
 *   for l in 0..n_layers-1: W_l, b_l with in_0 = in_x,
 *        in_l = width + in_x if l == skip_layer (input [h_{l-1}, gamma(x)]),
 *        in_l = width otherwise (skip_layer < 1 disables the skip input);
 *   sigma head (1 x width), sigma = softplus(w h + b);
 *   if dir_width > 0: feature (width x width, linear), dir
 *        (dir_width x (width + in_d), ReLU, input [feature, gamma(d)]),
 *        rgb (3 x dir_width, sigmoid);
 *   else rgb (3 x (width + in_d), sigmoid, input [h_{n_layers-1}, gamma(d)]).
 * The array is copied and repacked during loc_init_map.
 * Compiled map shapes: (n_layers, width, skip_layer, L_xyz, L_dir, dir_width)
 * = (4, 64, -1, 6, 2, 0) and (8, 256, 5, 10, 4, 128); others return
 * LOC_E_UNSUPPORTED.
 *
 * Rendering (Eq. 1 as a Riemann sum): stratified samples
 * t_k = near + (k + xi_k)(far - near)/n_coarse (xi = 0 when jitter == 0),
 * interval lengths delta_k = t_{k+1} - t_k, delta_last = far - t_last,
 * density and colour constant on each interval, black background.
 * n_fine > 0 adds hierarchical samples: inverse-CDF placement on the coarse
 * pdf with mass w_k + 1e-5 delta_k at u_m = (m + xi'_m)/n_fine (xi' = 1/2
 * when jitter == 0), merged with the coarse samples (stable order).
 * alpha: Eq. 5 threshold (the paper gives none; 0.05 by default);
 * tau: lower bound of F (0.1 in the paper's experiments).
 */
typedef struct {
  int n_layers, width, skip_layer;
  int L_xyz, L_dir, dir_width;
  const float* params;     /* HOST */
  size_t n_params;
  loc_precision precision; /* LOC_FP32, LOC_BF16 (bf16 map, float32 accumulate), or
                              LOC_FP8_E4M3 (8x256 map only: hidden-to-hidden products
                              in OCP E4M3 with per-layer power-of-two scales, products
                              with the encodings in bf16, heads in float32; needs
                              loc_calibrate_fp8 before use) */
  float near_, far_;
  int n_coarse, n_fine;    /* n_coarse in [1, 256], n_fine in [0, 256] */
  float alpha, tau;        /* 0 < alpha < 0.5, tau > 0 */
  int jitter;              /* 1 stratified jitter, 0 deterministic */
} loc_map_desc;

/* Full-resolution pinhole intrinsics K (OpenGL camera: x right, y up, looking
 * along -z; pixel (u, v) has centre (u + 1/2, v + 1/2)).  At level factor
 * s = 1/R the intrinsics are R K = (fx/s, fy/s, cx/s, cy/s). */
typedef struct { int W, H; double fx, fy, cx, cy; } loc_camera;

/* Multi-resolution grid map (the map type of Sec. IV-B, read as a
 * multiresolution hash encoding with a tiny MLP; no anti-aliased
 * multisampling).  The map covers [-bound, bound]^3 (u = (x + bound) /
 * (2 bound); points outside are empty); level l = 0..levels-1 has resolution
 * N_l = floor(n_min b^l + 1e-6), b = exp((ln n_max - ln n_min) / (levels - 1));
 * a point's level feature is the trilinear blend (weights prod (1 - |p - c|),
 * p = u N_l) of the two-feature entries of its cell's 8 corners c, indexed
 * densely (c_0 + c_1 (N_l + 1) + c_2 (N_l + 1)^2) while (N_l + 1)^3 <= T and
 * by the hash (c_0 xor 2654435761 c_1 xor 805459861 c_2) mod 2^32 mod T
 * otherwise.  Network: z = W2 relu(W1 f + b1) + b2 (64 hidden, 16 outputs),
 * sigma = softplus(z_0), rgb = sigmoid(W4 relu(W3 [z, gamma(d)] + b3) + b4)
 * (64 hidden).  Rendering settings as loc_map_desc; the map runs in float32.
 *   tables  HOST levels x T x 2 float32 (T = 2^log2_table, level-major);
 *           stored on the device in half precision (rounded to nearest even
 *           on upload; values representable in half precision are exact)
 *   mlp     HOST n_mlp float32: W1 (64 x 2 levels), b1, W2 (16 x 64), b2,
 *           W3 (64 x (16 + 3 + 6 L_dir)), b3, W4 (3 x 64), b4 (row-major)
 * levels in {4, 8, 16}, L_dir in {2, 4} (LOC_E_UNSUPPORTED otherwise),
 * log2_table in [10, 24], 2 <= n_min <= n_max <= 2^16.  Every update,
 * render and localisation call accepts the context; the coarse-to-fine level
 * path, FP8 calibration and map training return LOC_E_UNSUPPORTED.  Besides
 * the tables (4 B per entry) the context owns an evaluation workspace of
 * 2^21 samples: 8 B per sample and level of features plus 16 B per sample of
 * positions (288 MB at 16 levels); larger sample sets are evaluated in chunks
 * of that size, with results independent of the chunking. */
typedef struct {
  int levels, log2_table, n_min, n_max;
  float bound;
  int L_dir;
  const float* tables;
  const float* mlp;
  size_t n_mlp;
  float near_, far_;
  int n_coarse, n_fine;
  float alpha, tau;
  int jitter;
} loc_grid_desc;
loc_status loc_init_grid_map(const loc_grid_desc* map, void* hip_stream, loc_ctx** out);

/* Create a context for map `map` bound to `hip_stream` (a hipStream_t, or
 * NULL for the null stream) on the current HIP device.  *out receives the
 * context; on failure *out is NULL. */
loc_status loc_init_map(const loc_map_desc* map, void* hip_stream, loc_ctx** out);

/*
 * One MCL weighting pass over N particles (Alg. 1, per-particle loop;
 * Sec. III-B/C).
 *   image_rgb  DEVICE H x W x 3 float32 (row-major, RGB) full-resolution I_t
 *   cam        HOST   full-resolution intrinsics; W and H divisible by inv_R
 *   inv_R      level factor s in {1, 2, 4, 8}: R_t = 1/s; the observation is
 *              box-averaged over s x s blocks (downscale(I_t, R_t))
 *   B, N       query pixels per particle B_t (1..1024) and particles (>= 1,
 *              N B <= 2^22 rays per call; LOC_E_ARG otherwise)
 *   pose_in    DEVICE N x 12 float64 camera-to-world [R | t], row-major
 *   motion     HOST   12 float64 O_t, or NULL for the identity
 *   sigma_t, sigma_r  prediction noise (scene units, radians), >= 0
 *   seed, iter  Philox key / counter word (see the header comment)
 *   pose_out   DEVICE N x 12 float64: predicted x_t (may equal pose_in)
 *   loglik_out DEVICE N float64: l_i = 4 (ln B - ln max(S_i, 1e-12)) with
 *              S_i = sum_j E_ij F_ij and E_ij = |I^R(p_j) - C_ij|^2 summed
 *              over RGB (Eq. 6 in log form: w_i proportional to e^{l_i})
 *   weight_out DEVICE N float64: w_i = e^{l_i - max l} / sum_k e^{l_k - max l}
 *              (non-finite l_i -> 0; if none is finite all are 0 and loc_sync
 *              reports LOC_FLAG_DEGENERATE_WEIGHTS)
 *   uncert_out DEVICE N float32: mean_j F_ij, or NULL
 */
loc_status loc_update_particles(loc_ctx* ctx, const float* image_rgb, const loc_camera* cam,
                                int inv_R, int B, int N, const double* pose_in,
                                const double* motion, double sigma_t, double sigma_r,
                                uint64_t seed, uint64_t iter, double* pose_out,
                                double* loglik_out, double* weight_out, float* uncert_out);

/*
 * Alg. 1 draw loop: systematic resampling with integer thresholds.
 *   weight   DEVICE n_in float64 (w <= 0 or non-finite counts as 0)
 *   idx_out  DEVICE n_out int32, non-decreasing
 * q_i = floor(w_i / w_max * 2^40), Q = sum q_i (exact), r0 = word 0 of stream
 * 5, theta_k = floor((k 2^32 + r0) Q / (n_out 2^32)), idx_k = min{i : q_0 +
 * ... + q_i > theta_k}.  Every step is exact or a correctly rounded division,
 * so the indices are bit-identical to any exact implementation.  If Q = 0 all
 * indices are -1 and loc_sync reports LOC_FLAG_DEGENERATE_RESAMPLE.
 * 1 <= n_in <= 2^24 - 1 (so that Q < 2^64) and 1 <= n_out <= 2^24.
 */
loc_status loc_resample(loc_ctx* ctx, const double* weight, int n_in, int n_out,
                        uint64_t seed, uint64_t iter, int32_t* idx_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * loc_resample without any allocation.  Same arguments, result and flags as
 * loc_resample (bit-identical indices); the integer prefix lives in a fixed
 * library-owned device array of LOC_NOALLOC_MAX_WEIGHTS uint64 entries
 * (8 MiB), one per GPU, held from library load until the process ends, whose
 * address is resolved when a context is created.  The call allocates
 * nothing and calls no allocating routine.
 *   1 <= n_in <= LOC_NOALLOC_MAX_WEIGHTS, else LOC_E_ARG (no launch);
 *   1 <= n_out <= 2^24.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap in time on one GPU (several streams or
 * contexts) race, and the caller must serialise them.
 */
#define LOC_NOALLOC_MAX_WEIGHTS (1 << 20)
loc_status loc_resample_noalloc(loc_ctx* ctx, const double* weight, int n_in, int n_out,
                                uint64_t seed, uint64_t iter, int32_t* idx_out);

/*
 * Eq. 5 for a ray whose accumulated opacity never reaches alpha: the set
 * defining z_trans is empty.  mode 0 (default): inf of the empty set is
 * +inf, so the gap z_opaque - z_trans is -inf and F = tau (the smallest
 * factor; an empty ray is scored by its colour error alone).  mode 1: such a
 * ray has no transition from transparent to opaque in the sampled span and
 * counts as maximally uncertain, F = far - near.  Applies to later update,
 * level, localisation and render calls (a captured level graph is dropped).
 * LOC_E_ARG for another mode.
 */
loc_status loc_set_empty_ray_uncertainty(loc_ctx* ctx, int mode);

/* FP8 calibration of an LOC_FP8_E4M3 context (per-layer amax scaling): the
 * float32 map is evaluated at the midpoints of the n_coarse strata of each of
 * n_rays rays (o, d: DEVICE n_rays x 3 float32, e.g. loc_cast_rays output),
 * the largest |output| of every layer sets the power-of-two scale 2^ea of the
 * next layer's E4M3 input (largest with amax 2^ea <= 448), the largest |weight|
 * of every hidden-to-hidden block sets 2^ew likewise, and the weights are
 * packed.  Values beyond the calibrated range saturate at +-448.  Synchronous.
 * n_rays in [1, 2^20].  LOC_E_STATE for a context of another precision.
 * Update and teacher calls on an FP8 context return LOC_E_STATE until this has
 * run. */
loc_status loc_calibrate_fp8(loc_ctx* ctx, const float* o, const float* d, int n_rays);

/* The calibrated exponents (HOST arrays of n >= 10 entries, any may be NULL):
 * ew[l], ea[l] of layer l in execution order (0..7 trunk, 8 feature, 9
 * direction; ew[0] = ea[0] = 0, the input layer being bf16) and amax[l], the
 * calibrated largest |output| of layer l (l <= 8). */
loc_status loc_fp8_scales(loc_ctx* ctx, int* ew, int* ea, float* amax, int n);

/* ---------------------------------------------------------------- levels
 * Coarse-to-fine update (Alg. 1 with per-iteration R_t, B_t, N_t, Sec. III-C)
 * for the 4x64 map in BF16 with 32 coarse and no fine samples.  Level L of a
 * call is one MCL iteration with counter iter + L: the N_L particles are
 * predicted (motion O, noise sigma_t, sigma_r, as loc_update_particles), each
 * casts B rays at scale 1/inv_R, S_i and l_i follow Eq. 6, and with `reject`
 * particles whose mean F exceeds mean + one (population) standard deviation
 * over the particles are given weight 0 (1-sigma rejection); the weights are
 * normalised (Eq. 3) and n_out particles are drawn (systematic, integer-exact,
 * as loc_resample) to carry on: N_0 = N, N_{L+1} = levels[L].n_out.
 * Per level the work is one persistent fused kernel over the level's rays
 * (ray generation, samples, encoding, map, compositing, F, E), a kernel of
 * per-particle scores, and one single-workgroup kernel (rejection,
 * normalisation, read-out, resampling, gather, next prediction). */
typedef struct {
  int inv_R;   /* level scale R = 1 / inv_R, inv_R in {1, 2, 4, 8} */
  int B;       /* rays per particle, [1, 1024] */
  int n_out;   /* particles drawn at the end of the level, [1, 2^20] */
} loc_level;

/* image: DEVICE H x W x 3 float32; levels: HOST array of n_levels (1..8);
 * pose_in: DEVICE N x 12 float64 (N in [1, 2^20]); motion: HOST 12 float64 or
 * NULL; pose_out: DEVICE levels[n_levels-1].n_out x 12 float64, the last
 * level's drawn poses; est_out: DEVICE 12 float64 or NULL, the pose read-out
 * (loc_pose_estimate) of the last level's weighted set.  Per-level results are
 * kept until the next level call (loc_level_outputs).  N_L * B <= 2^26.
 * LOC_E_UNSUPPORTED for another map or sampling.  All weights zero at a level:
 * LOC_FLAG_DEGENERATE_RESAMPLE and NaN poses for the next level.  In graph
 * mode the sequence after a small key upload is a captured hipGraph, replayed
 * while image, camera, levels, N, pointers, `reject` and tile choices stay the
 * same (seed, iter, motion and noise may change). */
loc_status loc_update_levels(loc_ctx* ctx, const float* image, const loc_camera* cam, int n_levels,
                             const loc_level* levels, int N, const double* pose_in, const double* motion,
                             double sigma_t, double sigma_r, uint64_t seed, uint64_t iter, int reject,
                             double* pose_out, double* est_out);

/* enable (1) or disable (0) graph capture and replay of loc_update_levels */
loc_status loc_set_graph_mode(loc_ctx* ctx, int enable);

/* Results of level `level` of the last level call, copied on the context's
 * stream into DEVICE buffers (any may be NULL): loglik N_L float64 (-inf for
 * rejected particles), weight N_L float64, uncert N_L float32 (mean F), idx
 * n_out int32 (drawn indices), pose N_L x 12 float64 (predicted poses). */
loc_status loc_level_outputs(loc_ctx* ctx, int level, double* loglik, double* weight, float* uncert,
                             int32_t* idx, double* pose);

/* Per-ray results of level `level` (as loc_ray_outputs): N_L * B entries. */
loc_status loc_level_ray_outputs(loc_ctx* ctx, int level, float* rgb, float* opacity, float* F, float* E);

/* Autotuner of the fused ray kernel for the given level schedule (the same
 * arguments as loc_update_levels): times every tile configuration and grid
 * size on the level's real particles over `reps` launches and keeps the
 * fastest per level.  cache_path (HOST string or NULL): a file of one JSON
 * object per line {"key", "ntl", "waves", "blocks", "us_per_launch"}, read for
 * known levels and appended with new choices.  chosen: HOST 3 * n_levels ints
 * (column tiles per wave, waves per workgroup, workgroups) or NULL.
 * Synchronous.  Every configuration computes identical results. */
loc_status loc_autotune_levels(loc_ctx* ctx, const float* image, const loc_camera* cam, int n_levels,
                               const loc_level* levels, int N, const double* pose_in, int reps,
                               const char* cache_path, int* chosen);

/* Set level `level`'s tile choice by hand: ntl = 2 (rays per wave pass),
 * waves per workgroup in {2, 4, 8}, blocks >= 1; (0, 0, 0) restores the
 * default. */
loc_status loc_set_level_tiles(loc_ctx* ctx, int level, int ntl, int waves, int blocks);

/* Poses of the resampled set (Alg. 1, "add x_t^[i] to X_t"): pose_out[k] =
 * pose_in[idx[k]], DEVICE N x 12 float64 arrays and DEVICE int32 indices (an
 * index outside [0, n_in) leaves pose_out[k] unchanged). */
loc_status loc_gather_poses(loc_ctx* ctx, const double* pose_in, int n_in, const int32_t* idx, int n_out,
                            double* pose_out);

/* Pose read-out from a weighted particle set (the paper does not say how):
 * est (DEVICE 12 float64) = [R | t] with t = sum w_i t_i / sum w_i and R the
 * chordal L2 mean U diag(1, 1, det(U V^T)) V^T of sum_i w_i R_i = U S V^T
 * (w <= 0 or non-finite counts as 0).  All weights zero: est is NaN and
 * loc_sync reports LOC_FLAG_DEGENERATE_WEIGHTS; a singular sum: NaN and
 * LOC_FLAG_SINGULAR_ROTATION. */
loc_status loc_pose_estimate(loc_ctx* ctx, const double* pose, const double* weight, int N, double* est);

/* Spread of a weighted particle set, the quantity whose fall below a
 * threshold triggers the next refinement stage (Sec. III-C): var (DEVICE 1
 * float64) = sum_i w_i |t_i - t_bar|^2 / sum_i w_i, t_bar the weighted mean
 * position (the trace of the weighted covariance of the 3D positions; the
 * paper names the variance of the positions without fixing the estimator).
 * pose DEVICE N x 12 float64, weight DEVICE N float64 (w <= 0 or non-finite
 * counts as 0).  NaN if no particle has weight.  N in [1, 2^24]. */
loc_status loc_position_variance(loc_ctx* ctx, const double* pose, const double* weight, int N, double* var);

/* Render the map from one pose at every pixel of the level-1/inv_R image
 * (Eq. 1 with the context's samples: stratified coarse plus hierarchical or
 * proposal-placed fine, as the update's rays; pixel centres and intrinsics as
 * loc_update_particles; sample streams keyed (particle 0, ray p) with p the
 * row-major pixel index).  pose DEVICE 12 float64; rgb DEVICE (H/inv_R) x
 * (W/inv_R) x 3 float32 (C, row-major); opacity DEVICE (H/inv_R) x (W/inv_R)
 * float32 (1 - T(far)) or NULL.  At most 2^22 pixels.  Enqueued. */
loc_status loc_render_image(loc_ctx* ctx, const loc_camera* cam, int inv_R, const double* pose, uint64_t seed,
                            uint64_t iter, float* rgb, float* opacity);

/* ------------------------------------------------------------ localisation
 * The localisation loop with variance-triggered refinement (Sec. III-C): the
 * set moves through stages of growing resolution and rays per particle and
 * shrinking particle counts; stage k weights the set at scale 1/inv_R with B
 * rays per particle and the set drawn while in stage k has N particles.  At
 * iteration t (counter iter + t): the set is predicted and weighted
 * (loc_update_particles at the current stage), its position variance
 * (loc_position_variance) and pose read-out (loc_pose_estimate) are taken;
 * if the variance is below the current stage's delta the next stage begins
 * (the last stage's delta is not used; NaN never switches); then the new
 * current stage's N particles are drawn (loc_resample, counter iter + t) and
 * gathered.  One stream synchronisation per iteration (the variance decides
 * the next launch sizes on the host). */
typedef struct {
  int inv_R;      /* level scale 1/inv_R, inv_R in {1, 2, 4, 8} */
  int B;          /* rays per particle, [1, 1024] */
  int N;          /* particles drawn while in this stage, [1, 2^24 - 1] */
  double delta;   /* variance threshold that ends the stage */
  double noise;   /* factor (>= 0) on sigma_t and sigma_r for the iterations
                     this stage weights (the paper fixes no noise schedule) */
} loc_stage;

typedef struct {
  long long iter; /* counter of the iteration */
  int stage;      /* stage that weighted the set */
  int n;          /* particles weighted */
  int n_next;     /* particles drawn (0: the set had no weight, the loop ended) */
  double var;     /* position variance of the weighted set */
  double est[12]; /* pose read-out of the weighted set */
  double ms;      /* host wall time of the iteration, milliseconds */
} loc_step_info;

/* Optional per-iteration record of the loop in DEVICE buffers, appended
 * iteration by iteration: pose (12 x capacity float64) the predicted poses
 * and weight (capacity float64) the normalised weights of the n particles
 * weighted, idx (capacity int32) the n_next drawn indices.  The loop fails
 * with LOC_E_ARG once capacity particles would be exceeded. */
typedef struct {
  double* pose;
  double* weight;
  int32_t* idx;
  long capacity;
} loc_trace;

/* image DEVICE H x W x 3 float32; stages HOST n_stages (1..8); pose_in
 * DEVICE n_in x 12 float64, the initial set (n_in in [1, 2^24 - 1]); motion,
 * sigma_t, sigma_r, seed as loc_update_particles; pose_out DEVICE (max N over
 * the stages) x 12 float64 receives the final set and *n_out its size (0 if
 * the loop ended on a set without weight); info HOST n_iters records or NULL;
 * *n_done (may be NULL) the iterations run; trace NULL or as above.
 * Synchronous. */
loc_status loc_localize(loc_ctx* ctx, const float* image, const loc_camera* cam, int n_stages,
                        const loc_stage* stages, int n_iters, int n_in, const double* pose_in,
                        const double* motion, double sigma_t, double sigma_r, uint64_t seed, uint64_t iter,
                        double* pose_out, int* n_out, loc_step_info* info, int* n_done,
                        const loc_trace* trace);

/* Per-ray results of the last loc_update_particles on this context, copied
 * into DEVICE arrays of N*B entries (ray (i, j) at i*B + j); any pointer may be
 * NULL.  rgb: 3 floats per ray (C), opacity: A = 1 - T(far), F: uncertainty,
 * E: squared colour error.  Enqueued on the stream. */
loc_status loc_ray_outputs(loc_ctx* ctx, float* rgb, float* opacity, float* F, float* E);

enum { LOC_FLAG_DEGENERATE_WEIGHTS = 1, LOC_FLAG_DEGENERATE_RESAMPLE = 2, LOC_FLAG_SINGULAR_ROTATION = 4 };

/* Wait for the context's stream; *flags (may be NULL) receives the OR of
 * LOC_FLAG_* raised since the previous loc_sync.  Returns LOC_E_HIP if
 * enqueued work failed. */
loc_status loc_sync(loc_ctx* ctx, int* flags);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * launches: enable = 1 times every launch, 2 only the map-evaluation launches
 * (the MLP or grid kernels and the fused level ray kernel), so that a timed
 * region carries two events per map launch and nothing around the small
 * kernels; 0 switches timing off; other values are LOC_E_ARG.
 * loc_kernel_stats waits for the stream and fills up to max entries (name,
 * launches, summed milliseconds, summed algorithmic FLOP and HBM bytes of
 * those launches); *n receives the number of kernels.  Any call of
 * loc_set_profiling clears the counters. */
typedef struct {
  char name[48];
  long long launches;
  double ms;
  double flop;
  double bytes;
} loc_kernel_stat;
loc_status loc_set_profiling(loc_ctx* ctx, int enable);
loc_status loc_kernel_stats(loc_ctx* ctx, loc_kernel_stat* out, int max, int* n);

/*
 * Learned proposal network (an extension of the paper's sampling: it places a
 * ray's fine samples from a predicted 32-bin histogram of the compositing
 * weights instead of from a coarse render).
 *   x = [gamma_6(o), gamma_6(d)] (78), h1 = relu(W1 x + b1) (64),
 *   h2 = relu(W2 h1 + b2) (64), z = W3 h2 + b3 (32), p = softmax(z);
 *   parameters: 11296 float32 in the order W1 (64 x 78), b1, W2 (64 x 64), b2,
 *   W3 (32 x 64), b3, row-major.
 * Placement: pdf 0.99 p_b + 0.01/32 on 32 equal bins of [near, far), inverse
 * CDF at u_m = (m + xi'_m) / n_fine (stream 3), merged with the coarse samples.
 * Training targets: normalised 32-bin histograms of the map's compositing
 * weights (sample depth t in bin b) from a full hierarchical render; uniform
 * when the ray's opacity is below 1e-3.  Loss: mean over rays of
 * sum_b (p_b - h_b)^2; optimiser Adam.
 */
#define LOC_PROPOSAL_PARAMS 11296

/* Camera rays of N particles x B query pixels exactly as loc_update_particles
 * casts them (no prediction step): DEVICE pose N x 12 float64; outputs DEVICE
 * ray_o, ray_d of N*B*3 float32 (ray i*B + j). */
loc_status loc_cast_rays(loc_ctx* ctx, const loc_camera* cam, int inv_R, int B, int N, const double* pose,
                         uint64_t seed, uint64_t iter, float* ray_o, float* ray_d);

/* Training targets for n rays (DEVICE ray_o, ray_d: n*3 float32) from a full
 * render of the context's map with its n_coarse stratified samples and n_fine
 * hierarchical samples (0..256); random streams keyed (ray, 0) with
 * (seed, iter).  hist: DEVICE n*32 float32.  Uses the context's precision. */
loc_status loc_teacher_histograms(loc_ctx* ctx, const float* ray_o, const float* ray_d, int n, int n_fine,
                                  uint64_t seed, uint64_t iter, float* hist);

/* Load (HOST, n == LOC_PROPOSAL_PARAMS) proposal parameters; clears the Adam
 * moments and step.  loc_get_proposal copies them back to HOST memory. */
loc_status loc_set_proposal(loc_ctx* ctx, const float* params, size_t n);
loc_status loc_get_proposal(loc_ctx* ctx, float* params, size_t n);

/* Fine-sample placement used by loc_update_particles: 0 = hierarchical on the
 * coarse weights (default), 1 = learned proposal (needs loc_set_proposal). */
loc_status loc_set_fine_mode(loc_ctx* ctx, int mode);

/* Proposal histograms p (DEVICE n*32) for n rays (DEVICE n*3 each). */
loc_status loc_proposal_forward(loc_ctx* ctx, const float* ray_o, const float* ray_d, int n, float* hist);

/* Mean loss (DEVICE 1 float, may be NULL) and its gradient with respect to
 * the parameters (DEVICE LOC_PROPOSAL_PARAMS floats) over n <= 2^20 rays with
 * targets (DEVICE n*32).  Deterministic: per-wave partial sums reduced in a
 * fixed order. */
loc_status loc_proposal_grad(loc_ctx* ctx, const float* ray_o, const float* ray_d, const float* target, int n,
                             float* loss_out, float* grad_out);

/* Adam training on the GPU: step k uses the `batch` rays starting at
 * (k * batch) mod n (cyclic); the Adam step counter continues across calls
 * until loc_set_proposal.  loss_out: DEVICE `steps` floats (mean batch loss
 * before each step), or NULL. */
typedef struct { int batch, steps; float lr, beta1, beta2, eps; } loc_train_cfg;
loc_status loc_train_proposal(loc_ctx* ctx, const float* ray_o, const float* ray_d, const float* target, int n,
                              const loc_train_cfg* cfg, float* loss_out);

/* --------------------------------------------------------- map training
 * Training of the 4x64 map (no skip input, no direction branch; n_coarse <=
 * 64, n_fine = 0; FP32 or BF16 context) with the photometric loss of Eq. 2,
 * read for a minibatch as the mean over the batch's rays of |C_hat(r) -
 * C(r)|^2, C_hat the coarse render of Eq. 1 as the update computes it
 * (stratified samples of ray r keyed (r, 0) at the call's counter).  The
 * context keeps float32 master weights in the canonical order of
 * loc_map_desc.params and Adam moments; the first training call starts them
 * from the map the context was created with.
 *
 * loc_map_grad: gradient at the current master weights for n rays
 *   ray_o, ray_d DEVICE n x 3 float32 (unit directions), target DEVICE n x 3
 *   float32 colours; grad_out DEVICE 15345 float32 (canonical order);
 *   loss_out DEVICE 1 float32 or NULL.  Per-wave partials summed in a fixed
 *   order (deterministic).  1 <= n <= 2^20.
 * loc_train_map: `steps` Adam steps; step k uses the cfg->batch rays from
 *   (k * batch) mod n (cyclic) at counter (the context's step count, from 0);
 *   loss_out DEVICE `steps` floats (mean batch loss before each step) or
 *   NULL.  Synchronous; afterwards the context renders and localises with the
 *   trained map (repacked for its precision).
 * loc_get_map: the current map (HOST n_params floats, canonical order).
 * LOC_E_UNSUPPORTED for other maps or samplings. */
loc_status loc_map_grad(loc_ctx* ctx, const float* ray_o, const float* ray_d, const float* target, int n,
                        uint64_t seed, uint64_t iter, float* grad_out, float* loss_out);
loc_status loc_train_map(loc_ctx* ctx, const float* ray_o, const float* ray_d, const float* target, int n,
                         const loc_train_cfg* cfg, uint64_t seed, float* loss_out);
loc_status loc_get_map(loc_ctx* ctx, float* params, size_t n);

void loc_destroy(loc_ctx* ctx);
const char* loc_status_str(loc_status s);     /* static text, never NULL */
const char* loc_last_error(const loc_ctx* ctx);/* detail of the last failure; "" if none */

#ifdef __cplusplus
}
#endif
#endif /* FASTLOC_H */
