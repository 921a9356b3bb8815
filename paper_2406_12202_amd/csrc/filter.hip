// Per-step particle-filter kernels in float64: prediction, weight
// normalisation, integer-exact systematic resampling, the gather of resampled
// poses and the pose read-out (device functions in filter_dev.h).
#include <mutex>

#include "filter_dev.h"

namespace fl {

// one wave per workgroup: the float64 prediction is arithmetic-bound, so
// small workgroups spread a few hundred particles over as many CUs
__global__ __launch_bounds__(64) void k_predict(const PredictArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  predict_pose(a.pose_in + (long)i * 12, a.pose_out + (long)i * 12, a.motion.m, a.sigma_t, a.sigma_r, a.seed,
               a.iter, i);
}

hipError_t launch_predict(const PredictArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_predict, dim3((a.N + 63) / 64), dim3(64), 0, st, a);
  return hipGetLastError();
}

// a set that fits is read once into LDS, so the passes over it do not wait
// on memory (the arithmetic is the same either way)
__global__ __launch_bounds__(kRedThreads) void k_normalize(const double* ll, double* w, int N, int* flags) {
  __shared__ double s[kRedThreads / 64];
  __shared__ double s_l[kPrefixLds], s_w[kPrefixLds];
  if (N <= kPrefixLds) {
    for (int i = threadIdx.x; i < N; i += kRedThreads) s_l[i] = ll[i];
    __syncthreads();
    normalize_block(s_l, s_w, N, flags, s);
    for (int i = threadIdx.x; i < N; i += kRedThreads) w[i] = s_w[i];
  } else {
    normalize_block(ll, w, N, flags, s);
  }
}

hipError_t launch_normalize(const double* loglik, double* weight, int N, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize, dim3(1), dim3(kRedThreads), 0, st, loglik, weight, N, flags);
  return hipGetLastError();
}

__global__ __launch_bounds__(kRedThreads) void k_resample(const double* weight, int n_in, int n_out,
                                                          uint64_t seed, uint64_t iter, u64* prefix,
                                                          int32_t* idx, int* flags) {
  __shared__ double s_max[kRedThreads / 64];
  __shared__ u64 s_sum[kRedThreads / 64];
  __shared__ u64 s_prefix[kPrefixLds];
  __shared__ double s_w[kPrefixLds];
  if (n_in <= kPrefixLds) {
    for (int i = threadIdx.x; i < n_in; i += kRedThreads) s_w[i] = weight[i];
    __syncthreads();
    resample_block(s_w, n_in, n_out, seed, iter, prefix, idx, flags, s_max, s_sum, s_prefix);
  } else {
    resample_block(weight, n_in, n_out, seed, iter, prefix, idx, flags, s_max, s_sum, s_prefix);
  }
}

hipError_t launch_resample(const double* weight, int n_in, int n_out, uint64_t seed, uint64_t iter,
                           u64* prefix, int32_t* idx, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_resample, dim3(1), dim3(kRedThreads), 0, st, weight, n_in, n_out, seed, iter,
                     prefix, idx, flags);
  return hipGetLastError();
}

// Scratch of the allocation-free resampling call: the inclusive prefix of the
// integer weights, kNoAllocMaxWeights entries (8 MiB).  Each GPU the library
// runs on holds its own copy from module load to process end; every call on
// that GPU shares it, so calls that overlap in time on one GPU race.  Every
// entry the kernel reads is written earlier in the same launch (the prefix
// of all n_in weights precedes the searches), so nothing needs clearing.
static __device__ __align__(256) u64 scratch[kNoAllocMaxWeights];

// Device address of this GPU's scratch, looked up once per device with that
// device current (host code never passes the array's own name to a kernel:
// on the host that name is a stand-in, not a device address).
hipError_t noalloc_scratch(int device, u64** out) {
  static std::mutex mu;
  static u64* ptr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    ptr[device] = static_cast<u64*>(p);
  }
  *out = ptr[device];
  return hipSuccess;
}

// out[k] = in[idx[k]] (idx < 0 copies nothing)
__global__ void k_gather_poses(const double* in, const int32_t* idx, int n_in, int n_out, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out * 12) return;
  const int k = t / 12, q = t - k * 12;
  const int i = idx[k];
  if (i >= 0 && i < n_in) out[t] = in[(long)i * 12 + q];
}

hipError_t launch_gather_poses(const double* in, const int32_t* idx, int n_in, int n_out, double* out,
                               hipStream_t st) {
  const int n = n_out * 12;
  hipLaunchKernelGGL(k_gather_poses, dim3((n + 255) / 256), dim3(256), 0, st, in, idx, n_in, n_out, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kEstThreads) void k_pose_estimate(const double* pose, const double* w, int N,
                                                               double* est, int* flags) {
  __shared__ double s[kEstThreads][13];
  pose_estimate_block(pose, w, N, est, flags, s);
}

hipError_t launch_pose_estimate(const double* pose, const double* w, int N, double* est, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_estimate, dim3(1), dim3(kEstThreads), 0, st, pose, w, N, est, flags);
  return hipGetLastError();
}

__global__ __launch_bounds__(kEstThreads) void k_position_variance(const double* pose, const double* w, int N,
                                                                   double* var) {
  __shared__ double s[kEstThreads][4];
  position_variance_block(pose, w, N, var, s);
}

hipError_t launch_position_variance(const double* pose, const double* w, int N, double* var, hipStream_t st) {
  hipLaunchKernelGGL(k_position_variance, dim3(1), dim3(kEstThreads), 0, st, pose, w, N, var);
  return hipGetLastError();
}

}  // namespace fl
