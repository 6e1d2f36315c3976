// Vector kernels of the Lanczos estimate of lam_Nd, the largest eigenvalue of H that
// Alg. 1 takes as the top of the filter interval (the paper leaves its computation
// open; the library's reading is a k-step Lanczos run from a caller-given vector).
//
// One Lanczos step on the device:  w = H v_j (hx_apply with no Chebyshev terms), then
//   lanczos_dot:   w -= beta_{j-1} v_{j-1};  partial sums of v_j . w
//   lanczos_norm:  w -= alpha_j v_j;          partial sums of w . w
//   lanczos_scale: v_{j+1} = w / beta_j
// and sum_partials reduces the per-block sums.  Every reduction has a fixed grid and a
// fixed order (grid-stride partial per thread, LDS tree per block, one block over the
// block sums), so results are bitwise reproducible.  Orbital vectors are stored in the
// handle's precision (TV), w and all sums in FP64.
#include "common.h"

namespace chefsi {

namespace {

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int off = kVecThreads / 2; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  return red[0];
}

template <typename TV>
__global__ __launch_bounds__(kVecThreads) void lanczos_dot_kernel(double* __restrict__ w, const TV* __restrict__ v,
                                                                  const TV* __restrict__ vp, double beta,
                                                                  int64_t n, double* __restrict__ partial) {
  __shared__ double red[kVecThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    double wi = w[i];
    if (vp != nullptr) {
      wi -= beta * double(vp[i]);
      w[i] = wi;
    }
    acc += double(v[i]) * wi;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename TV>
__global__ __launch_bounds__(kVecThreads) void lanczos_norm_kernel(double* __restrict__ w, const TV* __restrict__ v,
                                                                   double alpha, int64_t n,
                                                                   double* __restrict__ partial) {
  __shared__ double red[kVecThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
    double wi = w[i];
    if (v != nullptr) {
      wi -= alpha * double(v[i]);
      w[i] = wi;
    }
    acc += wi * wi;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename TV>
__global__ __launch_bounds__(kVecThreads) void lanczos_scale_kernel(const double* __restrict__ w, double inv,
                                                                    int64_t n, TV* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
    out[i] = TV(w[i] * inv);
}

template <typename TV>
__global__ __launch_bounds__(kVecThreads) void widen_kernel(const TV* __restrict__ x, int64_t n,
                                                            double* __restrict__ w) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
    w[i] = double(x[i]);
}

__global__ __launch_bounds__(kVecThreads) void sum_blocks_kernel(const double* __restrict__ partial, int nparts,
                                                                 double* __restrict__ out) {
  __shared__ double red[kVecThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kVecThreads) acc += partial[i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

template <typename TV>
hipError_t launch_lanczos_dot(double* w, const TV* v, const TV* vp, double beta, int64_t n, double* partial,
                              double* out, hipStream_t s) {
  hipLaunchKernelGGL((lanczos_dot_kernel<TV>), dim3(kVecBlocks), dim3(kVecThreads), 0, s, w, v, vp, beta, n, partial);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(kVecThreads), 0, s, partial, kVecBlocks, out);
  return hipGetLastError();
}

template <typename TV>
hipError_t launch_lanczos_norm(double* w, const TV* v, double alpha, int64_t n, double* partial, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL((lanczos_norm_kernel<TV>), dim3(kVecBlocks), dim3(kVecThreads), 0, s, w, v, alpha, n, partial);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(kVecThreads), 0, s, partial, kVecBlocks, out);
  return hipGetLastError();
}

template <typename TV>
hipError_t launch_lanczos_scale(const double* w, double inv, int64_t n, TV* out, hipStream_t s) {
  hipLaunchKernelGGL((lanczos_scale_kernel<TV>), dim3(kVecBlocks), dim3(kVecThreads), 0, s, w, inv, n, out);
  return hipGetLastError();
}

template <typename TV>
hipError_t launch_widen(const TV* x, int64_t n, double* w, hipStream_t s) {
  hipLaunchKernelGGL((widen_kernel<TV>), dim3(kVecBlocks), dim3(kVecThreads), 0, s, x, n, w);
  return hipGetLastError();
}

template hipError_t launch_lanczos_dot<double>(double*, const double*, const double*, double, int64_t, double*,
                                               double*, hipStream_t);
template hipError_t launch_lanczos_dot<float>(double*, const float*, const float*, double, int64_t, double*,
                                              double*, hipStream_t);
template hipError_t launch_lanczos_norm<double>(double*, const double*, double, int64_t, double*, double*,
                                                hipStream_t);
template hipError_t launch_lanczos_norm<float>(double*, const float*, double, int64_t, double*, double*,
                                               hipStream_t);
template hipError_t launch_lanczos_scale<double>(const double*, double, int64_t, double*, hipStream_t);
template hipError_t launch_lanczos_scale<float>(const double*, double, int64_t, float*, hipStream_t);
template hipError_t launch_widen<double>(const double*, int64_t, double*, hipStream_t);
template hipError_t launch_widen<float>(const float*, int64_t, double*, hipStream_t);

}  // namespace chefsi
