// Plain initialisation and optimisation metrics.
//
// Ram-Lak filtering: the paper's Radon baseline filters each parallel-beam
// sinogram with a Ram-Lak filter and clips negative values (Sec. 2.3).  Here
// the filter is applied along u as the exact spatial-domain convolution with
// the band-limited ramp kernel sampled at the pixel pitch (Ramachandran and
// Lakshminarayanan; see Kak and Slaney, "Principles of Computerized
// Tomographic Imaging", ch. 3):
//   h[0] = 1 / (4 tau^2),  h[n] = 0 for even n != 0,
//   h[n] = -1 / (n^2 pi^2 tau^2) for odd n,
// scaled by tau so that a unit-pitch discrete convolution approximates the
// continuous filter, followed by clipping at zero.
//
// Export: see k_eq_map below.
//
// Dose error: the termination test of Sec. 2.7 compares simulated and target
// dose; here E = ||sigmoid(kappa (d - thr)) - t||_1 / ||t||_1 together with
// the fraction of voxels whose thresholded dose (d >= thr) differs from the
// binary target, both reduced in FP64.

#include <cmath>

#include "vam_internal.h"

namespace vam {

constexpr int kRowTile = 256;

// One block per projection row; the row is staged in LDS and each thread
// convolves outputs u = threadIdx.x, threadIdx.x + blockDim.x, ...
__global__ __launch_bounds__(kRowTile) void k_ramlak(const float* __restrict__ in, float* __restrict__ out, int nu,
                                                     float tau, int clip) {
  extern __shared__ float row[];  // [nu] row values, then [nu / 2] odd-tap weights
  float* hodd = row + nu;
  const int64_t base = (int64_t)blockIdx.x * nu;
  for (int u = threadIdx.x; u < nu; u += blockDim.x) row[u] = in[base + u];
  for (int m = threadIdx.x; 2 * m + 1 < nu; m += blockDim.x) {
    const float n = (float)(2 * m + 1);
    hodd[m] = -1.0f / ((float)(M_PI * M_PI) * n * n);
  }
  __syncthreads();
  for (int u = threadIdx.x; u < nu; u += blockDim.x) {
    float acc = 0.25f * row[u];
    for (int n = 1; n < nu; n += 2) {
      const float hn = hodd[n >> 1];
      float s = 0.0f;
      if (u - n >= 0) s += row[u - n];
      if (u + n < nu) s += row[u + n];
      acc = fmaf(hn, s, acc);
    }
    acc /= tau;
    out[base + u] = clip ? fmaxf(acc, 0.0f) : acc;
  }
}

constexpr int kErrThreads = 256;
constexpr int kErrBlocks = 1024;

__global__ __launch_bounds__(kErrThreads) void k_dose_error(const float* __restrict__ dose,
                                                            const float* __restrict__ target, int64_t n, float thr,
                                                            float kappa, double* __restrict__ part) {
  __shared__ double red[3][kErrThreads / 64];
  double l1 = 0.0, tsum = 0.0, wrong = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = dose[i], t = target[i];
    const double sig = 1.0 / (1.0 + exp(-(double)kappa * (d - thr)));
    l1 += fabs(sig - t);
    tsum += fabs(t);
    wrong += ((d >= thr) != (t >= 0.5)) ? 1.0 : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    l1 += __shfl_down(l1, off, 64);
    tsum += __shfl_down(tsum, off, 64);
    wrong += __shfl_down(wrong, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = l1;
    red[1][threadIdx.x >> 6] = tsum;
    red[2][threadIdx.x >> 6] = wrong;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int w = 0; w < kErrThreads / 64; ++w) s += red[threadIdx.x][w];
    part[3 * blockIdx.x + threadIdx.x] = s;
  }
}

__global__ void k_dose_error_final(const double* __restrict__ part, int nblocks, int64_t n, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double l1 = 0.0, tsum = 0.0, wrong = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      l1 += part[3 * b];
      tsum += part[3 * b + 1];
      wrong += part[3 * b + 2];
    }
    out[0] = tsum > 0.0 ? l1 / tsum : 0.0;
    out[1] = wrong / (double)n;
  }
}

// Projection export (Sec. 2.7): values above mean + 3 std over all pixels of
// all angles are clipped, then the range [0, clip] is rescaled to 8 bits.
// Statistics in FP64; the scaled value v = x * (255 / clip) is formed in FP64
// and rounded to nearest even.
constexpr int kEqThreads = 256;
constexpr int kEqBlocks = 1024;

__global__ __launch_bounds__(kEqThreads) void k_eq_stats(const float* __restrict__ p, int64_t n,
                                                         double* __restrict__ part) {
  __shared__ double red[2][kEqThreads / 64];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = p[i];
    s1 += x;
    s2 += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, 64);
    s2 += __shfl_down(s2, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s1;
    red[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int w = 0; w < kEqThreads / 64; ++w) s += red[threadIdx.x][w];
    part[2 * blockIdx.x + threadIdx.x] = s;
  }
}

// stats[0] mean, stats[1] population std, stats[2] clip = mean + 3 std
__global__ void k_eq_final(const double* __restrict__ part, int nblocks, int64_t n, double* __restrict__ stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      s1 += part[2 * b];
      s2 += part[2 * b + 1];
    }
    const double mean = s1 / (double)n;
    const double var = fmax(s2 / (double)n - mean * mean, 0.0);
    const double sd = sqrt(var);
    stats[0] = mean;
    stats[1] = sd;
    stats[2] = mean + 3.0 * sd;
  }
}

__global__ void k_eq_map(const float* __restrict__ p, int64_t n, const double* __restrict__ stats,
                         uint8_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double clip = stats[2];
  double v = 0.0;
  if (clip > 0.0) {
    const double x = fmin(fmax((double)p[i], 0.0), clip);
    v = rint(x * (255.0 / clip));
  }
  out[i] = (uint8_t)fmin(fmax(v, 0.0), 255.0);
}

}  // namespace vam

using namespace vam;

extern "C" {

vam_status vam_ramlak_filter(const float* proj_in, float* proj_out, int32_t n_rows, int32_t n_u, double pitch,
                             int32_t clip_negative, hipStream_t stream) {
  clear_error();
  if (!proj_in || !proj_out) return fail(VAM_ERR_INVALID_ARG, "NULL buffer");
  if (n_rows < 0 || n_u < 1 || n_u > 8192) return fail(VAM_ERR_INVALID_ARG, "bad sizes %d x %d", n_rows, n_u);
  if (!(pitch > 0) || !std::isfinite(pitch)) return fail(VAM_ERR_INVALID_ARG, "pitch must be finite and > 0");
  if (proj_in == proj_out) return fail(VAM_ERR_INVALID_ARG, "in-place filtering is not supported");
  if (n_rows == 0) return VAM_OK;
  hipLaunchKernelGGL(k_ramlak, dim3(n_rows), dim3(kRowTile), (n_u + n_u / 2 + 1) * sizeof(float), stream, proj_in,
                     proj_out, n_u,
                     (float)pitch, clip_negative);
  VAM_HIP_TRY(hipGetLastError(), "launching the Ram-Lak filter");
  return VAM_OK;
}

vam_status vam_dose_error(const float* dose, const float* target, int64_t n, double threshold, double sharpness,
                          double* out2, hipStream_t stream) {
  clear_error();
  if (!dose || !target || !out2) return fail(VAM_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return fail(VAM_ERR_INVALID_ARG, "n must be >= 1");
  if (!(sharpness > 0) || !std::isfinite(sharpness) || !std::isfinite(threshold))
    return fail(VAM_ERR_INVALID_ARG, "sharpness must be finite and > 0");
  double* part = nullptr;
  const int blocks = (int)std::min<int64_t>(kErrBlocks, (n + kErrThreads - 1) / kErrThreads);
  VAM_HIP_TRY(hipMallocAsync((void**)&part, (3 * blocks + 2) * sizeof(double), stream), "allocating partials");
  hipLaunchKernelGGL(k_dose_error, dim3(blocks), dim3(kErrThreads), 0, stream, dose, target, n, (float)threshold,
                     (float)sharpness, part);
  hipLaunchKernelGGL(k_dose_error_final, dim3(1), dim3(64), 0, stream, part, blocks, n, part + 3 * blocks);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(out2, part + 3 * blocks, 2 * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFreeAsync(part, stream);
  if (e != hipSuccess) return hip_check(e, "dose error");
  return VAM_OK;
}

vam_status vam_equalize_u8(const float* proj, int64_t n, uint8_t* out, double* stats3, hipStream_t stream) {
  clear_error();
  if (!proj || !out) return fail(VAM_ERR_INVALID_ARG, "NULL buffer");
  if (n < 1) return fail(VAM_ERR_INVALID_ARG, "n must be >= 1");
  double* part = nullptr;
  const int blocks = (int)std::min<int64_t>(kEqBlocks, (n + kEqThreads - 1) / kEqThreads);
  VAM_HIP_TRY(hipMallocAsync((void**)&part, (2 * blocks + 3) * sizeof(double), stream), "allocating partials");
  double* st = part + 2 * blocks;
  hipLaunchKernelGGL(k_eq_stats, dim3(blocks), dim3(kEqThreads), 0, stream, proj, n, part);
  hipLaunchKernelGGL(k_eq_final, dim3(1), dim3(64), 0, stream, part, blocks, n, st);
  hipLaunchKernelGGL(k_eq_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, proj, n, st, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && stats3) e = hipMemcpyAsync(stats3, st, 3 * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && stats3) e = hipStreamSynchronize(stream);
  (void)hipFreeAsync(part, stream);
  if (e != hipSuccess) return hip_check(e, "equalisation");
  return VAM_OK;
}

}  // extern "C"
