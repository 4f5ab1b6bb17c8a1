// One gradient step of projection optimisation.
//
// The paper optimises its projections with an iterative feedback method
// whose update rule it does not print (Sec. 2.7), terminating on the dose
// error.  Here the same loop is a projected gradient step on a smooth
// dose-threshold loss, built only from the projector pair:
//   d = A^T g                      (dose of the current projections)
//   sig = 1 / (1 + exp(-kappa (d - thr)))
//   loss = mean_v (sig_v - target_v)^2       (reduced in FP64)
//   r = (2/N) (sig - target) sig (1 - sig) kappa
//   grad = A r                     (the transpose of the transpose)
//   g <- max(0, g - lr grad)
// The loss partials are reduced per block and then summed in block order,
// so the FP64 loss is deterministic for a given dose.

#include "vam_internal.h"

namespace vam {

constexpr int kLossThreads = 256;
constexpr int kLossBlocks = 2048;

__global__ __launch_bounds__(kLossThreads) void k_loss_resid(const float* __restrict__ dose,
                                                             const float* __restrict__ target,
                                                             float* __restrict__ resid, int64_t n,
                                                             float thr, float kappa,
                                                             double* __restrict__ part) {
  __shared__ double red[kLossThreads / 64];
  double local = 0.0;
  const float two_over_n = (float)(2.0 / (double)n);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float sig = 1.0f / (1.0f + __expf(-kappa * (dose[i] - thr)));
    const float diff = sig - target[i];
    local += (double)diff * (double)diff;
    resid[i] = two_over_n * diff * sig * (1.0f - sig) * kappa;
  }
  for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kLossThreads / 64; ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

__global__ void k_loss_final(const double* __restrict__ part, int nparts, int64_t n,
                             double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    *out = s / (double)n;
  }
}

__global__ void k_update(float* __restrict__ g, const float* __restrict__ grad, int64_t n, float lr,
                         int clamp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x = g[i] - lr * grad[i];
  g[i] = clamp ? fmaxf(x, 0.0f) : x;
}

}  // namespace vam

using namespace vam;

extern "C" vam_status vam_optimize_step(vam_geometry_t h, const float* target, float* proj, float* dose,
                                        const vam_opt_params* prm, double* loss_out,
                                        hipStream_t stream) {
  clear_error();
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  if (!target || !proj || !prm) return fail(VAM_ERR_INVALID_ARG, "NULL argument");
  if (!(prm->sharpness > 0) || !(prm->lr >= 0) || !std::isfinite(prm->threshold) ||
      !std::isfinite(prm->sharpness) || !std::isfinite(prm->lr))
    return fail(VAM_ERR_INVALID_ARG, "optimisation parameters need sharpness > 0, lr >= 0, finite");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  const vam_geometry_desc& D = h->desc;
  const int64_t nvox = (int64_t)D.nx * D.ny * D.nz;
  const int64_t nproj = (int64_t)D.n_angles * D.n_v * D.n_u;
  if (!h->resid) {
    VAM_HIP_TRY(hipMalloc(&h->resid, nvox * sizeof(float)), "allocating the residual");
    VAM_HIP_TRY(hipMalloc(&h->grad, nproj * sizeof(float)), "allocating the gradient");
    VAM_HIP_TRY(hipMalloc(&h->dose_tmp, nvox * sizeof(float)), "allocating the dose");
    VAM_HIP_TRY(hipMalloc(&h->loss_part, (kLossBlocks + 1) * sizeof(double)), "allocating loss partials");
    h->loss_blocks = kLossBlocks;
  }
  float* d = dose ? dose : h->dose_tmp;
  vam_status st = launch_back(h, proj, VAM_F32, d, 0, 0, D.n_angles, stream);
  if (st != VAM_OK) return st;
  int blocks = (int)std::min<int64_t>(kLossBlocks, (nvox + kLossThreads - 1) / kLossThreads);
  hipLaunchKernelGGL(k_loss_resid, dim3(blocks), dim3(kLossThreads), 0, stream, d, target, h->resid, nvox,
                     (float)prm->threshold, (float)prm->sharpness, h->loss_part);
  VAM_HIP_TRY(hipGetLastError(), "launching the loss");
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, stream, h->loss_part, blocks, nvox,
                     h->loss_part + kLossBlocks);
  VAM_HIP_TRY(hipGetLastError(), "launching the loss reduction");
  st = launch_forward(h, h->resid, VAM_F32, h->grad, VAM_F32, 0, D.n_angles, stream);
  if (st != VAM_OK) return st;
  hipLaunchKernelGGL(k_update, dim3((unsigned)((nproj + 255) / 256)), dim3(256), 0, stream, proj, h->grad,
                     nproj, (float)prm->lr, prm->clamp_nonneg);
  VAM_HIP_TRY(hipGetLastError(), "launching the update");
  if (loss_out) {
    VAM_HIP_TRY(hipMemcpyAsync(loss_out, h->loss_part + kLossBlocks, sizeof(double), hipMemcpyDeviceToHost,
                               stream), "copying the loss");
    VAM_HIP_TRY(hipStreamSynchronize(stream), "synchronising the loss");
  }
  return VAM_OK;
}
