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
// The projections g may be stored in FP32, BF16 or FP16: the deposit reads
// them as stored, the gradient is FP32, and the update is formed in FP32 and
// rounded to nearest even on store.  The loss partials are reduced per block
// and then summed in block order, so the FP64 loss is deterministic for a
// given dose.

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

__device__ inline float ld(const float* p, int64_t i) { return p[i]; }
__device__ inline float ld(const uint16_t* p, int64_t i) { return __uint_as_float((uint32_t)p[i] << 16); }
__device__ inline float ld(const __half* p, int64_t i) { return __half2float(p[i]); }
__device__ inline void st(float* p, int64_t i, float x) { p[i] = x; }
__device__ inline void st(uint16_t* p, int64_t i, float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    p[i] = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);       // round to nearest even
    p[i] = (uint16_t)(u >> 16);
  }
}
__device__ inline void st(__half* p, int64_t i, float x) { p[i] = __float2half_rn(x); }

template <typename PT>
__global__ void k_update(PT* __restrict__ g, const float* __restrict__ grad, int64_t n, float lr, int clamp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = ld(g, i) - lr * grad[i];
  st(g, i, clamp ? fmaxf(x, 0.0f) : x);
}

// The step's buffers, allocated together on the first call: either all
// four are in the handle or none is.
static vam_status optimize_buffers(vam_geometry* h, int64_t nvox, int64_t nproj) {
  if (h->resid) return VAM_OK;
  float *resid = nullptr, *grad = nullptr, *dose = nullptr;
  double* part = nullptr;
  hipError_t e = dev_alloc((void**)&resid, nvox * sizeof(float));
  if (e == hipSuccess) e = dev_alloc((void**)&grad, nproj * sizeof(float));
  if (e == hipSuccess) e = dev_alloc((void**)&dose, nvox * sizeof(float));
  if (e == hipSuccess) e = dev_alloc((void**)&part, (kLossBlocks + 1) * sizeof(double));
  if (e != hipSuccess) {
    void* ptrs[] = {resid, grad, dose, part};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    return hip_check(e, "allocating the optimisation buffers");
  }
  h->resid = resid;
  h->grad = grad;
  h->dose_tmp = dose;
  h->loss_part = part;
  h->loss_blocks = kLossBlocks;
  return VAM_OK;
}

}  // namespace vam

using namespace vam;

extern "C" vam_status vam_optimize_step(vam_geometry_t h, const float* target, void* proj, vam_dtype proj_t,
                                        float* dose, const vam_opt_params* prm, double* loss_out,
                                        hipStream_t stream) {
  clear_error();
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  if (!target || !proj || !prm) return fail(VAM_ERR_INVALID_ARG, "NULL argument");
  if (proj_t != VAM_F32 && proj_t != VAM_BF16 && proj_t != VAM_F16)
    return fail(VAM_ERR_INVALID_ARG, "unknown projection dtype %d", (int)proj_t);
  if (!(prm->sharpness > 0) || !(prm->lr >= 0) || !std::isfinite(prm->threshold) ||
      !std::isfinite(prm->sharpness) || !std::isfinite(prm->lr))
    return fail(VAM_ERR_INVALID_ARG, "optimisation parameters need sharpness > 0, lr >= 0, finite");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  const vam_geometry_desc& D = h->desc;
  const int64_t nvox = (int64_t)D.nx * D.ny * D.nz;
  const int64_t nproj = (int64_t)D.n_angles * D.n_v * D.n_u;
  vam_status st = optimize_buffers(h, nvox, nproj);
  if (st != VAM_OK) return st;
  float* d = dose ? dose : h->dose_tmp;
  st = launch_back(h, proj, proj_t, d, 0, 0, D.n_angles, stream);
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
  const dim3 grid((unsigned)((nproj + 255) / 256));
  switch (proj_t) {
    case VAM_F32:
      hipLaunchKernelGGL(k_update<float>, grid, dim3(256), 0, stream, (float*)proj, h->grad, nproj, (float)prm->lr,
                         prm->clamp_nonneg);
      break;
    case VAM_BF16:
      hipLaunchKernelGGL(k_update<uint16_t>, grid, dim3(256), 0, stream, (uint16_t*)proj, h->grad, nproj,
                         (float)prm->lr, prm->clamp_nonneg);
      break;
    case VAM_F16:
      hipLaunchKernelGGL(k_update<__half>, grid, dim3(256), 0, stream, (__half*)proj, h->grad, nproj,
                         (float)prm->lr, prm->clamp_nonneg);
      break;
  }
  VAM_HIP_TRY(hipGetLastError(), "launching the update");
  if (loss_out) {
    VAM_HIP_TRY(hipMemcpyAsync(loss_out, h->loss_part + kLossBlocks, sizeof(double), hipMemcpyDeviceToHost,
                               stream), "copying the loss");
    VAM_HIP_TRY(hipStreamSynchronize(stream), "synchronising the loss");
  }
  return VAM_OK;
}
