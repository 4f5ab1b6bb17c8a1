// Ray-driven reference kernels of the projector pair on gfx950: forward
// projection (Sec. 2.4 of Webber et al., with the transmission factors of
// Sec. 2.5) and its exact transpose, the dose deposit (Sec. 2.5), with one
// lane per DMD pixel and angle; and the dispatch of both operators to the
// box-tiled default kernels (boxes.hip), these references, or the
// voxel-driven gather deposit (gather.hip).
//
// Work decomposition of the references.  The lane marches the n_pupil rays
// of its pixel one after the other (finite etendue, Sec. 2.4/2.5) and sums
// them in registers, so a wave writes 64 consecutive projection values of
// one row (coalesced).  Lanes of a wave are 64 neighbouring pixels of one
// row: at a given step their samples sit side by side in the volume.
//
// Sampling.  The ray table keeps each resin segment as its midpoint and
// direction (lab frame).  Per angle the midpoint and direction are rotated
// into the volume frame in FP64 and rounded once; sample k is then at
// g = m + t_k d with t_k = (k + 1/2 - K/2) step, one FMA per axis, short
// lever arms and no accumulated drift.  Anti-aliasing weights (Sec. 2.2)
// are the trilinear tent over the 8 surrounding voxel centres.
//
// Bounds.  The working volumes carry two zero voxels of padding per side.
// Per ray and angle the sample range is clipped to padded coordinates
// [0.5, n + 2.5] (the stencil touches the grid only in (1, n + 2)), and every
// position is also clamped into [0, n + 2.5] before indexing, so all eight
// corners stay inside the padded array whatever the rounding.

#include <cmath>
#include <mutex>

#include "vam_internal.h"

namespace vam {



// --------------------------------------------------------- element access --

__device__ inline float load_elem(const float* p, int64_t i) { return p[i]; }
__device__ inline float load_elem(const uint16_t* p, int64_t i) {
  return __uint_as_float((uint32_t)p[i] << 16);
}
__device__ inline float load_elem(const __half* p, int64_t i) { return __half2float(p[i]); }

__device__ inline void store_elem(float* p, int64_t i, float x) { p[i] = x; }
__device__ inline void store_elem(uint16_t* p, int64_t i, float x) {
  uint32_t u = __float_as_uint(x);
  uint16_t b;
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    b = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    b = (uint16_t)(u >> 16);
  }
  p[i] = b;
}
__device__ inline void store_elem(__half* p, int64_t i, float x) { p[i] = __float2half_rn(x); }

// ------------------------------------------------------- per-ray set-up ----

struct Seg {
  float gx, gy, gz;   // midpoint, padded grid coordinates (volume frame)
  float dx, dy, dz;   // direction (volume frame)
  float t0;           // t of sample k0 of the z-clipped range
  float cw;
  int k0, k1;         // samples [k0, k1) relative to t0
};

__device__ inline void clip_axis(float g, float d, float lo, float hi, float& tlo, float& thi) {
  if (fabsf(d) > 1e-20f) {
    float inv = 1.0f / d;
    float ta = (lo - g) * inv, tb = (hi - g) * inv;
    tlo = fmaxf(tlo, fminf(ta, tb));
    thi = fminf(thi, fmaxf(ta, tb));
  } else if (!(g >= lo && g <= hi)) {
    thi = -INFINITY;
  }
}

// Rotate ray r into the volume frame of angle (c, s) and clip its sample
// range to the padded grid.  Returns false when nothing is left.
__device__ inline bool segment(const MarchParams& P, const RayRec& R, double c, double s, Seg& g) {
  if (R.n <= 0) return false;
  g.gx = (float)(c * R.mx + s * R.my + P.cx);
  g.gy = (float)(-s * R.mx + c * R.my + P.cy);
  g.gz = R.gz;
  g.dx = (float)(c * R.dx + s * R.dy);
  g.dy = (float)(-s * R.dx + c * R.dy);
  g.dz = R.dz;
  g.t0 = R.t0;
  g.cw = R.cw;
  float tlo = R.t0;
  float thi = R.t0 + (float)(R.n - 1) * P.step;
  clip_axis(g.gx, g.dx, 0.5f, P.hix, tlo, thi);
  clip_axis(g.gy, g.dy, 0.5f, P.hiy, tlo, thi);
  if (!(thi >= tlo)) return false;
  // one spare sample on each side is harmless: it reads or writes padding
  int k0 = (int)floorf((tlo - R.t0) / P.step);
  int k1 = (int)ceilf((thi - R.t0) / P.step) + 1;
  g.k0 = max(k0, 0);
  g.k1 = min(k1, R.n);
  return g.k1 > g.k0;
}

// ---------------------------------------------------- tuned kernels (v2) --
//
// Same lanes, samples and weights as above, with cheaper per-sample work:
//  * the padded working arrays are addressed through buffer resources, so a
//    sample needs one 32-bit byte offset and the corner rows come from
//    uniform (scalar) offsets instead of 64-bit address arithmetic; the two
//    x-neighbours of a corner row are one 8-byte load;
//  * positions are non-negative after the clamp, so truncation is the floor
//    and v_fract gives the offset;
//  * the attenuation of consecutive samples is a geometric sequence with
//    ratio r = exp(-alpha step).  The forward sum is evaluated by Horner's
//    rule from the far end, S <- S r + val, and the deposit keeps
//    e <- e r; r is applied as r_hi + r_lo (two FMAs), so the rounding of r
//    itself does not accumulate along the ray.  One exp2 per ray segment.

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

__device__ inline float2 ld_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  auto a = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(a[0]), __uint_as_float(a[1]));
}

// Byte offset of the base voxel of a sample and its fractional offsets.
__device__ inline int cell4(const MarchParams& P, const Seg& g, float t, float& fx, float& fy, float& fz) {
  const float x = __builtin_amdgcn_fmed3f(fmaf(t, g.dx, g.gx), 0.0f, P.clx);
  const float y = __builtin_amdgcn_fmed3f(fmaf(t, g.dy, g.gy), 0.0f, P.cly);
  const float z = __builtin_amdgcn_fmed3f(fmaf(t, g.dz, g.gz), 0.0f, P.clz);
  fx = __builtin_amdgcn_fractf(x);
  fy = __builtin_amdgcn_fractf(y);
  fz = __builtin_amdgcn_fractf(z);
  const unsigned ix = (unsigned)x, iy = (unsigned)y, iz = (unsigned)z;
  return (int)(__umul24(iz, (unsigned)P.sxy4) + __umul24(iy, (unsigned)P.sx4) + (ix << 2));
}

template <typename PT>
__global__ __launch_bounds__(256) void k_forward2(MarchParams P, const float* __restrict__ vol,
                                                  PT* __restrict__ proj) {
  const int u = blockIdx.x * 64 + threadIdx.x;
  const int v = blockIdx.y * 4 + threadIdx.y;
  const int a = blockIdx.z;
  if (u >= P.nu || v >= P.nv) return;
  const __amdgpu_buffer_rsrc_t R4 = rsrc(vol, P.vol_bytes);
  const double2 cs = P.cs[P.a0 + a];
  const int64_t plane = (int64_t)P.nv * P.nu;
  const int o1 = P.sx4, o2 = P.sxy4, o3 = P.sxy4 + P.sx4;
  float acc = 0.0f;
  for (int j = 0; j < P.np; ++j) {
    const RayRec R = P.rays[j * plane + (int64_t)v * P.nu + u];
    Seg g;
    if (!segment(P, R, cs.x, cs.y, g)) continue;
    float S = 0.0f;
    float kf = (float)(g.k1 - 1);
    for (int k = g.k1 - 1; k >= g.k0; --k, kf -= 1.0f) {
      const float t = fmaf(kf, P.step, g.t0);
      float fx, fy, fz;
      const int off = cell4(P, g, t, fx, fy, fz);
      const float2 a0 = ld_pair(R4, off, 0);
      const float2 a1 = ld_pair(R4, off, o1);
      const float2 a2 = ld_pair(R4, off, o2);
      const float2 a3 = ld_pair(R4, off, o3);
      const float c00 = fmaf(fx, a0.y - a0.x, a0.x);
      const float c01 = fmaf(fx, a1.y - a1.x, a1.x);
      const float c10 = fmaf(fx, a2.y - a2.x, a2.x);
      const float c11 = fmaf(fx, a3.y - a3.x, a3.x);
      const float c0 = fmaf(fy, c01 - c00, c00);
      const float c1 = fmaf(fy, c11 - c10, c10);
      const float val = fmaf(fz, c1 - c0, c0);
      S = fmaf(S, P.r_hi, fmaf(S, P.r_lo, val));
    }
    const float t_first = fmaf((float)g.k0, P.step, g.t0);
    acc = fmaf(g.cw * __builtin_amdgcn_exp2f(P.nb * t_first), S, acc);
  }
  store_elem(proj, ((int64_t)a * P.nv + v) * P.nu + u, acc);
}

// Deposit with FP64 global atomics into the padded accumulator, aggregating
// consecutive samples that share a cell (FP32 atomics would bias the sum by
// ~1e-5 at ~1e5 deposits per voxel).
__device__ inline void flush8(double* dose, int off, const MarchParams& P, const double* w) {
  double* d = dose + (off >> 2);
  unsafeAtomicAdd(d, w[0]);
  unsafeAtomicAdd(d + 1, w[1]);
  unsafeAtomicAdd(d + P.sx, w[2]);
  unsafeAtomicAdd(d + P.sx + 1, w[3]);
  unsafeAtomicAdd(d + P.sxy, w[4]);
  unsafeAtomicAdd(d + P.sxy + 1, w[5]);
  unsafeAtomicAdd(d + P.sxy + P.sx, w[6]);
  unsafeAtomicAdd(d + P.sxy + P.sx + 1, w[7]);
}

template <typename PT>
__global__ __launch_bounds__(256) void k_back2(MarchParams P, const PT* __restrict__ proj,
                                               double* __restrict__ dose) {
  const int u = blockIdx.x * 64 + threadIdx.x;
  const int v = blockIdx.y * 4 + threadIdx.y;
  const int a = blockIdx.z;
  if (u >= P.nu || v >= P.nv) return;
  const float pv = load_elem(proj, ((int64_t)a * P.nv + v) * P.nu + u);
  if (pv == 0.0f) return;
  const double2 cs = P.cs[P.a0 + a];
  const int64_t plane = (int64_t)P.nv * P.nu;
  for (int j = 0; j < P.np; ++j) {
    const RayRec R = P.rays[j * plane + (int64_t)v * P.nu + u];
    Seg g;
    if (!segment(P, R, cs.x, cs.y, g)) continue;
    float kf = (float)g.k0;
    float e = g.cw * pv * __builtin_amdgcn_exp2f(P.nb * fmaf(kf, P.step, g.t0));
    int cur = -1;
    double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = g.k0; k < g.k1; ++k, kf += 1.0f) {
      const float t = fmaf(kf, P.step, g.t0);
      float fx, fy, fz;
      const int off = cell4(P, g, t, fx, fy, fz);
      const float z1 = e * fz, z0 = e - z1;
      const float y01 = z0 * fy, y00 = z0 - y01;
      const float y11 = z1 * fy, y10 = z1 - y11;
      const float q[8] = {y00 - y00 * fx, y00 * fx, y01 - y01 * fx, y01 * fx,
                          y10 - y10 * fx, y10 * fx, y11 - y11 * fx, y11 * fx};
      if (off != cur) {
        if (cur >= 0) flush8(dose, cur, P, w);
        cur = off;
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] = q[c];
      } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] += q[c];
      }
      e = fmaf(e, P.r_hi, e * P.r_lo);
    }
    if (cur >= 0) flush8(dose, cur, P, w);
  }
}

// Caller volume -> the padded FP32 working volume, padding included (zero),
// so that no earlier call's contents (16-bit pairs of the box forward) stay
// behind in it.
template <typename VT>
__global__ void k_pad(const VT* __restrict__ vol, float* __restrict__ vp, int nx, int ny, int nz, int px, int py,
                      int pz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)px * py * pz) return;
  const int x = (int)(i % px) - kPad, y = (int)((i / px) % py) - kPad, z = (int)(i / ((int64_t)px * py)) - kPad;
  float v = 0.0f;
  if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) v = load_elem(vol, ((int64_t)z * ny + y) * nx + x);
  vp[i] = v;
}

// Interior of the padded accumulator -> caller dose (overwrite or add).
template <typename AT>
__global__ void k_unpad(const AT* __restrict__ dp, float* __restrict__ dose, int accumulate,
                        int nx, int ny, int nz, int px, int py) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nx * ny * nz;
  if (i >= n) return;
  const int x = (int)(i % nx);
  const int y = (int)((i / nx) % ny);
  const int z = (int)(i / ((int64_t)nx * ny));
  const AT d = dp[((int64_t)(z + kPad) * py + (y + kPad)) * px + (x + kPad)];
  dose[i] = accumulate ? (float)(dose[i] + d) : (float)d;
}

// The box deposit's integer dose -> caller dose: the integer over the scale,
// plus the caller's dose if accumulating; NaN everywhere if a projection
// value was a NaN or an infinity.
__global__ void k_unpad_fx(const unsigned long long* __restrict__ acc, float* __restrict__ dose, int accumulate,
                           int nx, int ny, int nz, int px, int py, const unsigned* __restrict__ pmax, double coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nx * ny * nz;
  if (i >= n) return;
  const int x = (int)(i % nx);
  const int y = (int)((i / nx) % ny);
  const int z = (int)(i / ((int64_t)nx * ny));
  const unsigned pm = *pmax;
  const long long q = (long long)acc[((int64_t)(z + kPad) * py + (y + kPad)) * px + (x + kPad)];
  const double d = pm < 0x7f800000u ? (double)q / fx_scale(pm, coef) : __builtin_nan("");
  dose[i] = accumulate ? (float)(dose[i] + d) : (float)d;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

MarchParams march_params(const vam_geometry* h, int a0) {
  const vam_geometry_desc& D = h->desc;
  MarchParams P;
  P.rays = h->rays;
  P.cs = h->angle_cs;
  P.nu = D.n_u;
  P.nv = D.n_v;
  P.np = D.n_pupil;
  P.a0 = a0;
  P.sx = h->px;
  P.sxy = h->px * h->py;
  P.cx = 0.5 * (D.nx - 1) + kPad;
  P.cy = 0.5 * (D.ny - 1) + kPad;
  P.hix = (float)D.nx + 2.5f;
  P.hiy = (float)D.ny + 2.5f;
  P.clx = (float)D.nx + 2.5f;
  P.cly = (float)D.ny + 2.5f;
  P.clz = (float)D.nz + 2.5f;
  P.step = (float)D.step;
  P.nb = (float)(-D.alpha / std::log(2.0));
  const double r = std::exp(-D.alpha * D.step);
  P.r_hi = (float)r;
  P.r_lo = (float)(r - (double)P.r_hi);
  const double r2 = std::exp(-2.0 * D.alpha * D.step);
  P.r2_hi = (float)r2;
  P.r2_lo = (float)(r2 - (double)P.r2_hi);
  P.sx4 = 4 * P.sx;
  P.sxy4 = 4 * P.sxy;
  P.vol_bytes = (int)std::min<int64_t>(h->pad_voxels * 4, 0x7fffffff);
  return P;
}

// The ray-driven references address the padded arrays with 32-bit byte
// offsets and 24-bit multiplies.
static bool v2_eligible(const vam_geometry* h) {
  return h->pad_voxels * 8 < 0x7fffffffLL && (int64_t)h->px * h->py * 4 < (1 << 24);
}

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

vam_status launch_forward(vam_geometry* h, const void* vol, vam_dtype vol_t, void* proj,
                          vam_dtype proj_t, int a0, int na, hipStream_t s) {
  const vam_geometry_desc& D = h->desc;
  if (h->forward_variant == 1 && !v2_eligible(h))
    return fail(VAM_ERR_UNSUPPORTED, "the ray-driven forward needs a padded volume below 2^28 voxels");
  const unsigned vb = blocks_for(h->pad_voxels, 256);
  // the box forward stages a BF16 / FP16 volume as 16-bit pairs
  const bool pairs = h->forward_variant != 1 && vol_t != VAM_F32;
  if (pairs) pad_box_volume(h, vol, vol_t, s);
  else switch (vol_t) {
    case VAM_F32:
      hipLaunchKernelGGL(k_pad<float>, dim3(vb), dim3(256), 0, s, (const float*)vol, h->vol_pad,
                         D.nx, D.ny, D.nz, h->px, h->py, h->pz);
      break;
    case VAM_BF16:
      hipLaunchKernelGGL(k_pad<uint16_t>, dim3(vb), dim3(256), 0, s, (const uint16_t*)vol, h->vol_pad,
                         D.nx, D.ny, D.nz, h->px, h->py, h->pz);
      break;
    case VAM_F16:
      hipLaunchKernelGGL(k_pad<__half>, dim3(vb), dim3(256), 0, s, (const __half*)vol, h->vol_pad,
                         D.nx, D.ny, D.nz, h->px, h->py, h->pz);
      break;
  }
  VAM_HIP_TRY(hipGetLastError(), "launching the volume copy");
  MarchParams P = march_params(h, a0);
  VAM_HIP_TRY(hipEventRecord(h->ev[0], s), "recording an event");
  if (h->forward_variant != 1) {
    vam_status st = launch_box_forward(h, P, proj, proj_t, vol_t, na, s);
    if (st != VAM_OK) return st;
  } else {
    dim3 grid((D.n_u + 63) / 64, (D.n_v + 3) / 4, na), block(64, 4);
    switch (proj_t) {
      case VAM_F32: hipLaunchKernelGGL(k_forward2<float>, grid, block, 0, s, P, h->vol_pad, (float*)proj); break;
      case VAM_BF16:
        hipLaunchKernelGGL(k_forward2<uint16_t>, grid, block, 0, s, P, h->vol_pad, (uint16_t*)proj);
        break;
      case VAM_F16: hipLaunchKernelGGL(k_forward2<__half>, grid, block, 0, s, P, h->vol_pad, (__half*)proj); break;
    }
    VAM_HIP_TRY(hipGetLastError(), "launching the forward projector");
  }
  VAM_HIP_TRY(hipEventRecord(h->ev[1], s), "recording an event");
  h->ev_valid[0] = 1;
  return VAM_OK;
}

vam_status launch_back(vam_geometry* h, const void* proj, vam_dtype proj_t, float* dose, int accumulate,
                       int a0, int na, hipStream_t s, double* acc) {
  const vam_geometry_desc& D = h->desc;
  const int variant = h->adjoint_variant;
  if (variant == 2) {
    // voxel-driven gather: writes (or adds to) the output directly
    vam_status st = prepare_gather(h, s);
    if (st != VAM_OK) return st;
    VAM_HIP_TRY(hipEventRecord(h->ev[2], s), "recording an event");
    st = launch_gather_deposit(h, proj, proj_t, dose, accumulate, a0, na, s);
    if (st != VAM_OK) return st;
    VAM_HIP_TRY(hipEventRecord(h->ev[3], s), "recording an event");
    h->ev_valid[1] = 1;
    return VAM_OK;
  }
  if (variant == 1 && !v2_eligible(h))
    return fail(VAM_ERR_UNSUPPORTED, "the ray-driven deposit needs a padded volume below 2^28 voxels");
  if (!h->boxes_ready && variant == 0)
    return fail(VAM_ERR_INVALID_ARG, "the box decomposition is not available (a rebuild failed); "
                                     "set the box edge again or create a new geometry");
  if (!acc) {
    if (!h->dose_pad64)
      VAM_HIP_TRY(dev_alloc((void**)&h->dose_pad64, (h->pad_voxels + kAccTail) * sizeof(double)),
                  "allocating the dose accumulator");
    acc = h->dose_pad64;
  }
  // cleared by a kernel (no memset node when the caller captures a graph):
  // the dose words and the projection maximum after them (all-zero bits are
  // 0 both as FP64 and as integers)
  hipLaunchKernelGGL(k_fill<double>, dim3(blocks_for(h->pad_voxels + 1, 256)), dim3(256), 0, s, acc,
                     h->pad_voxels + 1, 0.0);
  VAM_HIP_TRY(hipGetLastError(), "launching the accumulator clear");
  MarchParams P = march_params(h, a0);
  VAM_HIP_TRY(hipEventRecord(h->ev[2], s), "recording an event");
  if (variant == 0) {
    vam_status st = launch_box_deposit(h, P, proj, proj_t, na, acc, s);
    if (st != VAM_OK) return st;
  } else {
    dim3 grid((D.n_u + 63) / 64, (D.n_v + 3) / 4, na), block(64, 4);
    switch (proj_t) {
      case VAM_F32:
        hipLaunchKernelGGL(k_back2<float>, grid, block, 0, s, P, (const float*)proj, acc);
        break;
      case VAM_BF16:
        hipLaunchKernelGGL(k_back2<uint16_t>, grid, block, 0, s, P, (const uint16_t*)proj, acc);
        break;
      case VAM_F16:
        hipLaunchKernelGGL(k_back2<__half>, grid, block, 0, s, P, (const __half*)proj, acc);
        break;
    }
  }
  VAM_HIP_TRY(hipGetLastError(), "launching the dose deposit");
  VAM_HIP_TRY(hipEventRecord(h->ev[3], s), "recording an event");
  h->ev_valid[1] = 1;
  const int64_t nvox = (int64_t)D.nx * D.ny * D.nz;
  if (variant == 0)
    hipLaunchKernelGGL(k_unpad_fx, dim3(blocks_for(nvox, 256)), dim3(256), 0, s, (const unsigned long long*)acc, dose,
                       accumulate, D.nx, D.ny, D.nz, h->px, h->py, (const unsigned*)(acc + h->pad_voxels),
                       deposit_coef(h, na));
  else
    hipLaunchKernelGGL(k_unpad<double>, dim3(blocks_for(nvox, 256)), dim3(256), 0, s, acc, dose, accumulate,
                       D.nx, D.ny, D.nz, h->px, h->py);
  VAM_HIP_TRY(hipGetLastError(), "launching the dose copy");
  return VAM_OK;
}

// ------------------------------------------------ allocation-free deposit --
//
// vam_back_project_noalloc takes the deposit's padded accumulator (and the
// kAccTail words after it) from this file-scope device array instead of
// allocating it.  Each device that
// loads the library holds its own copy until the process ends; its device
// address is looked up once per device (with that device current) and kept
// in scratch_dev, which is what host code passes to the kernels.
constexpr int64_t kScratchDoubles = 17825792;  // 136 MiB: padded grids up to 261^3 + kAccTail (volumes up to 257^3)
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static double* scratch_dev[kMaxDevices];
static std::mutex scratch_mutex;

static vam_status scratch_for(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(VAM_ERR_UNSUPPORTED, "device index %d >= %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "looking up the scratch array");
    scratch_dev[device] = (double*)p;
  }
  *out = scratch_dev[device];
  return VAM_OK;
}

static vam_status check_common(vam_geometry* h, const void* a, const void* b, int dt, int a0, int na) {
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  if (!a || !b) return fail(VAM_ERR_INVALID_ARG, "NULL buffer");
  if (dt != VAM_F32 && dt != VAM_BF16 && dt != VAM_F16) return fail(VAM_ERR_INVALID_ARG, "unknown dtype %d", dt);
  if (na < 1 || a0 < 0 || (int64_t)a0 + na > h->desc.n_angles)
    return fail(VAM_ERR_INVALID_ARG, "angle range [%d, %d) outside [0, %d)", a0, a0 + na, h->desc.n_angles);
  return VAM_OK;
}

}  // namespace vam

using namespace vam;

extern "C" {

vam_status vam_forward_project(vam_geometry_t h, const void* vol, vam_dtype vol_t, void* proj,
                               vam_dtype proj_t, int32_t angle_begin, int32_t angle_count,
                               hipStream_t stream) {
  clear_error();
  vam_status st = check_common(h, vol, proj, vol_t, angle_begin, angle_count);
  if (st != VAM_OK) return st;
  if (proj_t != VAM_F32 && proj_t != VAM_BF16 && proj_t != VAM_F16)
    return fail(VAM_ERR_INVALID_ARG, "unknown projection dtype %d", (int)proj_t);
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  return launch_forward(h, vol, vol_t, proj, proj_t, angle_begin, angle_count, stream);
}

vam_status vam_back_project(vam_geometry_t h, const void* proj, vam_dtype proj_t, float* dose,
                            int32_t accumulate, int32_t angle_begin, int32_t angle_count,
                            hipStream_t stream) {
  clear_error();
  vam_status st = check_common(h, proj, dose, proj_t, angle_begin, angle_count);
  if (st != VAM_OK) return st;
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  return launch_back(h, proj, proj_t, dose, accumulate, angle_begin, angle_count, stream);
}

vam_status vam_back_project_noalloc(vam_geometry_t h, const void* proj, vam_dtype proj_t, float* dose,
                                    int32_t accumulate, int32_t angle_begin, int32_t angle_count,
                                    hipStream_t stream) {
  clear_error();
  vam_status st = check_common(h, proj, dose, proj_t, angle_begin, angle_count);
  if (st != VAM_OK) return st;
  if (h->pad_voxels + kAccTail > kScratchDoubles)
    return fail(VAM_ERR_UNSUPPORTED,
                "allocation-free deposit: the padded grid (%d x %d x %d = %lld voxels) exceeds the %lld-voxel "
                "scratch array (volumes up to 257^3)",
                h->px, h->py, h->pz, (long long)h->pad_voxels, (long long)(kScratchDoubles - kAccTail));
  if (h->adjoint_variant == 2)
    return fail(VAM_ERR_UNSUPPORTED, "allocation-free deposit: the gather variant builds an inverse ray map");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  double* acc = nullptr;
  st = scratch_for(h->device, &acc);
  if (st != VAM_OK) return st;
  return launch_back(h, proj, proj_t, dose, accumulate, angle_begin, angle_count, stream, acc);
}

vam_status vam_kernel_times(vam_geometry_t h, float* forward_ms, float* back_ms) {
  clear_error();
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  if (forward_ms) {
    *forward_ms = -1.0f;
    if (h->ev_valid[0]) VAM_HIP_TRY(hipEventElapsedTime(forward_ms, h->ev[0], h->ev[1]), "reading events");
  }
  if (back_ms) {
    *back_ms = -1.0f;
    if (h->ev_valid[1]) VAM_HIP_TRY(hipEventElapsedTime(back_ms, h->ev[2], h->ev[3]), "reading events");
  }
  return VAM_OK;
}

}  // extern "C"
