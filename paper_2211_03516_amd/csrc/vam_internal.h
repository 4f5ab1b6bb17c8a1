// Internal declarations shared by the libvam translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "vam.h"

namespace vam {

constexpr uint64_t kMagic = 0x56414d4745304d31ull;  // "VAMGE0M1"
constexpr int kPad = 2;            // zero voxels on each side of the working grids
constexpr int kRay64Fields = 12;   // exported FP64 record, see vam_export_rays

// Resin segment of one ray, ready for marching.  The midpoint m is the centre
// of the sample set (e + K step / 2 d), so the sample positions are
// m + t_k d with t_k = (k + 1/2 - K/2) step, short lever arms on both sides.
// Lab-frame x, y of m and d are kept in FP64 because they are rotated for
// every angle; z does not rotate and is stored already shifted into padded
// grid coordinates.  64 bytes, one per (pupil j, pixel row v, pixel u).
struct alignas(16) RayRec {
  double mx, my;     // lab-frame midpoint, x and y
  double dx, dy;     // lab-frame unit direction in the resin, x and y
  float gz;          // midpoint z in padded grid coordinates
  float dz;          // direction z
  float cw;          // (T1 T2 / n_pupil) * step * exp(-alpha * K step / 2)
  float t0;          // t of the first sample inside the padded z range
  int32_t n;         // samples in the padded z range (0 if the ray misses)
  int32_t k0;        // index of that first sample in 0..K-1
  int32_t K;         // samples on the whole resin chord
  int32_t pad_;
};
static_assert(sizeof(RayRec) == 64, "RayRec layout");

}  // namespace vam

struct vam_geometry {
  uint64_t magic;
  vam_geometry_desc desc;
  std::vector<double> angles;    // radians
  std::vector<double> pupil;     // [n_pupil][2]
  int device;
  int64_t n_rays;
  int px, py, pz;                // padded grid sizes (n + 2 kPad)
  int64_t pad_voxels;
  // device memory owned by the handle
  vam::RayRec* rays;             // [n_pupil][n_v][n_u]
  double* ray64;                 // [n_rays][kRay64Fields]
  double2* angle_cs;             // [n_angles] (cos, sin)
  float* vol_pad;                // padded FP32 working volume (forward input)
  float* dose_pad;               // padded FP32 dose accumulator (adjoint)
  // optimisation buffers, allocated on first vam_optimize_step
  float* resid;                  // [nz][ny][nx]
  float* grad;                   // [n_angles][n_v][n_u]
  float* dose_tmp;               // [nz][ny][nx]
  double* loss_part;             // per-block partial sums
  int loss_blocks;
  // events around the last forward and dose-deposit kernels (instrumentation)
  hipEvent_t ev[4];
  int ev_valid[2];
  // statistics
  int64_t rays_hit;
  int64_t samples_per_pass;
  int32_t adjoint_variant;
};

namespace vam {

vam_status fail(vam_status s, const char* fmt, ...);
void clear_error();
bool valid_handle(const vam_geometry* h);
vam_status hip_check(hipError_t e, const char* what);

// projector launches (project.hip)
vam_status launch_forward(vam_geometry* h, const void* vol, vam_dtype vol_t,
                          void* proj, vam_dtype proj_t, int a0, int na,
                          hipStream_t s);
vam_status launch_back(vam_geometry* h, const void* proj, vam_dtype proj_t,
                       float* dose, int accumulate, int a0, int na,
                       hipStream_t s);

}  // namespace vam

#define VAM_HIP_TRY(expr, what)                                   \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return ::vam::hip_check(e_, what);      \
  } while (0)
