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

// Lab-frame boxes for the box-tiled kernels.  The resin samples of every ray
// are split into segments, one per lab box they cross; a segment is
// (ray index, first sample k, sample count, rank along the ray).  Samples
// live in the lab frame, so the decomposition does not depend on the angle.
struct BoxGrid {
  double x0, y0, z0;   // lab coordinates of the box grid origin
  int B;               // box edge in voxels
  int nbx, nby, nbz;
};

// Compact records of the lab-box segments (structure of arrays, one entry
// per segment, grouped by box): pw = first sample's lab position relative to
// its box (x, y from the box centre, z from its bottom face) and that
// sample's weight (T1 T2 / n_pupil) step exp(-alpha s); dn = lab direction
// and the sample count (int bits); idx = pixel (deposit order) or
// partial-sum slot rank * n_rays + ray (forward order).  36 bytes per
// segment.
struct SegTable {
  float4* pw = nullptr;
  float4* dn = nullptr;
  int* idx = nullptr;
};

// Per-launch constants of the marching kernels.
struct MarchParams {
  const RayRec* rays;
  const double2* cs;   // (cos, sin) per angle
  int nu, nv, np;
  int a0;
  int sx;              // padded x stride
  int sxy;             // padded slice stride
  double cx, cy;       // centre offsets into padded x, y
  float hix, hiy;      // clip upper bounds: n + 2.5
  float clx, cly, clz; // clamp upper bounds: n + 2.5
  float step;
  float nb;            // -alpha log2(e)
  float r_hi, r_lo;    // exp(-alpha step) split into two floats (hi + lo)
  float r2_hi, r2_lo;  // exp(-2 alpha step), the same way
  int sx4, sxy4;       // padded strides in bytes
  int vol_bytes;       // size of the padded FP32 working volume in bytes
};

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
  double* dose_pad64;            // padded dose accumulator (+ kAccTail words), allocated on first use:
                                 // 64-bit integers (box deposit) or FP64 (ray-driven deposit)
  // optimisation buffers, allocated on first vam_optimize_step
  float* resid;                  // [nz][ny][nx]
  float* grad;                   // [n_angles][n_v][n_u]
  float* dose_tmp;               // [nz][ny][nx]
  double* loss_part;             // per-block partial sums
  int loss_blocks;
  // events around the last forward and dose-deposit kernels (instrumentation)
  hipEvent_t ev[4];
  int ev_valid[2];
  // lab-box segment decomposition
  int box_edge;                  // box edge in voxels (0: library default)
  int seg_order;                 // deposit order of segments inside a box (see sort_segments)
  int seg_order_fwd;             // forward order of segments inside a box
  int deposit_threads;           // workgroup size of the box deposit (256 or 512)
  int xcd_forward, xcd_deposit;  // work order of the box kernels (see work_item)
  vam::BoxGrid boxes;
  int boxes_ready;               // 1 once the decomposition is complete; 0 after a failed rebuild
  int n_boxes;                   // boxes holding at least one segment
  int64_t n_segments;
  vam::SegTable seg_dep;         // segment records, deposit order within a box
  vam::SegTable seg_fwd;         // the same segments in the forward projection's order
  int* ray_nseg;                 // [n_rays] segments per ray
  int max_seg_per_ray;
  float* seg_part;               // forward partial sums [angle][rank][ray], on first use
  int seg_part_angles;           // angles per chunk of seg_part
  // fixed-point forward (variant 2): projections as 64-bit integers
  // [n_angles][n_v][n_u] and the volume's largest |value| (FP32 bits), on
  // first use; the most samples of one pixel (all its rays), set at build
  int64_t* proj_fx;
  unsigned* vol_absmax;
  int64_t pix_samples_max;
  int* box_begin;                // [n_boxes + 1] segment offsets
  int* box_id;                   // [n_boxes] linear box index (x fastest)
  int* box_supp;                 // [n_boxes] most samples of the box in any 4 x 4 x 3 block of lab unit cells
  int64_t supp_bound;            // most samples of all boxes in any such block: <= 8 x max box_supp
  int box_cells;                 // largest rotated-box footprint in cells (LDS)
  // inverse ray map of the voxel-driven gather deposit, built on first use
  vam::BoxGrid cells;            // lab-frame unit cells
  int* cell_begin;               // [cells + 1] entry offsets
  float4* gseg;                  // [n_gseg][2] cell entries
  int64_t n_gseg;
  // statistics
  int64_t rays_hit;
  int64_t samples_per_pass;
  int32_t adjoint_variant;
  int32_t forward_variant;
  int32_t forward_lanes;          // march mode of the fixed-point box forward: 1, 2, 3, or 0 (by format)
};

namespace vam {

// The dose accumulator holds pad_voxels values and then kAccTail more words;
// the first of them keeps the largest |projection value| of a deposit (FP32
// bits) for its integer scale.
constexpr int64_t kAccTail = 32;

// Power-of-two scale of a 64-bit fixed-point sum whose exact value and every
// partial sum are at most bound = |largest value| x coef in magnitude:
// 2^(61 - e) with bound < 2^e, so that each scaled term (an FP32 or FP64
// value times a power of two) is below 2^61 and the sum below 2^62; 1 if
// the bound is 0.
__device__ inline double fx_scale(unsigned max_bits, double coef) {
  const double bound = (double)__uint_as_float(max_bits) * coef;
  if (!(bound > 0.0)) return 1.0;
  int e;
  (void)frexp(bound, &e);
  return ldexp(1.0, 61 - e);
}

vam_status fail(vam_status s, const char* fmt, ...);
void clear_error();
bool valid_handle(const vam_geometry* h);
vam_status hip_check(hipError_t e, const char* what);
// Every device allocation of the library goes through dev_alloc, so that
// vam_debug_fail_allocations can make a chosen one fail.
hipError_t dev_alloc(void** p, size_t bytes);

// projector launches (project.hip)
vam_status launch_forward(vam_geometry* h, const void* vol, vam_dtype vol_t,
                          void* proj, vam_dtype proj_t, int a0, int na,
                          hipStream_t s);
// acc: the padded FP64 accumulator to use (pad_voxels doubles), or NULL for
// the handle's own (allocated on first use)
vam_status launch_back(vam_geometry* h, const void* proj, vam_dtype proj_t,
                       float* dose, int accumulate, int a0, int na,
                       hipStream_t s, double* acc = nullptr);
MarchParams march_params(const vam_geometry* h, int a0);
// lab-box decomposition and the box-tiled operators (boxes.hip); build_boxes
// rebuilds from scratch and leaves boxes_ready = 0 (and nothing allocated)
// on failure
vam_status build_boxes(vam_geometry* h, hipStream_t s);
vam_status launch_box_forward(vam_geometry* h, const MarchParams& P, void* proj, vam_dtype proj_t, vam_dtype vol_t,
                              int na, hipStream_t s);
// the box forward's padded working volume from a BF16 or FP16 volume
void pad_box_volume(vam_geometry* h, const void* vol, vam_dtype vol_t, hipStream_t s);
// acc: pad_voxels + kAccTail words, cleared (pad_voxels + 1 of them) by the
// caller; the box deposit leaves the dose there as 64-bit integers at the
// scale fx_scale(acc[pad_voxels] bits, deposit_coef(h, na))
vam_status launch_box_deposit(vam_geometry* h, const MarchParams& P, const void* proj, vam_dtype proj_t,
                              int na, double* acc, hipStream_t s);
double deposit_coef(const vam_geometry* h, int na);
void free_boxes(vam_geometry* h);
bool supported_box_edge(int B);
// voxel-driven gather deposit through the inverse ray map (gather.hip);
// prepare_gather builds the map on first use (synchronises the stream)
vam_status prepare_gather(vam_geometry* h, hipStream_t s);
vam_status launch_gather_deposit(vam_geometry* h, const void* proj, vam_dtype proj_t, float* dose,
                                 int accumulate, int a0, int na, hipStream_t s);
void free_gather(vam_geometry* h);

}  // namespace vam

#define VAM_HIP_TRY(expr, what)                                   \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return ::vam::hip_check(e_, what);      \
  } while (0)
