// Voxel-driven gather form of the dose deposit (the transpose of the forward
// projection of Sec. 2.5, computed per voxel instead of per ray sample).
//
// Each voxel owns its dose and sums, for every angle, the contributions of
// the ray samples inside its trilinear support: no atomics, and a fixed
// summation order.  Finding those samples needs an inverse ray map.  The
// vial turns about +z, so sample positions are fixed in the lab frame: the
// map bins every resin sample run into the lab-frame unit cell it lies in
// (an entry per maximal run of consecutive samples of a ray in one cell,
// holding the first sample's position inside the cell, the step vector, the
// attenuated ray weight and the pixel).  For a voxel at angle theta the
// support is the voxel's unit cube turned by theta about z; the kernel visits
// the lab cells under its bounding box (three or four per axis in x and y,
// two in z) and evaluates the tent weight of every sample there.
//
// Work: each sample is visited once per voxel whose support box covers its
// cell, i.e. ~8 (x the bounding-box excess) times more sample visits than
// the scatter, each without atomics.  The library measures both forms and
// keeps the scatter as the default.

#include <algorithm>
#include <cmath>
#include <vector>

#include "vam_internal.h"

namespace vam {

struct CellGrid {
  double x0, y0;      // lab coordinates of cell (0, 0); cell iz covers padded z [iz, iz + 1)
  int ncx, ncy, ncz;
};

// Position of sample k of a ray: the marching kernels' definition, from the
// FP64 midpoint and direction of the ray record.
struct SamplePos {
  double x, y, z, t;
};
__device__ inline SamplePos sample_pos(const RayRec& R, int k, double step) {
  SamplePos p;
  p.t = ((double)k + 0.5 - 0.5 * (double)R.K) * step;
  p.x = R.mx + p.t * R.dx;
  p.y = R.my + p.t * R.dy;
  p.z = (double)R.gz + p.t * (double)R.dz;
  return p;
}

__device__ inline int cell_of(const CellGrid& C, const SamplePos& p) {
  const int ix = min(max((int)floor(p.x - C.x0), 0), C.ncx - 1);
  const int iy = min(max((int)floor(p.y - C.y0), 0), C.ncy - 1);
  const int iz = min(max((int)floor(p.z), 0), C.ncz - 1);
  return (iz * C.ncy + iy) * C.ncx + ix;
}

// Call emit(cell, first k, count) once per maximal run of samples of the
// ray in one cell, split so that no run is longer than 7 samples (a unit
// cell holds at most 4 samples at steps of 0.5 voxel or more).
template <class F>
__device__ inline void walk_cells(const CellGrid& C, const RayRec& R, double step, F emit) {
  if (R.n <= 0) return;
  int cur = -1, start = 0;
  for (int k = R.k0; k < R.k0 + R.n; ++k) {
    const int c = cell_of(C, sample_pos(R, k, step));
    if (c != cur || k - start == 7) {
      if (cur >= 0) emit(cur, start, k - start);
      cur = c;
      start = k;
    }
  }
  if (cur >= 0) emit(cur, start, R.k0 + R.n - start);
}

__global__ void k_cell_count(CellGrid C, const RayRec* rays, int64_t n_rays, double step, int* count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  walk_cells(C, rays[r], step, [&](int c, int, int) { atomicAdd(count + c, 1); });
}

__global__ void k_cell_fill(CellGrid C, const RayRec* rays, int64_t n_rays, double step, const int* begin,
                            int* cursor, int4* ent) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  walk_cells(C, rays[r], step, [&](int c, int k, int n) {
    ent[begin[c] + atomicAdd(cursor + c, 1)] = make_int4((int)r, k, n, c);
  });
}

// Order the entries of each cell by (ray, first sample): the fill kernel's
// order depends on scheduling, the gather's summation order must not.
__global__ void k_cell_sort(const int* begin, int ncell, int4* ent) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int b = begin[c], e = begin[c + 1];
  for (int i = b + 1; i < e; ++i) {
    const int4 v = ent[i];
    int j = i - 1;
    while (j >= b && (ent[j].x > v.x || (ent[j].x == v.x && ent[j].y > v.y))) {
      ent[j + 1] = ent[j];
      --j;
    }
    ent[j + 1] = v;
  }
}

// Entry i -> two float4: (x, y, z of the first sample relative to the
// cell's lower corner, its attenuated weight c_k) and (step vector, pixel
// index * 8 + sample count as raw bits).
__global__ void k_cell_build(CellGrid C, const RayRec* rays, const int4* ent, int64_t n, double step,
                             double alpha, int npix, float4* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 en = ent[i];
  const RayRec R = rays[en.x];
  const SamplePos p = sample_pos(R, en.y, step);
  const int c = en.w;
  const int ix = c % C.ncx, iy = (c / C.ncx) % C.ncy, iz = c / (C.ncx * C.ncy);
  const double w = (double)R.cw * exp(-alpha * p.t);
  out[2 * i] = make_float4((float)(p.x - (C.x0 + ix)), (float)(p.y - (C.y0 + iy)), (float)(p.z - iz), (float)w);
  const unsigned bits = ((unsigned)(en.x % npix) << 3) | (unsigned)en.z;
  out[2 * i + 1] = make_float4((float)(step * R.dx), (float)(step * R.dy), (float)(step * (double)R.dz),
                               __uint_as_float(bits));
}

void free_gather(vam_geometry* h) {
  if (h->cell_begin) (void)hipFree(h->cell_begin);
  if (h->gseg) (void)hipFree(h->gseg);
  h->cell_begin = nullptr;
  h->gseg = nullptr;
  h->n_gseg = 0;
}

static CellGrid cell_grid(const vam_geometry* h) {
  const double R = h->desc.r_inner + 1.0;
  CellGrid C;
  C.x0 = -R;
  C.y0 = -R;
  C.ncx = (int)std::ceil(2.0 * R);
  C.ncy = C.ncx;
  C.ncz = h->pz;
  return C;
}

// Build the inverse ray map (synchronises the stream).
static vam_status build_gather(vam_geometry* h, hipStream_t s) {
  const vam_geometry_desc& D = h->desc;
  const int64_t npix = (int64_t)D.n_u * D.n_v;
  if (npix >= (1 << 29)) return fail(VAM_ERR_UNSUPPORTED, "gather deposit: more than 2^29 pixels");
  const CellGrid C = cell_grid(h);
  const int64_t ncell = (int64_t)C.ncx * C.ncy * C.ncz;
  if (ncell >= 0x7fffffffLL) return fail(VAM_ERR_UNSUPPORTED, "gather deposit: more than 2^31 cells");
  int* count = nullptr;
  int4* ent = nullptr;
  auto release = [&]() {
    if (count) (void)hipFree(count);
    if (ent) (void)hipFree(ent);
  };
  const int threads = 256;
  const unsigned rblocks = (unsigned)((h->n_rays + threads - 1) / threads);
  hipError_t e = dev_alloc((void**)&count, ncell * sizeof(int));
  if (e == hipSuccess) e = dev_alloc((void**)&h->cell_begin, (ncell + 1) * sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(count, 0, ncell * sizeof(int), s);
  if (e != hipSuccess) {
    release();
    free_gather(h);
    return hip_check(e, "allocating the inverse ray map");
  }
  hipLaunchKernelGGL(k_cell_count, dim3(rblocks), dim3(threads), 0, s, C, h->rays, h->n_rays, D.step, count);
  std::vector<int> hc(ncell);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), count, ncell * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release();
    free_gather(h);
    return hip_check(e, "counting inverse-map entries");
  }
  std::vector<int> hb(ncell + 1);
  int64_t total = 0;
  for (int64_t c = 0; c < ncell; ++c) {
    hb[c] = (int)std::min<int64_t>(total, 0x7fffffff);
    total += hc[c];
  }
  hb[ncell] = (int)std::min<int64_t>(total, 0x7fffffff);
  if (total >= 0x7fffffffLL) {
    release();
    free_gather(h);
    return fail(VAM_ERR_UNSUPPORTED, "gather deposit: more than 2^31 inverse-map entries");
  }
  e = dev_alloc((void**)&ent, std::max<int64_t>(total, 1) * sizeof(int4));
  if (e == hipSuccess) e = dev_alloc((void**)&h->gseg, std::max<int64_t>(total, 1) * 2 * sizeof(float4));
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->cell_begin, hb.data(), (ncell + 1) * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(count, 0, ncell * sizeof(int), s);
  if (e != hipSuccess) {
    release();
    free_gather(h);
    return hip_check(e, "allocating inverse-map entries");
  }
  hipLaunchKernelGGL(k_cell_fill, dim3(rblocks), dim3(threads), 0, s, C, h->rays, h->n_rays, D.step,
                     h->cell_begin, count, ent);
  hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)((ncell + threads - 1) / threads)), dim3(threads), 0, s,
                     h->cell_begin, (int)ncell, ent);
  if (total > 0)
    hipLaunchKernelGGL(k_cell_build, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, C,
                       h->rays, ent, total, D.step, D.alpha, (int)npix, h->gseg);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) {
    free_gather(h);
    return hip_check(e, "building the inverse ray map");
  }
  h->cells.x0 = C.x0;
  h->cells.y0 = C.y0;
  h->cells.z0 = 0.0;
  h->cells.B = 1;
  h->cells.nbx = C.ncx;
  h->cells.nby = C.ncy;
  h->cells.nbz = C.ncz;
  h->n_gseg = total;
  return VAM_OK;
}

struct GatherParams {
  const float4* seg;
  const int* begin;
  const double2* cs;
  CellGrid C;
  int nx, ny, nz;
  int a0, na, npix;
  float r_hi, r_lo;   // exp(-alpha step) as hi + lo
  double rmax2;       // voxels farther than this (squared) from the axis get no dose
};

template <typename PT>
__device__ inline float gload(const PT* p, int64_t i);
template <>
__device__ inline float gload<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ inline float gload<uint16_t>(const uint16_t* p, int64_t i) { return __uint_as_float((uint32_t)p[i] << 16); }
template <>
__device__ inline float gload<__half>(const __half* p, int64_t i) { return __half2float(p[i]); }

__device__ inline float tent(float d) { return fmaxf(0.0f, 1.0f - fabsf(d)); }

// One thread per voxel, 16 x 16 voxels of one z slice per workgroup; the
// voxel's dose over the launch's angles is summed per angle in FP32 and
// across angles in FP64, then written (or added) once.
template <typename PT>
__global__ __launch_bounds__(256) void k_back_gather(GatherParams Q, const PT* __restrict__ proj,
                                                     float* __restrict__ dose, int accumulate) {
  const int x = blockIdx.x * 16 + (threadIdx.x & 15);
  const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int z = blockIdx.z;
  if (x >= Q.nx || y >= Q.ny) return;
  const int64_t vi = ((int64_t)z * Q.ny + y) * Q.nx + x;
  const double vx = x - 0.5 * (Q.nx - 1), vy = y - 0.5 * (Q.ny - 1);
  const int zp = z + kPad;
  double total = 0.0;
  if (vx * vx + vy * vy <= Q.rmax2) {
    for (int a = 0; a < Q.na; ++a) {
      const double2 cs = Q.cs[Q.a0 + a];
      // the voxel centre in the lab frame, relative to the cell grid origin
      const double qx = cs.x * vx - cs.y * vy - Q.C.x0;
      const double qy = cs.y * vx + cs.x * vy - Q.C.y0;
      const double hw = fabs(cs.x) + fabs(cs.y);  // half-width of the turned support's bounding box
      const int ix0 = max((int)floor(qx - hw), 0), ix1 = min((int)floor(qx + hw), Q.C.ncx - 1);
      const int iy0 = max((int)floor(qy - hw), 0), iy1 = min((int)floor(qy + hw), Q.C.ncy - 1);
      const float fx = (float)(qx - ix0), fy = (float)(qy - iy0);
      const float c = (float)cs.x, s = (float)cs.y;
      const PT* pa = proj + (int64_t)a * Q.npix;  // the caller's projections start at angle a0
      float acc = 0.0f;
      for (int iz = max(zp - 1, 0); iz <= min(zp, Q.C.ncz - 1); ++iz) {
        const float oz = (float)(iz - zp);
        for (int iy = iy0; iy <= iy1; ++iy) {
          const float oy = (float)(iy - iy0) - fy;
          const int row = (iz * Q.C.ncy + iy) * Q.C.ncx;
          for (int ix = ix0; ix <= ix1; ++ix) {
            const float ox = (float)(ix - ix0) - fx;
            const int e1 = Q.begin[row + ix + 1];
            for (int e = Q.begin[row + ix]; e < e1; ++e) {
              const float4 A = Q.seg[2 * (int64_t)e];
              const float4 S = Q.seg[2 * (int64_t)e + 1];
              // first sample relative to the voxel centre: lab offset, then
              // turned into the volume frame (p_vol = R_z(-theta) p_lab)
              const float lx = ox + A.x, ly = oy + A.y;
              float dx = c * lx + s * ly, dy = c * ly - s * lx, dz = oz + A.z;
              const float sx = c * S.x + s * S.y, sy = c * S.y - s * S.x, sz = S.z;
              const unsigned bits = __float_as_uint(S.w);
              const int cnt = (int)(bits & 7u);
              float wsum = 0.0f, att = 1.0f;
              for (int j = 0; j < cnt; ++j) {
                wsum = fmaf(att, tent(dx) * tent(dy) * tent(dz), wsum);
                att = fmaf(att, Q.r_hi, att * Q.r_lo);
                dx += sx;
                dy += sy;
                dz += sz;
              }
              if (wsum != 0.0f) acc = fmaf(A.w * wsum, gload(pa, (int64_t)(bits >> 3)), acc);
            }
          }
        }
      }
      total += (double)acc;
    }
  }
  dose[vi] = accumulate ? (float)((double)dose[vi] + total) : (float)total;
}

vam_status prepare_gather(vam_geometry* h, hipStream_t s) { return h->gseg ? VAM_OK : build_gather(h, s); }

vam_status launch_gather_deposit(vam_geometry* h, const void* proj, vam_dtype proj_t, float* dose, int accumulate,
                                 int a0, int na, hipStream_t s) {
  if (!h->gseg) return fail(VAM_ERR_INVALID_ARG, "gather deposit: inverse ray map not built");
  const vam_geometry_desc& D = h->desc;
  GatherParams Q;
  Q.seg = h->gseg;
  Q.begin = h->cell_begin;
  Q.cs = h->angle_cs;
  Q.C.x0 = h->cells.x0;
  Q.C.y0 = h->cells.y0;
  Q.C.ncx = h->cells.nbx;
  Q.C.ncy = h->cells.nby;
  Q.C.ncz = h->cells.nbz;
  Q.nx = D.nx;
  Q.ny = D.ny;
  Q.nz = D.nz;
  Q.a0 = a0;
  Q.na = na;
  Q.npix = D.n_u * D.n_v;
  const double r = std::exp(-D.alpha * D.step);
  Q.r_hi = (float)r;
  Q.r_lo = (float)(r - (double)Q.r_hi);
  const double rm = D.r_inner + 1.5;
  Q.rmax2 = rm * rm;
  const dim3 grid((D.nx + 15) / 16, (D.ny + 15) / 16, D.nz);
  switch (proj_t) {
    case VAM_F32:
      hipLaunchKernelGGL(k_back_gather<float>, grid, dim3(256), 0, s, Q, (const float*)proj, dose, accumulate);
      break;
    case VAM_BF16:
      hipLaunchKernelGGL(k_back_gather<uint16_t>, grid, dim3(256), 0, s, Q, (const uint16_t*)proj, dose,
                         accumulate);
      break;
    case VAM_F16:
      hipLaunchKernelGGL(k_back_gather<__half>, grid, dim3(256), 0, s, Q, (const __half*)proj, dose, accumulate);
      break;
  }
  VAM_HIP_TRY(hipGetLastError(), "launching the gather deposit");
  return VAM_OK;
}

}  // namespace vam
