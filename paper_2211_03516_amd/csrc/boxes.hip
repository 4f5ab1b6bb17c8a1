// Lab-box tiling of the dose deposit (Sec. 2.5 of Webber et al.).
//
// The vial turns about +z, so every ray sample has a fixed position in the
// lab frame; only its volume-frame position depends on the angle.  At setup
// the resin samples of every ray are cut into segments, one per lab-frame
// box of B^3 voxels that they cross.  The deposit then runs one workgroup
// per (box, angle): the box, rotated into the volume frame, covers a small
// footprint of the padded grid (at most ~(B sqrt 2 + 3)^2 (B + 2) cells),
// which the workgroup accumulates in LDS with LDS atomics while it marches
// all segments of the box -- about 40 samples per voxel at the full-optics
// workload, i.e. ~320 corner deposits per cell -- and then adds to the
// global FP64 accumulator once per cell.  The per-sample work (position,
// weights, attenuation) is the same as in the ray-driven kernels; only the
// place the eight corner deposits land changes, from global atomics to LDS.

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "vam_internal.h"

namespace vam {

constexpr int kBox = 12;
constexpr int kMaxLdsBytes = 160 * 1024;  // LDS per CU on gfx950

// Cells of the largest rotated-box footprint for box edge B in a padded
// grid of px x py x pz: a rotated box spans at most B sqrt 2 cells in x and
// y and B in z; the footprint adds the rounding margin and the +1 corner.
static void footprint_bound(int B, int px, int py, int pz, int& wxy, int& wz) {
  wxy = std::min((int)std::floor(B * std::sqrt(2.0) + 3.02), std::max(px, py));
  wz = std::min(B + 2, pz);
}

int max_box_edge(const vam_geometry* h) {
  int best = 4;
  for (int B = 4; B <= 64; ++B) {
    int wxy, wz;
    footprint_bound(B, h->px, h->py, h->pz, wxy, wz);
    if ((int64_t)wxy * wxy * wz * 8 <= kMaxLdsBytes) best = B;
  }
  return best;
}

__device__ inline int box_of(const BoxGrid& G, double x, double y, double z) {
  int bx = (int)floor((x - G.x0) / G.B);
  int by = (int)floor((y - G.y0) / G.B);
  int bz = (int)floor((z - G.z0) / G.B);
  bx = min(max(bx, 0), G.nbx - 1);
  by = min(max(by, 0), G.nby - 1);
  bz = min(max(bz, 0), G.nbz - 1);
  return (bz * G.nby + by) * G.nbx + bx;
}

// Walk the z-clipped samples of every ray in the lab frame (FP64) and call
// emit(box, first k, count, rank) once per maximal run of samples in one
// box; rank numbers the runs of a ray from 0 in marching order.
template <class F>
__device__ inline void walk_segments(const BoxGrid& G, const RayRec& R, const double* o, double step,
                                     F emit) {
  if (R.n <= 0) return;
  int cur = -1, start = 0, rank = 0;
  for (int k = R.k0; k < R.k0 + R.n; ++k) {
    const double s = (k + 0.5) * step;
    const int b = box_of(G, o[0] + s * o[3], o[1] + s * o[4], o[2] + s * o[5]);
    if (b != cur) {
      if (cur >= 0) emit(cur, start, k - start, rank++);
      cur = b;
      start = k;
    }
  }
  if (cur >= 0) emit(cur, start, R.k0 + R.n - start, rank);
}

__global__ void k_seg_count(BoxGrid G, const RayRec* rays, const double* ray64, int64_t n_rays, double step,
                            int* box_count, int* ray_nseg) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  int n = 0;
  walk_segments(G, rays[r], ray64 + r * kRay64Fields, step, [&](int b, int, int, int) {
    atomicAdd(box_count + b, 1);
    ++n;
  });
  ray_nseg[r] = n;
}

__global__ void k_seg_fill(BoxGrid G, const RayRec* rays, const double* ray64, int64_t n_rays, double step,
                           const int* box_off, int* cursor, int4* segs) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  walk_segments(G, rays[r], ray64 + r * kRay64Fields, step, [&](int b, int k, int n, int rank) {
    const int slot = box_off[b] + atomicAdd(cursor + b, 1);
    segs[slot] = make_int4((int)r, k, n, rank);
  });
}

void free_boxes(vam_geometry* h) {
  void* ptrs[] = {h->segs, h->segs_fwd, h->box_begin, h->box_id, h->ray_nseg, h->seg_part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->segs = nullptr;
  h->segs_fwd = nullptr;
  h->box_begin = nullptr;
  h->box_id = nullptr;
  h->ray_nseg = nullptr;
  h->seg_part = nullptr;
  h->n_boxes = 0;
  h->n_segments = 0;
  h->max_seg_per_ray = 0;
}

struct BoxParams {
  BoxGrid G;
  int nboxes, na;      // work items of the launch: boxes x angles
  int xcd;             // 1: XCD-aware work order (see work_item)
  const int4* segs;
  const int* box_begin;
  const int* box_id;
  int wxy_max, wz_max;
  int npix;            // n_u * n_v
  int px, py, pz;
  double supp_coef;    // integer LDS accumulation: n_supp * step / n_pupil
};

BoxParams box_params(const vam_geometry* h);

// Samples per lab-frame unit cell (x, y from -R, padded z), from the same
// positions the marching kernels use (midpoint + t direction, FP64).
__global__ void k_lab_count(const RayRec* rays, int64_t n_rays, double step, double x0, int ncx, int ncz,
                            unsigned* count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  const RayRec R = rays[r];
  for (int k = R.k0; k < R.k0 + R.n; ++k) {
    const double t = ((double)k + 0.5 - 0.5 * (double)R.K) * step;
    const int ix = min(max((int)floor(R.mx + t * R.dx - x0), 0), ncx - 1);
    const int iy = min(max((int)floor(R.my + t * R.dy - x0), 0), ncx - 1);
    const int iz = min(max((int)floor((double)R.gz + t * (double)R.dz), 0), ncz - 1);
    atomicAdd(count + ((int64_t)iz * ncx + iy) * ncx + ix, 1u);
  }
}

// Largest sample count of any 4 x 4 x 3 block of cells.
__global__ void k_window_max(const unsigned* count, int ncx, int ncz, unsigned* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ncx * ncx * ncz) return;
  const int ix = (int)(i % ncx), iy = (int)((i / ncx) % ncx), iz = (int)(i / ((int64_t)ncx * ncx));
  unsigned sum = 0;
  for (int dz = 0; dz < 3 && iz + dz < ncz; ++dz)
    for (int dy = 0; dy < 4 && iy + dy < ncx; ++dy)
      for (int dx = 0; dx < 4 && ix + dx < ncx; ++dx) sum += count[((int64_t)(iz + dz) * ncx + iy + dy) * ncx + ix + dx];
  atomicMax(out, sum);
}

// n_supp of the integer LDS deposit (synchronises the stream).
static vam_status support_bound(vam_geometry* h, hipStream_t s) {
  const double R = h->desc.r_inner + 1.0;
  const int ncx = (int)std::ceil(2.0 * R), ncz = h->pz;
  const int64_t ncell = (int64_t)ncx * ncx * ncz;
  unsigned* count = nullptr;
  VAM_HIP_TRY(hipMalloc(&count, (ncell + 1) * sizeof(unsigned)), "allocating lab cell counts");
  unsigned* out = count + ncell;
  hipError_t e = hipMemsetAsync(count, 0, (ncell + 1) * sizeof(unsigned), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_lab_count, dim3((unsigned)((h->n_rays + 255) / 256)), dim3(256), 0, s, h->rays, h->n_rays,
                       h->desc.step, -R, ncx, ncz, count);
    hipLaunchKernelGGL(k_window_max, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, count, ncx, ncz, out);
    e = hipGetLastError();
  }
  unsigned hmax = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hmax, out, sizeof(unsigned), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(count);
  if (e != hipSuccess) return hip_check(e, "bounding samples per voxel support");
  h->n_supp = std::max<int64_t>(hmax, 1);
  return VAM_OK;
}

vam_status build_boxes(vam_geometry* h, hipStream_t s) {
  if (h->n_supp == 0) {
    vam_status st = support_bound(h, s);
    if (st != VAM_OK) return st;
  }
  const vam_geometry_desc& D = h->desc;
  BoxGrid G;
  G.B = h->box_edge > 0 ? h->box_edge : kBox;
  const double R = D.r_inner + 1.0;
  G.x0 = -R;
  G.y0 = -R;
  G.z0 = -(0.5 * (D.nz - 1) + kPad);  // lab z of padded grid coordinate 0
  G.nbx = (int)std::ceil(2.0 * R / G.B);
  G.nby = G.nbx;
  G.nbz = (int)std::ceil((double)h->pz / G.B);
  h->boxes = G;
  const int nb_all = G.nbx * G.nby * G.nbz;

  int* count = nullptr;
  int* off = nullptr;
  VAM_HIP_TRY(hipMalloc(&count, nb_all * sizeof(int)), "allocating box counts");
  VAM_HIP_TRY(hipMalloc(&off, nb_all * sizeof(int)), "allocating box offsets");
  VAM_HIP_TRY(hipMalloc(&h->ray_nseg, h->n_rays * sizeof(int)), "allocating segment counts");
  auto release = [&]() {
    (void)hipFree(count);
    (void)hipFree(off);
  };
  hipError_t e = hipMemsetAsync(count, 0, nb_all * sizeof(int), s);
  if (e != hipSuccess) {
    release();
    return hip_check(e, "clearing box counts");
  }
  const int threads = 256;
  const unsigned blocks = (unsigned)((h->n_rays + threads - 1) / threads);
  hipLaunchKernelGGL(k_seg_count, dim3(blocks), dim3(threads), 0, s, G, h->rays, h->ray64, h->n_rays,
                     D.step, count, h->ray_nseg);
  std::vector<int> hc(nb_all);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), count, nb_all * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release();
    return hip_check(e, "counting box segments");
  }
  std::vector<int> hoff(nb_all), begin, ids;
  int64_t total = 0;
  for (int b = 0; b < nb_all; ++b) {
    hoff[b] = (int)total;
    if (hc[b] > 0) {
      ids.push_back(b);
      begin.push_back((int)total);
    }
    total += hc[b];
  }
  begin.push_back((int)total);
  if (total >= 0x7fffffffLL) {
    release();
    return fail(VAM_ERR_UNSUPPORTED, "more than 2^31 ray segments");
  }
  h->n_boxes = (int)ids.size();
  h->n_segments = total;
  e = hipMalloc(&h->segs, std::max<int64_t>(total, 1) * sizeof(int4));
  if (e == hipSuccess) e = hipMalloc(&h->box_begin, begin.size() * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&h->box_id, std::max<size_t>(ids.size(), 1) * sizeof(int));
  if (e == hipSuccess) e = hipMemcpyAsync(off, hoff.data(), nb_all * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->box_begin, begin.data(), begin.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !ids.empty())
    e = hipMemcpyAsync(h->box_id, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(count, 0, nb_all * sizeof(int), s);
  if (e != hipSuccess) {
    release();
    return hip_check(e, "allocating box segments");
  }
  hipLaunchKernelGGL(k_seg_fill, dim3(blocks), dim3(threads), 0, s, G, h->rays, h->ray64, h->n_rays, D.step,
                     off, count, h->segs);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) return hip_check(e, "filling box segments");
  // Order each box's segments, once for the deposit (h->segs) and once for
  // the forward projection (h->segs_fwd); sorting also makes the order
  // independent of the scheduling of the fill kernel:
  //  0: by ray -- neighbouring lanes handle neighbouring pixels;
  //  1: by decreasing length -- lanes of a wave march similar lengths;
  //  2: by pixel parity class (u mod 2, v mod 2), then ray -- the lanes of
  //     a wave handle pixels two apart, whose trilinear stencils are disjoint;
  //  3, 4: the same with classes (u mod m, v mod m), m = 3, 4;
  //  5: by a hash of the ray index (lanes at unrelated positions);
  //  6: by pixel, then pupil sample -- the rays of one pixel, which meet at
  //     the focus plane, go to neighbouring lanes;
  //  7, 8: order 3, then each run of 1024 (7) or 2048 (8) consecutive
  //     segments by decreasing length in steps of two samples (a stable sort:
  //     equal steps keep their class order; exact lengths measured 1.5 %
  //     slower), so that the 64 lanes of a wave march similar lengths and
  //     the four waves of a workgroup get equal shares
  //     (the same runs on order 0 make the forward slower: 180 -> 187 ms);
  //  9: by pupil sample, then pixel column u, then row v -- neighbouring
  //     lanes march rays one pixel apart in z, which does not turn;
  //  10: by class (u mod 3, v mod 2), then ray (lanes three pixels apart
  //     along a row, rows two apart);
  //  11, 12, 13: order 10, then each run of 1024 (11), 512 (12) or 2048
  //     (13) consecutive segments by decreasing length.
  {
    std::vector<int4> hs(std::max<int64_t>(total, 1));
    e = hipMemcpy(hs.data(), h->segs, total * sizeof(int4), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(e, "reading box segments");
    const int nu = D.n_u, nv = D.n_v;
    auto sort_by = [&](int order) {
      auto key = [&](const int4& s, int order) -> int64_t {
        const int r = s.x;
        const int u = r % nu, v = (r / nu) % nv;
        if (order == 1) return ((int64_t)(0x7fff - s.z) << 32) | (uint32_t)r;
        if (order >= 2 && order <= 4) {
          const int m = order;
          return ((int64_t)((v % m) * m + (u % m)) << 32) | (uint32_t)r;
        }
        if (order == 6) return (int64_t)(r % (nu * nv)) * D.n_pupil + r / (nu * nv);
        if (order == 9) return ((int64_t)(r / (nu * nv)) * nu + u) * nv + v;
        if (order == 10) return ((int64_t)((v % 2) * 3 + (u % 3)) << 32) | (uint32_t)r;
        if (order == 5) {
          uint64_t x = (uint64_t)r + 0x9e3779b97f4a7c15ull;  // SplitMix64 finaliser
          x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
          x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
          return (int64_t)((x ^ (x >> 31)) >> 1);
        }
        return r;
      };
      const int korder = (order == 7 || order == 8) ? 3 : (order >= 11 && order <= 13) ? 10 : order;
      const int run = (order == 7 || order == 11)   ? 1024
                      : (order == 8 || order == 13) ? 2048
                      : order == 12                 ? 512
                                                    : 0;
      for (size_t i = 0; i + 1 < begin.size(); ++i) {
        std::sort(hs.begin() + begin[i], hs.begin() + begin[i + 1],
                  [&](const int4& x, const int4& y) { return key(x, korder) < key(y, korder); });
        for (int64_t g = begin[i]; run && g < begin[i + 1]; g += run)
          std::stable_sort(hs.begin() + g, hs.begin() + std::min<int64_t>(g + run, begin[i + 1]),
                           [](const int4& x, const int4& y) { return (x.z >> 1) > (y.z >> 1); });
      }
    };
    e = hipMalloc(&h->segs_fwd, std::max<int64_t>(total, 1) * sizeof(int4));
    if (e != hipSuccess) return hip_check(e, "allocating forward segments");
    sort_by(h->seg_order_fwd);
    e = hipMemcpy(h->segs_fwd, hs.data(), total * sizeof(int4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_check(e, "writing forward segments");
    sort_by(h->seg_order);
    e = hipMemcpy(h->segs, hs.data(), total * sizeof(int4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_check(e, "writing box segments");
    std::vector<int> ns(h->n_rays);
    e = hipMemcpy(ns.data(), h->ray_nseg, h->n_rays * sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(e, "reading segment counts");
    h->max_seg_per_ray = ns.empty() ? 0 : *std::max_element(ns.begin(), ns.end());
  }
  // largest footprint of a rotated box: extent B(|cos| + |sin|) <= B sqrt 2
  // in x and y, B in z, plus the rounding margin and the +1 corner
  const BoxParams Bp = box_params(h);
  h->box_cells = Bp.wxy_max * Bp.wxy_max * Bp.wz_max;
  return VAM_OK;
}

// --------------------------------------------------------------- deposit --



template <typename PT>
__device__ inline float load_p(const PT* p, int64_t i);
template <>
__device__ inline float load_p<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ inline float load_p<uint16_t>(const uint16_t* p, int64_t i) {
  return __uint_as_float((uint32_t)p[i] << 16);
}
template <>
__device__ inline float load_p<__half>(const __half* p, int64_t i) { return __half2float(p[i]); }


__device__ inline void store_proj(float* p, int64_t i, float x) { p[i] = x; }
__device__ inline void store_proj(uint16_t* p, int64_t i, float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    p[i] = (uint16_t)((u >> 16) | 0x40u);
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    p[i] = (uint16_t)(u >> 16);
  }
}
__device__ inline void store_proj(__half* p, int64_t i, float x) { p[i] = __float2half_rn(x); }


// XCD-aware work order.  Workgroups of a launch are handed to the 8 XCDs
// round-robin (workgroup L runs on XCD L mod 8), each XCD with its own L2.
// Work item w = (box, angle) is numbered box-major, angle-minor; XCD x takes
// the contiguous range [x per, (x + 1) per) in order.  The workgroups in
// flight on one XCD then share one or two boxes at neighbouring angles, so
// the box's segment and ray records and its volume footprint are fetched
// from HBM once and reused from that XCD's L2.
constexpr int kXcds = 8;

// Work order of the (box, angle) workgroups.
//   xcd = 0: boxes fastest, every XCD on the same angles;
//   xcd = 1: each XCD takes a contiguous range of (box, all angles) items, so
//            a box's segment and ray records are reused from that XCD's L2
//            across all angles;
//   xcd = A >= 2: the same, with the angles in blocks of A: a box's records
//            are reused across A angles while at most A workgroups of one box
//            flush into the same dose cells at a time.
// Workgroups are dispatched to the XCDs round-robin, so workgroup L runs on
// XCD L mod 8.
__device__ inline bool work_item(int nboxes, int na, int xcd, int& b, int& a) {
  if (!xcd) {
    const int64_t L = blockIdx.x;
    if (L >= (int64_t)nboxes * na) return false;
    a = (int)(L / nboxes);
    b = (int)(L - (int64_t)a * nboxes);
    return true;
  }
  const int A = xcd == 1 ? na : xcd;
  const int nblk = (na + A - 1) / A;
  const int64_t W = (int64_t)nblk * nboxes * A;
  const int64_t per = (W + kXcds - 1) / kXcds;
  const int64_t L = blockIdx.x;
  const int64_t i = L / kXcds;
  const int64_t w = (L % kXcds) * per + i;
  if (i >= per || w >= W) return false;
  const int64_t blk = w / ((int64_t)nboxes * A);
  const int64_t rem = w - blk * nboxes * A;
  b = (int)(rem / A);
  a = (int)(blk * A + (rem - (int64_t)b * A));
  return a < na;
}

static inline dim3 work_grid(int nboxes, int na, int xcd) {
  if (!xcd) return dim3((unsigned)((int64_t)nboxes * na));
  const int A = xcd == 1 ? na : xcd;
  const int64_t W = (int64_t)((na + A - 1) / A) * nboxes * A;
  return dim3((unsigned)(((W + kXcds - 1) / kXcds) * kXcds));
}

// Rotated-box footprint [X0, X1) x [Y0, Y1) x [Z0, Z1) in padded grid cells.
struct Foot {
  int X0, Y0, Z0, WX, WY, WZ;
};

__device__ inline Foot footprint(const BoxParams& Bp, int box, double c, double s, double cx, double cy) {
  const BoxGrid& G = Bp.G;
  const int bx = box % G.nbx, by = (box / G.nbx) % G.nby, bz = box / (G.nbx * G.nby);
  const double xa = G.x0 + bx * G.B, ya = G.y0 + by * G.B;
  double gxmin = 1e300, gxmax = -1e300, gymin = 1e300, gymax = -1e300;
  for (int q = 0; q < 4; ++q) {
    const double x = xa + (q & 1) * G.B, y = ya + (q >> 1) * G.B;
    const double gx = c * x + s * y + cx, gy = -s * x + c * y + cy;
    gxmin = fmin(gxmin, gx);
    gxmax = fmax(gxmax, gx);
    gymin = fmin(gymin, gy);
    gymax = fmax(gymax, gy);
  }
  // [lo, hi) clamped inside the padded grid, at least 2 and at most wmax
  // cells wide; a box outside the grid maps onto the padding at its edge
  auto range = [](double gmin, double gmax, int n, int wmax, int& lo, int& w) {
    lo = min(max((int)floor(gmin - 0.01), 0), n - 2);
    int hi = min(min((int)floor(gmax + 0.01) + 2, n), lo + wmax);
    w = max(hi, lo + 2) - lo;
  };
  Foot f;
  range(gxmin, gxmax, Bp.px, Bp.wxy_max, f.X0, f.WX);
  range(gymin, gymax, Bp.py, Bp.wxy_max, f.Y0, f.WY);
  // z does not turn and the boxes sit on whole cells: the box's samples have
  // z in [bz B, (bz + 1) B) up to the FP32 rounding of their positions, so
  // the footprint starts at bz B (a sample a rounding error below is clamped
  // onto it) and ends one cell above the last corner
  f.Z0 = min(max(bz * G.B, 0), Bp.pz - 2);
  const int zhi = min(min((bz + 1) * G.B + 2, Bp.pz), f.Z0 + Bp.wz_max);
  f.WZ = max(zhi, f.Z0 + 2) - f.Z0;
  return f;
}

// LT is the LDS accumulator type.  FP64: gfx950 executes LDS FP64 atomic
// adds ~20x faster than FP32 ones (measured 7.7 vs 0.33 lanes per clock per
// CU), and the partial sums keep FP64 precision.  AGG keeps the 8 corner
// sums of consecutive samples in one cell in registers and adds them to LDS
// when the cell changes.
template <typename PT, typename LT, bool AGG>
__global__ __launch_bounds__(256) void k_back_box(MarchParams P, BoxParams Bp, const PT* __restrict__ proj,
                                                  double* __restrict__ dose) {
  extern __shared__ __align__(16) unsigned char smem[];
  LT* acc = reinterpret_cast<LT*>(smem);
  int b, a;
  if (!work_item(Bp.nboxes, Bp.na, Bp.xcd, b, a)) return;
  const int box = Bp.box_id[b];
  const double2 cs = P.cs[P.a0 + a];
  const Foot f = footprint(Bp, box, cs.x, cs.y, P.cx, P.cy);
  const int ncell = f.WX * f.WY * f.WZ;
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) acc[i] = (LT)0;
  __syncthreads();

  // positions are clamped into the footprint (they lie inside it up to
  // rounding), so every LDS index is in range
  const float lox = (float)f.X0, hix = (float)(f.X0 + f.WX) - 1.001f;
  const float loy = (float)f.Y0, hiy = (float)(f.Y0 + f.WY) - 1.001f;
  const float loz = (float)f.Z0, hiz = (float)(f.Z0 + f.WZ) - 1.001f;
  const int sy = f.WX, sz = f.WX * f.WY;
  const int64_t pbase = (int64_t)a * Bp.npix;
  const int s_end = Bp.box_begin[b + 1];
  for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x) {
    const int4 sg = Bp.segs[si];
    const int r = sg.x, kb = sg.y, cnt = sg.z;
    const float pv = load_p(proj, pbase + r % Bp.npix);
    if (pv == 0.0f) continue;
    const RayRec R = P.rays[r];
    const float gx = (float)(cs.x * R.mx + cs.y * R.my + P.cx);
    const float gy = (float)(-cs.y * R.mx + cs.x * R.my + P.cy);
    const float dx = (float)(cs.x * R.dx + cs.y * R.dy);
    const float dy = (float)(-cs.y * R.dx + cs.x * R.dy);
    const float tb = fmaf((float)(kb - R.k0), P.step, R.t0);
    float e = R.cw * pv * __builtin_amdgcn_exp2f(P.nb * tb);
    float kf = 0.0f;
    int cur = -1;
    float w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < cnt; ++k, kf += 1.0f) {
      const float t = fmaf(kf, P.step, tb);
      const float x = __builtin_amdgcn_fmed3f(fmaf(t, dx, gx), lox, hix);
      const float y = __builtin_amdgcn_fmed3f(fmaf(t, dy, gy), loy, hiy);
      const float z = __builtin_amdgcn_fmed3f(fmaf(t, R.dz, R.gz), loz, hiz);
      const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y),
                  fz = __builtin_amdgcn_fractf(z);
      const int i = ((int)z - f.Z0) * sz + ((int)y - f.Y0) * sy + ((int)x - f.X0);
      const float z1 = e * fz, z0 = e - z1;
      const float y01 = z0 * fy, y00 = z0 - y01;
      const float y11 = z1 * fy, y10 = z1 - y11;
      const float q[8] = {y00 - y00 * fx, y00 * fx, y01 - y01 * fx, y01 * fx,
                          y10 - y10 * fx, y10 * fx, y11 - y11 * fx, y11 * fx};
      if (AGG) {
        if (i != cur) {
          if (cur >= 0) {
            LT* p = acc + cur;
            atomicAdd(p, (LT)w[0]);
            atomicAdd(p + 1, (LT)w[1]);
            atomicAdd(p + sy, (LT)w[2]);
            atomicAdd(p + sy + 1, (LT)w[3]);
            atomicAdd(p + sz, (LT)w[4]);
            atomicAdd(p + sz + 1, (LT)w[5]);
            atomicAdd(p + sz + sy, (LT)w[6]);
            atomicAdd(p + sz + sy + 1, (LT)w[7]);
          }
          cur = i;
#pragma unroll
          for (int c = 0; c < 8; ++c) w[c] = q[c];
        } else {
#pragma unroll
          for (int c = 0; c < 8; ++c) w[c] += q[c];
        }
      } else {
        LT* p = acc + i;
        atomicAdd(p, (LT)q[0]);
        atomicAdd(p + 1, (LT)q[1]);
        atomicAdd(p + sy, (LT)q[2]);
        atomicAdd(p + sy + 1, (LT)q[3]);
        atomicAdd(p + sz, (LT)q[4]);
        atomicAdd(p + sz + 1, (LT)q[5]);
        atomicAdd(p + sz + sy, (LT)q[6]);
        atomicAdd(p + sz + sy + 1, (LT)q[7]);
      }
      e = fmaf(e, P.r_hi, e * P.r_lo);
    }
    if (AGG && cur >= 0) {
      LT* p = acc + cur;
      atomicAdd(p, (LT)w[0]);
      atomicAdd(p + 1, (LT)w[1]);
      atomicAdd(p + sy, (LT)w[2]);
      atomicAdd(p + sy + 1, (LT)w[3]);
      atomicAdd(p + sz, (LT)w[4]);
      atomicAdd(p + sz + 1, (LT)w[5]);
      atomicAdd(p + sz + sy, (LT)w[6]);
      atomicAdd(p + sz + sy + 1, (LT)w[7]);
    }
  }
  __syncthreads();
  // one global FP64 add per touched cell
  const int plane = f.WX * f.WY;
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    const LT v = acc[i];
    if (v == (LT)0) continue;
    const int z = i / plane, rem = i - z * plane, y = rem / f.WX, x = rem - y * f.WX;
    const int64_t gi = ((int64_t)(f.Z0 + z) * Bp.py + (f.Y0 + y)) * Bp.px + (f.X0 + x);
    unsafeAtomicAdd(dose + gi, (double)v);
  }
}


// ------------------------------------------ fixed-footprint kernels ------
//
// The same two kernels with the LDS footprint laid out at compile-time
// strides for a given box edge B (row pitch WXY, slice pitch WXY^2, WZ
// slices, the largest footprint of a rotated box).  Corner offsets become
// immediates, index arithmetic uses 24-bit multiplies by constants, and the
// per-segment origin is formed in FP64 and rounded once:
//   p_k = P0 + k D,  P0 = g_mid + t_first d - footprint origin,  D = step d.

template <int B>
struct Fixed;
template <>
struct Fixed<8> {
  static constexpr int WXY = 14, WZ = 10;
};
template <>
struct Fixed<12> {
  static constexpr int WXY = 19, WZ = 14;
};
template <>
struct Fixed<16> {
  static constexpr int WXY = 25, WZ = 18;
};
static_assert(Fixed<8>::WZ == 8 + 2 && Fixed<12>::WZ == 12 + 2 && Fixed<16>::WZ == 16 + 2,
              "fixed footprints must match footprint_bound");

struct SegStart {
  float px, py, pz;   // first sample, footprint-local cell coordinates
  float dx, dy, dz;   // step between samples
  float tb;           // t of the first sample
};

__device__ inline SegStart seg_start(const MarchParams& P, const RayRec& R, double c, double s, const Foot& f,
                                     int kb) {
  const double tb = ((double)kb + 0.5 - 0.5 * (double)R.K) * (double)P.step;
  const double ddx = c * R.dx + s * R.dy, ddy = -s * R.dx + c * R.dy;
  SegStart g;
  g.px = (float)(c * R.mx + s * R.my + P.cx - f.X0 + tb * ddx);
  g.py = (float)(-s * R.mx + c * R.my + P.cy - f.Y0 + tb * ddy);
  g.pz = (float)((double)R.gz - f.Z0 + tb * (double)R.dz);
  g.dx = (float)(P.step * ddx);
  g.dy = (float)(P.step * ddy);
  g.dz = (float)(P.step * (double)R.dz);
  g.tb = (float)tb;
  return g;
}

// CACHE keeps the 8 corner values of the current cell in registers: at
// steps of half a voxel about a third of the samples stay in the cell of the
// previous one and then read nothing from LDS.
template <int B, bool CACHE>
__global__ __launch_bounds__(256) void k_forward_boxc(MarchParams P, BoxParams Bp, const float* __restrict__ vol,
                                                      float* __restrict__ part, int64_t n_rays, int smax) {
  constexpr int SY = Fixed<B>::WXY, SZ = SY * SY, NC = SZ * Fixed<B>::WZ;
  __shared__ float sv[NC];
  int b, a;
  if (!work_item(Bp.nboxes, Bp.na, Bp.xcd, b, a)) return;
  const double2 cs = P.cs[P.a0 + a];
  const Foot f = footprint(Bp, Bp.box_id[b], cs.x, cs.y, P.cx, P.cy);
  for (int i = threadIdx.x; i < NC; i += blockDim.x) {
    const int z = i / SZ, rem = i - z * SZ, y = rem / SY, x = rem - y * SY;
    float v = 0.0f;
    if (x < f.WX && y < f.WY && z < f.WZ)
      v = vol[((int64_t)(f.Z0 + z) * Bp.py + (f.Y0 + y)) * Bp.px + (f.X0 + x)];
    sv[i] = v;
  }
  __syncthreads();
  const float hx = (float)f.WX - 1.001f, hy = (float)f.WY - 1.001f, hz = (float)f.WZ - 1.001f;
  const int s_end = Bp.box_begin[b + 1];
  float* out = part + (int64_t)a * smax * n_rays;
  for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x) {
    const int4 sg = Bp.segs[si];
    const int r = sg.x, cnt = sg.z;
    const RayRec R = P.rays[r];
    const SegStart g = seg_start(P, R, cs.x, cs.y, f, sg.y);
    float S = 0.0f;
    float kf = (float)(cnt - 1);
    unsigned cur = 0xffffffffu;
    float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, v3 = 0.0f, v4 = 0.0f, v5 = 0.0f, v6 = 0.0f, v7 = 0.0f;
    for (int k = cnt - 1; k >= 0; --k, kf -= 1.0f) {
      const float x = __builtin_amdgcn_fmed3f(fmaf(kf, g.dx, g.px), 0.0f, hx);
      const float y = __builtin_amdgcn_fmed3f(fmaf(kf, g.dy, g.py), 0.0f, hy);
      const float z = __builtin_amdgcn_fmed3f(fmaf(kf, g.dz, g.pz), 0.0f, hz);
      const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y),
                  fz = __builtin_amdgcn_fractf(z);
      const unsigned o = __umul24((unsigned)z, SZ) + __umul24((unsigned)y, SY) + (unsigned)x;
      if (!CACHE || o != cur) {
        const float* p = sv + o;
        const float* q = p + SZ;
        v0 = p[0];
        v1 = p[1];
        v2 = p[SY];
        v3 = p[SY + 1];
        v4 = q[0];
        v5 = q[1];
        v6 = q[SY];
        v7 = q[SY + 1];
        cur = o;
      }
      const float c00 = fmaf(fx, v1 - v0, v0);
      const float c01 = fmaf(fx, v3 - v2, v2);
      const float c10 = fmaf(fx, v5 - v4, v4);
      const float c11 = fmaf(fx, v7 - v6, v6);
      const float c0 = fmaf(fy, c01 - c00, c00);
      const float c1 = fmaf(fy, c11 - c10, c10);
      const float val = fmaf(fz, c1 - c0, c0);
      S = fmaf(S, P.r_hi, fmaf(S, P.r_lo, val));
    }
    out[(int64_t)sg.w * n_rays + r] = R.cw * __builtin_amdgcn_exp2f(P.nb * g.tb) * S;
  }
}

// LDS adds of the deposit: FP64, or 32-bit integers in fixed point (the
// values already carry the workgroup's scale S and are rounded to the
// nearest integer, halves upwards, by one v_cvt_rpi_i32_f32).
__device__ inline int round_to_int(float v) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}
template <typename LT>
__device__ inline void lds_add(LT* p, float v, float S);
template <>
__device__ inline void lds_add<double>(double* p, float v, float) {
  atomicAdd(p, (double)v);
}
template <>
__device__ inline void lds_add<int>(int* p, float v, float) {
  atomicAdd(p, round_to_int(v));
}
// Packed pairs: the 64-bit word of a cell holds the exact integer
// hi * 2^32 + lo, the sum of the fixed-point deposits into corner x (lo) and
// corner x + 1 (hi) of the lanes whose cell it is.  Both parts stay within
// +-2^31, so the sign-extended low half of the word is the x corner's sum
// and the rest, shifted down by 32, the x + 1 corner's.
__device__ inline unsigned long long pack_pair(float lo_v, float hi_v) {
  const int lo = round_to_int(lo_v), hi = round_to_int(hi_v);
  return ((unsigned long long)(unsigned)(hi + (lo >> 31)) << 32) | (unsigned)lo;
}
__device__ inline void lds_add_pair(long long* p, float lo, float hi) {
  atomicAdd((unsigned long long*)p, pack_pair(lo, hi));
}

// LT = int: the footprint is accumulated in 32-bit fixed point (gfx950 adds
// 32-bit integers in LDS about twice as fast as FP64).  Overflow is ruled
// out per workgroup: a cell's sum is bounded by (samples inside one voxel's
// support) x (largest sample weight), where the first factor is n_supp, the
// most samples of all rays in any 4 x 4 x 3 block of lab-frame unit cells
// (the turned support of a voxel fits in such a block), and the second is
// step / n_pupil times the largest |projection value| among the box's
// segments at this angle.  S is the power of two that maps that bound to at
// most 2^30, so every partial sum stays below 2^31 and S is exact; the
// rounding error of an add is at most 1/(2S).  A non-finite projection value
// makes the whole footprint NaN.
template <int B, typename PT, int AGG, int NT, typename LT>
__global__ __launch_bounds__(NT) void k_back_boxc(MarchParams P, BoxParams Bp, const PT* __restrict__ proj,
                                                  double* __restrict__ dose) {
  // slice pitch one word longer than a slice: the 32-bit deposit at edge 12
  // measured 3 % faster than with SY * SY (pitches SY * SY + 2 .. + 4 were
  // slower again; the pitch decides which LDS banks the lanes' adds share);
  // packed pairs keep SY * SY so that four workgroups fit in the LDS
  constexpr int SY = Fixed<B>::WXY, SZ = SY * SY + (sizeof(LT) == 8 ? 0 : 1), NC = SZ * Fixed<B>::WZ;
  constexpr bool kInt = std::is_integral<LT>::value;      // fixed point
  constexpr bool kPair = kInt && sizeof(LT) == 8;          // packed x pairs
  static_assert(!kPair || AGG == 1, "packed pairs are built with run aggregation only");
  __shared__ LT acc[NC];
  __shared__ unsigned s_pvmax;
  __shared__ int s_bad;
  int b, a;
  if (!work_item(Bp.nboxes, Bp.na, Bp.xcd, b, a)) return;
  const double2 cs = P.cs[P.a0 + a];
  const Foot f = footprint(Bp, Bp.box_id[b], cs.x, cs.y, P.cx, P.cy);
  for (int i = threadIdx.x; i < NC; i += blockDim.x) acc[i] = (LT)0;
  if (kInt && threadIdx.x == 0) {
    s_pvmax = 0u;
    s_bad = 0;
  }
  __syncthreads();
  const float hx = (float)f.WX - 1.001f, hy = (float)f.WY - 1.001f, hz = (float)f.WZ - 1.001f;
  const int64_t pbase = (int64_t)a * Bp.npix;
  const int s_end = Bp.box_begin[b + 1];
  float S = 1.0f;
  double invS = 1.0;
  bool bad = false;
  if (kInt) {
    float m = 0.0f;
    bool nonfinite = false;
    for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x) {
      const float apv = fabsf(load_p(proj, pbase + Bp.segs[si].x % Bp.npix));
      if (apv <= 3.4028234e38f)
        m = fmaxf(m, apv);
      else
        nonfinite = true;
    }
    atomicMax(&s_pvmax, __float_as_uint(m));  // non-negative floats order as their bits
    if (nonfinite) atomicOr(&s_bad, 1);
    __syncthreads();
    bad = s_bad != 0;
    const double bound = Bp.supp_coef * (double)__uint_as_float(s_pvmax);
    int e2 = 0;
    if (bound > 0.0) e2 = min(max((int)floor(log2(1073741824.0 / bound)), -120), 120);
    S = ldexpf(1.0f, e2);
    invS = ldexp(1.0, -e2);
  }
  for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x) {
    const int4 sg = Bp.segs[si];
    const int r = sg.x, cnt = sg.z;
    const float pv = load_p(proj, pbase + r % Bp.npix);
    if (pv == 0.0f) continue;
    const RayRec R = P.rays[r];
    const SegStart g = seg_start(P, R, cs.x, cs.y, f, sg.y);
    float e = R.cw * pv * __builtin_amdgcn_exp2f(P.nb * g.tb);
    if (kInt) e *= S;  // sample weights in the fixed-point units
    float kf = 0.0f;
    const float kend = (float)cnt;  // exact: a segment has fewer than 2^24 samples
    float w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // AGG == 2: the cell whose corners w holds, starting at the first sample's
    int cx = 0, cy = 0, cz = 0;
    unsigned base = 0;
    if (AGG == 2) {
      cx = (int)__builtin_amdgcn_fmed3f(g.px, 0.0f, hx);
      cy = (int)__builtin_amdgcn_fmed3f(g.py, 0.0f, hy);
      cz = (int)__builtin_amdgcn_fmed3f(g.pz, 0.0f, hz);
      base = __umul24((unsigned)cz, SZ) + __umul24((unsigned)cy, SY) + (unsigned)cx;
    }
    // AGG == 1: byte offset in acc of the cell whose corners w holds, also
    // starting at the first sample's (w is zero until its first add)
    constexpr unsigned kL = sizeof(LT);
    auto cell_bytes = [&](float x, float y, float z) {
      return __umul24((unsigned)z, SZ * kL) + __umul24((unsigned)y, SY * kL) + (unsigned)x * kL;
    };
    unsigned cur = 0;
    if (AGG == 1)
      cur = cell_bytes(__builtin_amdgcn_fmed3f(g.px, 0.0f, hx), __builtin_amdgcn_fmed3f(g.py, 0.0f, hy),
                       __builtin_amdgcn_fmed3f(g.pz, 0.0f, hz));
    for (; kf < kend; kf += 1.0f) {
      const float x = __builtin_amdgcn_fmed3f(fmaf(kf, g.dx, g.px), 0.0f, hx);
      const float y = __builtin_amdgcn_fmed3f(fmaf(kf, g.dy, g.py), 0.0f, hy);
      const float z = __builtin_amdgcn_fmed3f(fmaf(kf, g.dz, g.pz), 0.0f, hz);
      const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y),
                  fz = __builtin_amdgcn_fractf(z);
      const unsigned o = __umul24((unsigned)z, SZ) + __umul24((unsigned)y, SY) + (unsigned)x;
      const float z1 = e * fz, z0 = e - z1;
      const float y01 = z0 * fy, y00 = z0 - y01;
      const float y11 = z1 * fy, y10 = z1 - y11;
      const float q[8] = {y00 - y00 * fx, y00 * fx, y01 - y01 * fx, y01 * fx,
                          y10 - y10 * fx, y10 * fx, y11 - y11 * fx, y11 * fx};
      if constexpr (AGG == 2) {
        // Corner sharing: moving one cell along an axis keeps the four
        // corners on the far face, so only the four on the near face are
        // added to LDS; the kept sums shift to the near side and the far
        // side restarts at zero.  Steps of more than one cell (only possible
        // for Delta s > 1) flush all eight corners.
        const int ix = (int)x, iy = (int)y, iz = (int)z;
        int ex = ix - cx, ey = iy - cy, ez = iz - cz;
        if (P.step > 1.0f) {
          if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ez < -1 || ez > 1) {
            LT* p = acc + base;
            lds_add(p, w[0], S);
            lds_add(p + 1, w[1], S);
            lds_add(p + SY, w[2], S);
            lds_add(p + SY + 1, w[3], S);
            lds_add(p + SZ, w[4], S);
            lds_add(p + SZ + 1, w[5], S);
            lds_add(p + SZ + SY, w[6], S);
            lds_add(p + SZ + SY + 1, w[7], S);
#pragma unroll
            for (int c = 0; c < 8; ++c) w[c] = 0.0f;
            cx = ix;
            cy = iy;
            cz = iz;
            base = __umul24((unsigned)cz, SZ) + __umul24((unsigned)cy, SY) + (unsigned)cx;
            ex = ey = ez = 0;
          }
        }
        if (ex != 0) {
          const bool up = ex > 0;  // near face: corners with x bit 0 (up) or 1
          LT* p = acc + base + (up ? 0 : 1);
          lds_add(p, (up ? w[0] : w[1]), S);
          lds_add(p + SY, (up ? w[2] : w[3]), S);
          lds_add(p + SZ, (up ? w[4] : w[5]), S);
          lds_add(p + SZ + SY, (up ? w[6] : w[7]), S);
#pragma unroll
          for (int c = 0; c < 8; c += 2) {
            const float lo = w[c], hi = w[c + 1];
            w[c] = up ? hi : 0.0f;
            w[c + 1] = up ? 0.0f : lo;
          }
          base += ex;
          cx = ix;
        }
        if (ey != 0) {
          const bool up = ey > 0;
          LT* p = acc + base + (up ? 0 : SY);
          lds_add(p, (up ? w[0] : w[2]), S);
          lds_add(p + 1, (up ? w[1] : w[3]), S);
          lds_add(p + SZ, (up ? w[4] : w[6]), S);
          lds_add(p + SZ + 1, (up ? w[5] : w[7]), S);
          const int pair[4] = {0, 1, 4, 5};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int c = pair[j];
            const float lo = w[c], hi = w[c + 2];
            w[c] = up ? hi : 0.0f;
            w[c + 2] = up ? 0.0f : lo;
          }
          base += ey * SY;
          cy = iy;
        }
        if (ez != 0) {
          const bool up = ez > 0;
          LT* p = acc + base + (up ? 0 : SZ);
          lds_add(p, (up ? w[0] : w[4]), S);
          lds_add(p + 1, (up ? w[1] : w[5]), S);
          lds_add(p + SY, (up ? w[2] : w[6]), S);
          lds_add(p + SY + 1, (up ? w[3] : w[7]), S);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float lo = w[c], hi = w[c + 4];
            w[c] = up ? hi : 0.0f;
            w[c + 4] = up ? 0.0f : lo;
          }
          base += ez * SZ;
          cz = iz;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] += q[c];
      } else if constexpr (AGG == 1) {
        // The run's sums are only read inside the flush and restart through
        // keep = 0, so the loop carries w and cur without copies between
        // iterations.
        const unsigned ob = cell_bytes(x, y, z);
        const bool fl = ob != cur;
        if (fl) {
          LT* p = (LT*)((char*)acc + cur);
          if constexpr (kPair) {
            lds_add_pair(p, w[0], w[1]);
            lds_add_pair(p + SY, w[2], w[3]);
            lds_add_pair(p + SZ, w[4], w[5]);
            lds_add_pair(p + SZ + SY, w[6], w[7]);
          } else {
            lds_add(p, w[0], S);
            lds_add(p + 1, w[1], S);
            lds_add(p + SY, w[2], S);
            lds_add(p + SY + 1, w[3], S);
            lds_add(p + SZ, w[4], S);
            lds_add(p + SZ + 1, w[5], S);
            lds_add(p + SZ + SY, w[6], S);
            lds_add(p + SZ + SY + 1, w[7], S);
          }
        }
        const float keep = fl ? 0.0f : 1.0f;
        cur = ob;
        // w[2j] += yz (1 - fx), w[2j+1] += yz fx, written so that every
        // update accumulates into w itself
        const float yz[4] = {y00, y01, y10, y11};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          w[2 * j] = fmaf(-yz[j], fx, fmaf(keep, w[2 * j], yz[j]));
          w[2 * j + 1] = fmaf(yz[j], fx, keep * w[2 * j + 1]);
        }
      } else {
        LT* p = acc + o;
        lds_add(p, q[0], S);
        lds_add(p + 1, q[1], S);
        lds_add(p + SY, q[2], S);
        lds_add(p + SY + 1, q[3], S);
        lds_add(p + SZ, q[4], S);
        lds_add(p + SZ + 1, q[5], S);
        lds_add(p + SZ + SY, q[6], S);
        lds_add(p + SZ + SY + 1, q[7], S);
      }
      e = fmaf(e, P.r_hi, e * P.r_lo);
    }
    if constexpr (AGG == 2) {
      if (cnt > 0) {
        LT* p = acc + base;
        lds_add(p, w[0], S);
        lds_add(p + 1, w[1], S);
        lds_add(p + SY, w[2], S);
        lds_add(p + SY + 1, w[3], S);
        lds_add(p + SZ, w[4], S);
        lds_add(p + SZ + 1, w[5], S);
        lds_add(p + SZ + SY, w[6], S);
        lds_add(p + SZ + SY + 1, w[7], S);
      }
    } else if constexpr (kPair) {
      if (cnt > 0) {
        LT* p = (LT*)((char*)acc + cur);
        lds_add_pair(p, w[0], w[1]);
        lds_add_pair(p + SY, w[2], w[3]);
        lds_add_pair(p + SZ, w[4], w[5]);
        lds_add_pair(p + SZ + SY, w[6], w[7]);
      }
    } else if constexpr (AGG == 1) {
      if (cnt > 0) {
        LT* p = (LT*)((char*)acc + cur);
        lds_add(p, w[0], S);
        lds_add(p + 1, w[1], S);
        lds_add(p + SY, w[2], S);
        lds_add(p + SY + 1, w[3], S);
        lds_add(p + SZ, w[4], S);
        lds_add(p + SZ + 1, w[5], S);
        lds_add(p + SZ + SY, w[6], S);
        lds_add(p + SZ + SY + 1, w[7], S);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NC; i += blockDim.x) {
    LT raw = acc[i];
    if (!kPair && raw == (LT)0 && !bad) continue;
    const int z = i / SZ, rem = i - z * SZ, y = rem / SY, x = rem - y * SY;
    if (x >= f.WX || y >= f.WY || z >= f.WZ) continue;
    if constexpr (kPair) {
      // this cell's sum: the low half of its own word plus the high half of
      // the word of its x - 1 neighbour in the same row
      const long long lo = (long long)(int)(unsigned)raw;
      long long hi = 0;
      if (x > 0) {
        const long long u = acc[i - 1];
        hi = (u - (long long)(int)(unsigned)u) >> 32;
      }
      raw = lo + hi;
      if (raw == 0 && !bad) continue;
    }
    const int64_t gi = ((int64_t)(f.Z0 + z) * Bp.py + (f.Y0 + y)) * Bp.px + (f.X0 + x);
    unsafeAtomicAdd(dose + gi, bad ? __builtin_nan("") : (double)raw * invS);
  }
}

// Fixed-footprint kernels exist for these edges; other edges use the
// runtime-stride kernels above.
static bool fixed_edge(int B) { return B == 8 || B == 12 || B == 16; }

BoxParams box_params(const vam_geometry* h) {
  BoxParams Bp;
  Bp.G = h->boxes;
  Bp.nboxes = h->n_boxes;
  Bp.na = 0;
  Bp.xcd = 0;
  Bp.segs = h->segs;
  Bp.box_begin = h->box_begin;
  Bp.box_id = h->box_id;
  footprint_bound(h->boxes.B, h->px, h->py, h->pz, Bp.wxy_max, Bp.wz_max);
  Bp.npix = h->desc.n_u * h->desc.n_v;
  Bp.px = h->px;
  Bp.py = h->py;
  Bp.pz = h->pz;
  Bp.supp_coef = (double)h->n_supp * h->desc.step / h->desc.n_pupil;
  return Bp;
}

template <typename PT, typename LT, bool AGG>
static void launch_box_k(vam_geometry* h, const MarchParams& P, const BoxParams& Bp, const PT* proj, int na,
                         hipStream_t s) {
  const size_t lds = (size_t)h->box_cells * sizeof(LT);
  static thread_local int configured = 0;  // bit per (LT, AGG) instantiation
  const int bit = (sizeof(LT) == 8 ? 1 : 0) + (AGG ? 2 : 0);
  if (!(configured & (1 << bit))) {
    (void)hipFuncSetAttribute((const void*)k_back_box<PT, LT, AGG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxLdsBytes);
    configured |= 1 << bit;
  }
  BoxParams Bw = Bp;
  Bw.nboxes = h->n_boxes;
  Bw.na = na;
  Bw.xcd = h->xcd_deposit;
  hipLaunchKernelGGL((k_back_box<PT, LT, AGG>), work_grid(h->n_boxes, na, Bw.xcd), dim3(256), lds, s, P, Bw, proj,
                     h->dose_pad64);
}

template <int B, typename PT, int AGG, typename LT>
static void launch_boxc(vam_geometry* h, const MarchParams& P, const BoxParams& Bp, const PT* proj, int na,
                        hipStream_t s) {
  BoxParams Bw = Bp;
  Bw.nboxes = h->n_boxes;
  Bw.na = na;
  Bw.xcd = h->xcd_deposit;
  const dim3 grid = work_grid(h->n_boxes, na, Bw.xcd);
  if (h->deposit_threads == 512)
    hipLaunchKernelGGL((k_back_boxc<B, PT, AGG, 512, LT>), grid, dim3(512), 0, s, P, Bw, proj, h->dose_pad64);
  else
    hipLaunchKernelGGL((k_back_boxc<B, PT, AGG, 256, LT>), grid, dim3(256), 0, s, P, Bw, proj, h->dose_pad64);
}

template <int B, typename PT, typename LT>
static void launch_boxc_agg(vam_geometry* h, const MarchParams& P, const BoxParams& Bp, const PT* proj, int na,
                            int agg, hipStream_t s) {
  switch (agg) {
    case 0: launch_boxc<B, PT, 0, LT>(h, P, Bp, proj, na, s); break;
    case 1: launch_boxc<B, PT, 1, LT>(h, P, Bp, proj, na, s); break;
    default: launch_boxc<B, PT, 2, LT>(h, P, Bp, proj, na, s); break;
  }
}

template <typename PT, typename LT>
static void launch_boxc_edge(vam_geometry* h, const MarchParams& P, const BoxParams& Bp, const PT* proj, int na,
                             int agg, hipStream_t s) {
  switch (h->boxes.B) {
    case 8: launch_boxc_agg<8, PT, LT>(h, P, Bp, proj, na, agg, s); break;
    case 12: launch_boxc_agg<12, PT, LT>(h, P, Bp, proj, na, agg, s); break;
    default: launch_boxc_agg<16, PT, LT>(h, P, Bp, proj, na, agg, s); break;
  }
}

template <typename PT>
static void launch_boxc_pair(vam_geometry* h, const MarchParams& P, const BoxParams& Bp, const PT* proj, int na,
                             hipStream_t s) {
  switch (h->boxes.B) {
    case 8: launch_boxc<8, PT, 1, long long>(h, P, Bp, proj, na, s); break;
    case 12: launch_boxc<12, PT, 1, long long>(h, P, Bp, proj, na, s); break;
    default: launch_boxc<16, PT, 1, long long>(h, P, Bp, proj, na, s); break;
  }
}

// Deposit variants of the box kernels: 6, 8, 10 accumulate the footprint in
// FP64, 13, 11, 12 in 32-bit fixed point, each without aggregation, with
// cell-run aggregation and with corner sharing; 14 in fixed point packed in
// 64-bit x pairs, with run aggregation.  Edges without a fixed-footprint
// kernel use the runtime-stride FP64 kernels.
template <typename PT>
static void launch_box_t(vam_geometry* h, const MarchParams& P, const PT* proj, int na, int variant,
                         hipStream_t s) {
  const BoxParams Bp = box_params(h);
  const bool fixed = fixed_edge(h->boxes.B) && h->fixed_kernels;
  const int agg = (variant == 10 || variant == 12) ? 2 : (variant == 8 || variant == 11 || variant == 14) ? 1 : 0;
  if (fixed && variant == 14) {
    launch_boxc_pair<PT>(h, P, Bp, proj, na, s);
    return;
  }
  if (fixed && (variant == 6 || variant == 8 || variant == 10)) {
    launch_boxc_edge<PT, double>(h, P, Bp, proj, na, agg, s);
    return;
  }
  if (fixed && variant >= 11) {
    launch_boxc_edge<PT, int>(h, P, Bp, proj, na, agg, s);
    return;
  }
  if (variant >= 10) variant = agg ? 8 : 6;
  switch (variant) {
    case 7: launch_box_k<PT, float, false>(h, P, Bp, proj, na, s); break;
    case 8: launch_box_k<PT, double, true>(h, P, Bp, proj, na, s); break;
    default: launch_box_k<PT, double, false>(h, P, Bp, proj, na, s); break;
  }
}

void launch_box_deposit(vam_geometry* h, const MarchParams& P, const void* proj, vam_dtype proj_t, int na,
                        int variant, hipStream_t s) {
  if (h->n_boxes == 0) return;
  switch (proj_t) {
    case VAM_F32: launch_box_t(h, P, (const float*)proj, na, variant, s); break;
    case VAM_BF16: launch_box_t(h, P, (const uint16_t*)proj, na, variant, s); break;
    case VAM_F16: launch_box_t(h, P, (const __half*)proj, na, variant, s); break;
  }
}


// --------------------------------------------------------------- forward --
//
// Forward projection over the same decomposition: the workgroup of a
// (box, angle) stages the rotated box footprint of the padded volume in LDS
// (one coalesced read per cell), then every segment of the box gathers its
// samples from LDS.  The segment's partial sum (Horner over its samples,
// times the ray weight and the attenuation of its first sample) is written to
// part[angle][rank][ray]; a second kernel adds, per pixel, the partials of
// its rays in a fixed order (pupil index, then rank), so the result does not
// depend on scheduling.

template <typename AT>
__global__ __launch_bounds__(256) void k_forward_box(MarchParams P, BoxParams Bp, const float* __restrict__ vol,
                                                     float* __restrict__ part, int64_t n_rays, int smax) {
  extern __shared__ float sv[];
  int b, a;
  if (!work_item(Bp.nboxes, Bp.na, Bp.xcd, b, a)) return;
  const int box = Bp.box_id[b];
  const double2 cs = P.cs[P.a0 + a];
  const Foot f = footprint(Bp, box, cs.x, cs.y, P.cx, P.cy);
  const int plane = f.WX * f.WY;
  const int ncell = plane * f.WZ;
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    const int z = i / plane, rem = i - z * plane, y = rem / f.WX, x = rem - y * f.WX;
    sv[i] = vol[((int64_t)(f.Z0 + z) * Bp.py + (f.Y0 + y)) * Bp.px + (f.X0 + x)];
  }
  __syncthreads();
  const float lox = (float)f.X0, hix = (float)(f.X0 + f.WX) - 1.001f;
  const float loy = (float)f.Y0, hiy = (float)(f.Y0 + f.WY) - 1.001f;
  const float loz = (float)f.Z0, hiz = (float)(f.Z0 + f.WZ) - 1.001f;
  const int sy = f.WX, sz = plane;
  const int s_end = Bp.box_begin[b + 1];
  float* out = part + (int64_t)a * smax * n_rays;
  for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x) {
    const int4 sg = Bp.segs[si];
    const int r = sg.x, kb = sg.y, cnt = sg.z;
    const RayRec R = P.rays[r];
    const float gx = (float)(cs.x * R.mx + cs.y * R.my + P.cx);
    const float gy = (float)(-cs.y * R.mx + cs.x * R.my + P.cy);
    const float dx = (float)(cs.x * R.dx + cs.y * R.dy);
    const float dy = (float)(-cs.y * R.dx + cs.x * R.dy);
    const float tb = fmaf((float)(kb - R.k0), P.step, R.t0);
    float S = 0.0f;
    float kf = (float)(cnt - 1);
    for (int k = cnt - 1; k >= 0; --k, kf -= 1.0f) {
      const float t = fmaf(kf, P.step, tb);
      const float x = __builtin_amdgcn_fmed3f(fmaf(t, dx, gx), lox, hix);
      const float y = __builtin_amdgcn_fmed3f(fmaf(t, dy, gy), loy, hiy);
      const float z = __builtin_amdgcn_fmed3f(fmaf(t, R.dz, R.gz), loz, hiz);
      const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y),
                  fz = __builtin_amdgcn_fractf(z);
      const float* p = sv + (((int)z - f.Z0) * sz + ((int)y - f.Y0) * sy + ((int)x - f.X0));
      const float c00 = fmaf(fx, p[1] - p[0], p[0]);
      const float c01 = fmaf(fx, p[sy + 1] - p[sy], p[sy]);
      const float c10 = fmaf(fx, p[sz + 1] - p[sz], p[sz]);
      const float c11 = fmaf(fx, p[sz + sy + 1] - p[sz + sy], p[sz + sy]);
      const float c0 = fmaf(fy, c01 - c00, c00);
      const float c1 = fmaf(fy, c11 - c10, c10);
      const float val = fmaf(fz, c1 - c0, c0);
      S = fmaf(S, P.r_hi, fmaf(S, P.r_lo, val));
    }
    out[(int64_t)sg.w * n_rays + r] = R.cw * __builtin_amdgcn_exp2f(P.nb * tb) * S;
  }
}

template <typename PT>
__global__ void k_reduce_segments(const float* __restrict__ part, const int* __restrict__ nseg,
                                  PT* __restrict__ proj, int npix, int np, int64_t n_rays, int smax, int na) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)na * npix) return;
  const int a = (int)(i / npix);
  const int pix = (int)(i - (int64_t)a * npix);
  const float* base = part + (int64_t)a * smax * n_rays;
  float acc = 0.0f;
  for (int j = 0; j < np; ++j) {
    const int64_t r = (int64_t)j * npix + pix;
    const int ns = nseg[r];
    const float* b = base + r;
    // four running sums in a fixed interleave keep four loads in flight
    // (38 % faster than one chain); the order is the same on every call
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    int q = 0;
    for (; q + 4 <= ns; q += 4) {
      s0 += b[(int64_t)q * n_rays];
      s1 += b[(int64_t)(q + 1) * n_rays];
      s2 += b[(int64_t)(q + 2) * n_rays];
      s3 += b[(int64_t)(q + 3) * n_rays];
    }
    for (; q < ns; ++q) s0 += b[(int64_t)q * n_rays];
    acc += (s0 + s1) + (s2 + s3);
  }
  store_proj(proj, i, acc);
}

template <typename PT>
static vam_status forward_box_t(vam_geometry* h, const MarchParams& P0, PT* proj, int na, hipStream_t s) {
  const vam_geometry_desc& D = h->desc;
  const int smax = std::max(h->max_seg_per_ray, 1);
  const int64_t per_angle = (int64_t)smax * h->n_rays;
  if (!h->seg_part) {
    // partial sums for a chunk of angles, at most ~8 GiB (5 chunks of 80
    // angles at 256^3 with 16 pupil samples: 1.7 % faster than 2 GiB chunks,
    // fewer launch tails and reductions); if the device cannot hold that
    // much, halve the chunk until the allocation succeeds
    int64_t angles = std::max<int64_t>(1, std::min<int64_t>(D.n_angles, (int64_t(1) << 31) / per_angle));
    for (;;) {
      const hipError_t e = hipMalloc(&h->seg_part, per_angle * angles * sizeof(float));
      if (e == hipSuccess) break;
      h->seg_part = nullptr;
      if (e != hipErrorOutOfMemory || angles == 1) return hip_check(e, "allocating segment partial sums");
      (void)hipGetLastError();  // the failed allocation's error is handled here
      angles = (angles + 1) / 2;
    }
    h->seg_part_angles = (int)angles;
  }
  const BoxParams Bp = box_params(h);
  const size_t lds = (size_t)h->box_cells * sizeof(float);
  const int npix = D.n_u * D.n_v;
  for (int c0 = 0; c0 < na; c0 += h->seg_part_angles) {
    const int nc = std::min(h->seg_part_angles, na - c0);
    MarchParams P = P0;
    P.a0 = P0.a0 + c0;
    BoxParams Bw = Bp;
    Bw.nboxes = h->n_boxes;
    Bw.na = nc;
    Bw.xcd = h->xcd_forward;
    Bw.segs = h->segs_fwd;
    if (h->n_boxes > 0 && fixed_edge(h->boxes.B) && h->fixed_kernels) {
      const dim3 grid = work_grid(h->n_boxes, nc, Bw.xcd);
      switch (h->boxes.B * 2 + (h->fwd_cache ? 1 : 0)) {
        case 16: hipLaunchKernelGGL((k_forward_boxc<8, false>), grid, dim3(256), 0, s, P, Bw, h->vol_pad, h->seg_part, h->n_rays, smax); break;
        case 17: hipLaunchKernelGGL((k_forward_boxc<8, true>), grid, dim3(256), 0, s, P, Bw, h->vol_pad, h->seg_part, h->n_rays, smax); break;
        case 24: hipLaunchKernelGGL((k_forward_boxc<12, false>), grid, dim3(256), 0, s, P, Bw, h->vol_pad, h->seg_part, h->n_rays, smax); break;
        case 25: hipLaunchKernelGGL((k_forward_boxc<12, true>), grid, dim3(256), 0, s, P, Bw, h->vol_pad, h->seg_part, h->n_rays, smax); break;
        case 32: hipLaunchKernelGGL((k_forward_boxc<16, false>), grid, dim3(256), 0, s, P, Bw, h->vol_pad, h->seg_part, h->n_rays, smax); break;
        default: hipLaunchKernelGGL((k_forward_boxc<16, true>), grid, dim3(256), 0, s, P, Bw, h->vol_pad, h->seg_part, h->n_rays, smax); break;
      }
    } else if (h->n_boxes > 0) {
      static thread_local bool configured = false;
      if (!configured) {
        (void)hipFuncSetAttribute((const void*)k_forward_box<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kMaxLdsBytes);
        configured = true;
      }
      hipLaunchKernelGGL((k_forward_box<float>), work_grid(h->n_boxes, nc, Bw.xcd), dim3(256), lds, s, P, Bw, h->vol_pad,
                         h->seg_part, h->n_rays, smax);
    }
    const int64_t n = (int64_t)nc * npix;
    hipLaunchKernelGGL(k_reduce_segments<PT>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->seg_part,
                       h->ray_nseg, proj + (int64_t)c0 * npix, npix, D.n_pupil, h->n_rays, smax, nc);
    VAM_HIP_TRY(hipGetLastError(), "launching the box-tiled forward projector");
  }
  return VAM_OK;
}

vam_status launch_box_forward(vam_geometry* h, const MarchParams& P, void* proj, vam_dtype proj_t, int na,
                              hipStream_t s) {
  switch (proj_t) {
    case VAM_F32: return forward_box_t(h, P, (float*)proj, na, s);
    case VAM_BF16: return forward_box_t(h, P, (uint16_t*)proj, na, s);
    case VAM_F16: return forward_box_t(h, P, (__half*)proj, na, s);
  }
  return fail(VAM_ERR_INVALID_ARG, "unknown projection dtype");
}

}  // namespace vam
