// Lab-box tiling of the forward projection (Sec. 2.4 of Webber et al.) and
// of the dose deposit (Sec. 2.5).
//
// The vial turns about +z, so every ray sample has a fixed position in the
// lab frame; only its volume-frame position depends on the angle.  At setup
// the resin samples of every ray are cut into segments, one per lab-frame
// box of B^3 voxels that they cross, and each segment is stored as a compact
// record: its first sample's lab position relative to the box, its
// direction, its sample count and the attenuated weight of its first sample.
// Both operators then run one workgroup per (box, angle): the box, rotated
// into the volume frame, covers a small footprint of the padded grid (at
// most ~(B sqrt 2 + 3)^2 (B + 2) cells), which the workgroup stages in LDS
// (forward: the volume; deposit: a fixed-point accumulator) while it marches
// all segments of the box -- about 40 samples per voxel at the full-optics
// workload.  The per-sample work (position, trilinear weights of Sec. 2.2,
// Beer-Lambert attenuation) is the same as in the ray-driven kernels; only
// the place where the eight corner values are read or added changes, from
// global memory to LDS.

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "vam_internal.h"

namespace vam {

constexpr int kBox = 12;  // default lab box edge (fastest measured for both operators)
constexpr int kXcds = 8;  // XCDs of an MI355X; workgroup L of a launch runs on XCD L mod 8

// Compile-time footprints for the supported box edges: row pitch WXY, WZ
// slices (the largest footprint of a rotated box: extent B(|cos| + |sin|) <=
// B sqrt 2 cells in x and y plus the rounding margin and the +1 corner, B + 2
// in z).
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

bool supported_box_edge(int B) { return B == 8 || B == 12 || B == 16; }

static void footprint_bound(int B, int px, int py, int pz, int& wxy, int& wz) {
  wxy = std::min((int)std::floor(B * std::sqrt(2.0) + 3.02), std::max(px, py));
  wz = std::min(B + 2, pz);
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

// Walk the z-clipped samples of a ray in the lab frame (FP64, sample k at
// e + (k + 1/2) step d) and call emit(box, first k, count, rank) once per
// maximal run of samples in one box; rank numbers the runs of a ray from 0
// in marching order.
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

// Compact records of the (sorted) segments {ray, first k, count, rank} of
// every box, one workgroup per box.  The lab position of the segment's
// middle sample m = (count - 1) / 2 (rounded down) is formed in FP64 and
// stored relative to the box (x, y from its centre, z from its bottom face),
// so FP32 keeps it to ~1e-6 voxel, and the kernels step from it by at most
// half the segment (the rounding of the direction grows with the distance
// stepped); the weight is (T1 T2 / n_pupil) step exp(-alpha s) at the
// segment's first sample, rounded once.
//   pw = (x_m - xc, y_m - yc, z_m - zb, weight), dn = (d_x, d_y, d_z, count),
//   idx = pixel (deposit) or partial-sum slot rank * n_rays + ray (forward:
//   lanes marching neighbouring rays write neighbouring slots).
__global__ void k_seg_pack(BoxGrid G, const int* box_id, const int* box_begin, const int4* segs,
                           const double* ray64, int n_rays, double step, double alpha, int npix,
                           int forward, float4* pw, float4* dn, int* idx) {
  const int b = blockIdx.x;
  const int box = box_id[b];
  const int bx = box % G.nbx, by = (box / G.nbx) % G.nby, bz = box / (G.nbx * G.nby);
  const double xc = G.x0 + (bx + 0.5) * G.B, yc = G.y0 + (by + 0.5) * G.B, zb = G.z0 + (double)bz * G.B;
  for (int i = box_begin[b] + threadIdx.x; i < box_begin[b + 1]; i += blockDim.x) {
    const int4 sg = segs[i];
    const double* o = ray64 + (int64_t)sg.x * kRay64Fields;
    const double s = (sg.y + 0.5) * step;
    const double sm = (sg.y + (sg.z - 1) / 2 + 0.5) * step;
    pw[i] = make_float4((float)(o[0] + sm * o[3] - xc), (float)(o[1] + sm * o[4] - yc),
                        (float)(o[2] + sm * o[5] - zb), (float)(o[8] * step * exp(-alpha * s)));
    dn[i] = make_float4((float)o[3], (float)o[4], (float)o[5], __int_as_float(sg.z));
    idx[i] = forward ? sg.w * n_rays + sg.x : sg.x % npix;
  }
}

// ------------------------------------------------- fixed-point bound ------

// Samples per lab-frame unit cell (x, y from -R, padded z), from the same
// FP64 positions the segment records are made of.
__global__ void k_lab_count(const RayRec* rays, const double* ray64, int64_t n_rays, double step, double x0,
                            double z0, int ncx, int ncz, unsigned* count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  const RayRec R = rays[r];
  const double* o = ray64 + r * kRay64Fields;
  for (int k = R.k0; k < R.k0 + R.n; ++k) {
    const double s = (k + 0.5) * step;
    const int ix = min(max((int)floor(o[0] + s * o[3] - x0), 0), ncx - 1);
    const int iy = min(max((int)floor(o[1] + s * o[4] - x0), 0), ncx - 1);
    const int iz = min(max((int)floor(o[2] + s * o[5] - z0), 0), ncz - 1);
    atomicAdd(count + ((int64_t)iz * ncx + iy) * ncx + ix, 1u);
  }
}

// Per-box bound of the fixed-point deposit: the most samples OF THE BOX in
// any 4 x 4 x 3 block of lab-frame unit cells.  The box's samples are the
// samples inside its B^3 cells, so that is the largest window sum of the
// cell counts clipped to the box; a voxel's turned support (a 2 x 2 x 2
// cube: at most 2 sqrt 2 wide in x and y) always fits in such a block, so
// at any angle the box adds at most that many samples into one LDS cell.
// One workgroup per box.
__global__ void k_box_supp(BoxGrid G, const int* box_id, const unsigned* count, int ncx, int ncz, int* supp) {
  __shared__ unsigned s_max;
  if (threadIdx.x == 0) s_max = 0u;
  __syncthreads();
  const int box = box_id[blockIdx.x];
  const int bx = box % G.nbx, by = (box / G.nbx) % G.nby, bz = box / (G.nbx * G.nby);
  const int x0 = bx * G.B, y0 = by * G.B, z0 = bz * G.B;
  const int x1 = min(x0 + G.B, ncx), y1 = min(y0 + G.B, ncx), z1 = min(z0 + G.B, ncz);
  // window anchors (lowest cell) from 3 (x, y) or 2 (z) cells before the box
  const int nwx = G.B + 3, nwz = G.B + 2;
  unsigned best = 0;
  for (int w = threadIdx.x; w < nwx * nwx * nwz; w += blockDim.x) {
    const int wx = x0 - 3 + w % nwx, wy = y0 - 3 + (w / nwx) % nwx, wz = z0 - 2 + w / (nwx * nwx);
    unsigned sum = 0;
    for (int z = max(wz, z0); z < min(wz + 3, z1); ++z)
      for (int y = max(wy, y0); y < min(wy + 4, y1); ++y)
        for (int x = max(wx, x0); x < min(wx + 4, x1); ++x) sum += count[((int64_t)z * ncx + y) * ncx + x];
    best = max(best, sum);
  }
  atomicMax(&s_max, best);
  __syncthreads();
  if (threadIdx.x == 0) supp[blockIdx.x] = (int)min(max(s_max, 1u), 0x3fffffffu);
}

// Per-box n_supp of the fixed-point deposit (synchronises the stream).
static vam_status support_bound(vam_geometry* h, const BoxGrid& G, hipStream_t s) {
  const double R = h->desc.r_inner + 1.0;
  const int ncx = (int)std::ceil(2.0 * R), ncz = h->pz;
  const int64_t ncell = (int64_t)ncx * ncx * ncz;
  unsigned* count = nullptr;
  VAM_HIP_TRY(dev_alloc((void**)&count, ncell * sizeof(unsigned)), "allocating lab cell counts");
  hipError_t e = hipMemsetAsync(count, 0, ncell * sizeof(unsigned), s);
  if (e == hipSuccess) {
    const double z0 = -(0.5 * (h->desc.nz - 1) + kPad);
    hipLaunchKernelGGL(k_lab_count, dim3((unsigned)((h->n_rays + 255) / 256)), dim3(256), 0, s, h->rays, h->ray64,
                       h->n_rays, h->desc.step, -R, z0, ncx, ncz, count);
    if (h->n_boxes > 0)
      hipLaunchKernelGGL(k_box_supp, dim3((unsigned)h->n_boxes), dim3(256), 0, s, G, h->box_id, count, ncx, ncz,
                         h->box_supp);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(count);
  if (e != hipSuccess) return hip_check(e, "bounding samples per voxel support");
  // a 4 x 4 x 3 block of cells meets at most 2 boxes along each axis (the
  // box edge is at least 8), so all boxes together put at most 8 x the
  // largest box_supp samples into one voxel's support
  std::vector<int> hb(std::max(h->n_boxes, 1), 0);
  if (h->n_boxes > 0) {
    e = hipMemcpy(hb.data(), h->box_supp, h->n_boxes * sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(e, "reading the support bounds");
  }
  h->supp_bound = 8 * (int64_t)*std::max_element(hb.begin(), hb.end());
  return VAM_OK;
}

// ------------------------------------------------------ decomposition ------

static void free_table(SegTable& t) {
  void* ptrs[] = {t.pw, t.dn, t.idx};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  t = SegTable{};
}

void free_boxes(vam_geometry* h) {
  free_table(h->seg_dep);
  free_table(h->seg_fwd);
  void* ptrs[] = {h->box_begin, h->box_id, h->box_supp, h->ray_nseg, h->seg_part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->box_begin = nullptr;
  h->box_id = nullptr;
  h->box_supp = nullptr;
  h->ray_nseg = nullptr;
  h->seg_part = nullptr;
  h->seg_part_angles = 0;
  h->n_boxes = 0;
  h->n_segments = 0;
  h->max_seg_per_ray = 0;
  h->boxes_ready = 0;
}

static vam_status alloc_table(SegTable& t, int64_t n) {
  const int64_t m = std::max<int64_t>(n, 1);
  VAM_HIP_TRY(dev_alloc((void**)&t.pw, m * sizeof(float4)), "allocating segment records");
  VAM_HIP_TRY(dev_alloc((void**)&t.dn, m * sizeof(float4)), "allocating segment records");
  VAM_HIP_TRY(dev_alloc((void**)&t.idx, m * sizeof(int)), "allocating segment records");
  return VAM_OK;
}

// Order of the segments inside a box, which decides which lanes march
// together (host sort keys; measured orders, see vam_set_variant op 4):
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
//     equal steps keep their class order), so that the 64 lanes of a wave
//     march similar lengths and the waves of a workgroup get equal shares;
//  9: by pupil sample, then pixel column u, then row v -- neighbouring
//     lanes march rays one pixel apart in z, which does not turn;
//  10: by class (u mod 3, v mod 2), then ray (lanes three pixels apart
//     along a row, rows two apart);
//  11, 12, 13: order 10, then each run of 1024 (11), 512 (12) or 2048
//     (13) consecutive segments by decreasing length;
//  14, 15, 16: by ray, then each run of 256 (14) or 1024 (15) segments, or
//     the whole box (16), by decreasing length in steps of two samples
//     (ties keep the ray order).
static void sort_segments(std::vector<int4>& hs, const std::vector<int>& begin, int order, int nu, int nv,
                          int np) {
  auto key = [&](const int4& s, int ord) -> int64_t {
    const int r = s.x;
    const int u = r % nu, v = (r / nu) % nv;
    if (ord == 1) return ((int64_t)(0x7fffffff - s.z) << 32) | (uint32_t)r;
    if (ord >= 2 && ord <= 4) return ((int64_t)((v % ord) * ord + (u % ord)) << 32) | (uint32_t)r;
    if (ord == 6) return (int64_t)(r % (nu * nv)) * np + r / (nu * nv);
    if (ord == 9) return ((int64_t)(r / (nu * nv)) * nu + u) * nv + v;
    if (ord == 10) return ((int64_t)((v % 2) * 3 + (u % 3)) << 32) | (uint32_t)r;
    if (ord == 5) {
      uint64_t x = (uint64_t)r + 0x9e3779b97f4a7c15ull;  // SplitMix64 finaliser
      x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
      x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
      return (int64_t)((x ^ (x >> 31)) >> 1);
    }
    return r;
  };
  const int korder = (order == 7 || order == 8) ? 3 : (order >= 11 && order <= 13) ? 10 : order >= 14 ? 0 : order;
  const int run = (order == 7 || order == 11 || order == 15) ? 1024 : (order == 8 || order == 13) ? 2048
                : order == 12 ? 512 : order == 14 ? 256 : order == 16 ? 0x7fffffff : 0;
  for (size_t i = 0; i + 1 < begin.size(); ++i) {
    std::sort(hs.begin() + begin[i], hs.begin() + begin[i + 1],
              [&](const int4& x, const int4& y) { return key(x, korder) < key(y, korder); });
    for (int64_t g = begin[i]; run && g < begin[i + 1]; g += run)
      std::stable_sort(hs.begin() + g, hs.begin() + std::min<int64_t>(g + run, begin[i + 1]),
                       [](const int4& x, const int4& y) { return (x.z >> 1) > (y.z >> 1); });
  }
}

// Build the decomposition into the handle (everything it allocates is
// recorded in the handle as soon as it exists, so free_boxes releases it
// on any failure).  Synchronises the stream.
static vam_status build_boxes_into(vam_geometry* h, hipStream_t s) {
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

  VAM_HIP_TRY(dev_alloc((void**)&h->ray_nseg, h->n_rays * sizeof(int)), "allocating segment counts");
  // staging: box counts, offsets and cursors, then the unsorted segments
  int* count = nullptr;
  int4* segs = nullptr;
  auto release = [&]() {
    if (count) (void)hipFree(count);
    if (segs) (void)hipFree(segs);
    count = nullptr;
    segs = nullptr;
  };
  hipError_t e = dev_alloc((void**)&count, 2 * (int64_t)nb_all * sizeof(int));
  if (e != hipSuccess) return hip_check(e, "allocating box counts");
  int* off = count + nb_all;
  e = hipMemsetAsync(count, 0, nb_all * sizeof(int), s);
  const int threads = 256;
  const unsigned blocks = (unsigned)((h->n_rays + threads - 1) / threads);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_seg_count, dim3(blocks), dim3(threads), 0, s, G, h->rays, h->ray64, h->n_rays, D.step,
                       count, h->ray_nseg);
    e = hipGetLastError();
  }
  std::vector<int> hc(nb_all), ns(h->n_rays);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), count, nb_all * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ns.data(), h->ray_nseg, h->n_rays * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release();
    return hip_check(e, "counting box segments");
  }
  std::vector<int> hoff(nb_all), begin, ids;
  int64_t total = 0;
  for (int b = 0; b < nb_all; ++b) {
    hoff[b] = (int)std::min<int64_t>(total, 0x7fffffff);
    if (hc[b] > 0) {
      ids.push_back(b);
      begin.push_back((int)std::min<int64_t>(total, 0x7fffffff));
    }
    total += hc[b];
  }
  begin.push_back((int)std::min<int64_t>(total, 0x7fffffff));
  if (total >= 0x7fffffffLL) {
    release();
    return fail(VAM_ERR_UNSUPPORTED, "more than 2^31 ray segments");
  }
  // forward partial-sum slots rank * n_rays + ray must be 32-bit offsets
  h->max_seg_per_ray = ns.empty() ? 0 : *std::max_element(ns.begin(), ns.end());
  if ((int64_t)h->max_seg_per_ray * h->n_rays >= 0x7fffffffLL) {
    release();
    return fail(VAM_ERR_UNSUPPORTED, "more than 2^31 forward partial-sum slots per angle");
  }
  e = dev_alloc((void**)&segs, std::max<int64_t>(total, 1) * sizeof(int4));
  if (e == hipSuccess) e = dev_alloc((void**)&h->box_begin, begin.size() * sizeof(int));
  if (e == hipSuccess) e = dev_alloc((void**)&h->box_id, std::max<size_t>(ids.size(), 1) * sizeof(int));
  if (e == hipSuccess) e = dev_alloc((void**)&h->box_supp, std::max<size_t>(ids.size(), 1) * sizeof(int));
  if (e == hipSuccess) e = hipMemcpyAsync(off, hoff.data(), nb_all * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->box_begin, begin.data(), begin.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !ids.empty())
    e = hipMemcpyAsync(h->box_id, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(count, 0, nb_all * sizeof(int), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_seg_fill, dim3(blocks), dim3(threads), 0, s, G, h->rays, h->ray64, h->n_rays, D.step,
                       off, count, segs);
    e = hipGetLastError();
  }
  std::vector<int4> hs(std::max<int64_t>(total, 1));
  if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), segs, total * sizeof(int4), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release();
    return hip_check(e, "filling box segments");
  }
  h->n_boxes = (int)ids.size();
  h->n_segments = total;
  {
    // the most samples of one pixel over all its rays (bounds the
    // fixed-point forward's sums)
    const int npix = D.n_u * D.n_v;
    std::vector<int64_t> per(npix, 0);
    for (int64_t i = 0; i < total; ++i) per[hs[i].x % npix] += hs[i].z;
    h->pix_samples_max = per.empty() ? 0 : *std::max_element(per.begin(), per.end());
  }
  {
    vam_status st = support_bound(h, G, s);
    if (st != VAM_OK) {
      release();
      return st;
    }
  }
  // both orders, each packed into compact records (the sort also makes the
  // order independent of the scheduling of the fill kernel)
  const int npix = D.n_u * D.n_v;
  for (int fwd = 0; fwd < 2; ++fwd) {
    SegTable& t = fwd ? h->seg_fwd : h->seg_dep;
    vam_status st = alloc_table(t, total);
    if (st != VAM_OK) {
      release();
      return st;
    }
    sort_segments(hs, begin, fwd ? h->seg_order_fwd : h->seg_order, D.n_u, D.n_v, D.n_pupil);
    e = hipMemcpyAsync(segs, hs.data(), total * sizeof(int4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && h->n_boxes > 0) {
      hipLaunchKernelGGL(k_seg_pack, dim3((unsigned)h->n_boxes), dim3(256), 0, s, G, h->box_id, h->box_begin, segs,
                         h->ray64, (int)h->n_rays, D.step, D.alpha, npix, fwd, t.pw, t.dn, t.idx);
      e = hipGetLastError();
    }
    // the host copy is re-sorted next: wait for the upload
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      release();
      return hip_check(e, "packing box segments");
    }
  }
  release();
  int wxy, wz;
  footprint_bound(G.B, h->px, h->py, h->pz, wxy, wz);
  h->box_cells = wxy * wxy * wz;
  return VAM_OK;
}

vam_status build_boxes(vam_geometry* h, hipStream_t s) {
  free_boxes(h);
  const vam_status st = build_boxes_into(h, s);
  if (st != VAM_OK) {
    free_boxes(h);  // nothing half-built stays behind; boxes_ready stays 0
    return st;
  }
  h->boxes_ready = 1;
  return VAM_OK;
}

// ---------------------------------------------------------- launch data ----

struct BoxParams {
  BoxGrid G;
  int nboxes, na;      // work items of the launch: boxes x angles
  int xcd;             // work order (see work_item)
  SegTable seg;
  const int* box_begin;
  const int* box_id;
  const int* box_supp; // fixed-point deposit: per-box n_supp
  int wxy_max, wz_max;
  int npix;            // n_u * n_v
  int px, py, pz;
  double w_coef;       // step / n_pupil: no sample weight exceeds it times |P|
};

static BoxParams box_params(const vam_geometry* h, const SegTable& t, int na, int xcd) {
  BoxParams Bp;
  Bp.G = h->boxes;
  Bp.nboxes = h->n_boxes;
  Bp.na = na;
  Bp.xcd = xcd;
  Bp.seg = t;
  Bp.box_begin = h->box_begin;
  Bp.box_id = h->box_id;
  Bp.box_supp = h->box_supp;
  footprint_bound(h->boxes.B, h->px, h->py, h->pz, Bp.wxy_max, Bp.wz_max);
  Bp.npix = h->desc.n_u * h->desc.n_v;
  Bp.px = h->px;
  Bp.py = h->py;
  Bp.pz = h->pz;
  Bp.w_coef = h->desc.step / h->desc.n_pupil;
  return Bp;
}

// Work order of the (box, angle) workgroups.
//   xcd = 0: boxes fastest, every XCD on the same angles;
//   xcd = 1: each XCD takes a contiguous range of (box, all angles) items, so
//            a box's segment records are reused from that XCD's L2 across
//            all angles;
//   xcd = A >= 2: the same, with the angles in blocks of A: a box's records
//            are reused across A angles while at most A workgroups of one box
//            flush into the same dose cells at a time.
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

// Rotated-box footprint [X0, X0 + WX) x [Y0, Y0 + WY) x [Z0, Z0 + WZ) in
// padded grid cells, and the box's centre in footprint coordinates.
struct Foot {
  int X0, Y0, Z0, WX, WY, WZ;
  float cx, cy, zoff;  // box centre (x, y) and bottom face (z) in footprint cells
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
  // the footprint starts at bz B and ends one cell above the last corner
  f.Z0 = min(max(bz * G.B, 0), Bp.pz - 2);
  const int zhi = min(min((bz + 1) * G.B + 2, Bp.pz), f.Z0 + Bp.wz_max);
  f.WZ = max(zhi, f.Z0 + 2) - f.Z0;
  const double xc = xa + 0.5 * G.B, yc = ya + 0.5 * G.B;
  f.cx = (float)(c * xc + s * yc + cx - f.X0);
  f.cy = (float)(-s * xc + c * yc + cy - f.Y0);
  f.zoff = (float)(bz * G.B - f.Z0);
  return f;
}

// Middle sample and step of a segment in footprint cells at angle (c, s);
// sample k of the segment (k = 0 .. count - 1) is at p + (k - m) d.
struct SegPos {
  float px, py, pz;   // middle sample m = (count - 1) / 2, rounded down
  float dx, dy, dz;   // step between samples
  float k0, k1;       // first and last sample relative to m: -m and count - 1 - m
};

__device__ inline SegPos seg_pos(const float4& pw, const float4& dn, int cnt, const Foot& f, float c, float s,
                                 float sc, float ss, float step) {
  SegPos g;
  g.px = fmaf(c, pw.x, fmaf(s, pw.y, f.cx));
  g.py = fmaf(c, pw.y, fmaf(-s, pw.x, f.cy));
  g.pz = pw.z + f.zoff;
  g.dx = fmaf(sc, dn.x, ss * dn.y);
  g.dy = fmaf(sc, dn.y, -ss * dn.x);
  g.dz = step * dn.z;
  const int m = (cnt - 1) >> 1;
  g.k0 = (float)(-m);
  g.k1 = (float)(cnt - 1 - m);
  return g;
}

// Lower bound of the unclamped fast path: a sample computed as
// fma(k, d, p) lies within one rounding (< 2^-20 cell here) of the segment
// between its endpoints, so endpoints at >= 2^-12 keep every sample's floor
// >= 0.
constexpr float kLo = 1.0f / 4096.0f;

// True when every sample of the segment lies inside [kLo, h] on all axes, so
// the sample loop needs no clamps (the samples lie on the line between its
// two ends).
__device__ inline bool seg_inside(const SegPos& g, float hx, float hy, float hz) {
  const float x0 = fmaf(g.k0, g.dx, g.px), y0 = fmaf(g.k0, g.dy, g.py), z0 = fmaf(g.k0, g.dz, g.pz);
  const float x1 = fmaf(g.k1, g.dx, g.px), y1 = fmaf(g.k1, g.dy, g.py), z1 = fmaf(g.k1, g.dz, g.pz);
  return fminf(x0, x1) >= kLo && fmaxf(x0, x1) <= hx && fminf(y0, y1) >= kLo && fmaxf(y0, y1) <= hy &&
         fminf(z0, z1) >= kLo && fmaxf(z0, z1) <= hz;
}

// Coordinate of a sample, clamped into [0, h] where the segment may leave
// the footprint (rounding at its faces, or a box beyond the padded grid,
// whose samples then read or write only padding).
template <bool CLAMP>
__device__ inline float coord(float k, float d, float p, float h) {
  const float x = fmaf(k, d, p);
  return CLAMP ? __builtin_amdgcn_fmed3f(x, 0.0f, h) : x;
}

// ------------------------------------------------------------- forward ---
//
// The workgroup of a (box, angle) stages the rotated box footprint of the
// padded volume in LDS (one coalesced read per cell), then every segment of
// the box gathers its samples from LDS.  The segment's partial sum (Horner
// over its samples from the far end, S <- S r + val with r = exp(-alpha
// step) applied as r_hi + r_lo, times the weight of its first sample) is
// added to its pixel as a 64-bit integer (the default), or written to
// part[angle][rank][ray] for a second kernel that adds, per pixel, the
// partials of its rays in a fixed order (pupil index, then rank).  Either
// way the result does not depend on scheduling.

// Storage of the staged volume footprint: FP32 values, or (for BF16 and FP16
// volumes) one 32-bit word per cell holding the 16-bit values of voxel x
// (low half) and voxel x + 1 (high half), so that a sample reads its 8
// corners as 4 words instead of 8.  Widening a BF16 or FP16 value to FP32 is
// exact, so both layouts give the same sums.
enum { kVolF32 = 0, kVolBF16Pairs = 1, kVolF16Pairs = 2 };

// The x-lerp of the corner pair at word o: v_x + fx (v_{x+1} - v_x), FP32.
// FP16 halves feed the mixed-precision FMA directly (v_fma_mix_f32 widens
// either half of its operands), so the pair costs the same two VALU ops as
// two FP32 values; BF16 halves are widened by a shift and a mask.
template <int FMT>
__device__ inline float lerp_x(const uint32_t* sv, unsigned o, float fx) {
  if constexpr (FMT == kVolF32) {
    const float lo = __uint_as_float(sv[o]), hi = __uint_as_float(sv[o + 1]);
    return fmaf(fx, hi - lo, lo);
  } else if constexpr (FMT == kVolBF16Pairs) {
    const uint32_t w = sv[o];
    const float lo = __uint_as_float(w << 16), hi = __uint_as_float(w & 0xffff0000u);
    return fmaf(fx, hi - lo, lo);
  } else {
    const uint32_t w = sv[o];
    // d = hi - lo straight from the two halves (exact to one FP32 rounding,
    // as a subtraction of the widened values); the compiler folds the
    // product by one and would widen both halves separately first.
    float d;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(w));
    const float lo = (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
    return fmaf(fx, d, lo);
  }
}

// Horner sum over the samples kfirst, kfirst + STRIDE, ..., klast of a
// segment, from the far end: S <- S r + val with r = r_hi + r_lo the
// attenuation over STRIDE samples.
template <int SY, int SZ, bool CLAMP, int FMT, int STRIDE>
__device__ inline float march_forward(const uint32_t* sv, const SegPos& g, float kfirst, float klast, float hx,
                                      float hy, float hz, float r_hi, float r_lo) {
  float S = 0.0f;
  for (float kf = klast; kf >= kfirst; kf -= (float)STRIDE) {
    const float x = coord<CLAMP>(kf, g.dx, g.px, hx);
    const float y = coord<CLAMP>(kf, g.dy, g.py, hy);
    const float z = coord<CLAMP>(kf, g.dz, g.pz, hz);
    const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y), fz = __builtin_amdgcn_fractf(z);
    const unsigned o = __umul24((unsigned)z, SZ) + __umul24((unsigned)y, SY) + (unsigned)x;
    const float c00 = lerp_x<FMT>(sv, o, fx);
    const float c01 = lerp_x<FMT>(sv, o + SY, fx);
    const float c10 = lerp_x<FMT>(sv, o + SZ, fx);
    const float c11 = lerp_x<FMT>(sv, o + SZ + SY, fx);
    const float c0 = fmaf(fy, c01 - c00, c00);
    const float c1 = fmaf(fy, c11 - c10, c10);
    const float val = fmaf(fz, c1 - c0, c0);
    S = fmaf(S, r_hi, fmaf(S, r_lo, val));
  }
  return S;
}

// The same sum, one lane per segment, keeping the LDS words of the current
// cell in registers: a sample in the same cell as the one before reads no
// LDS (the reads are issued only for lanes whose cell changed).
template <int SY, int SZ, bool CLAMP, int FMT>
__device__ inline float march_forward_cached(const uint32_t* sv, const SegPos& g, float hx, float hy, float hz,
                                             float r_hi, float r_lo) {
  constexpr bool F32 = FMT == kVolF32;
  float S = 0.0f;
  unsigned cur = 0xffffffffu;
  uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (float kf = g.k1; kf >= g.k0; kf -= 1.0f) {
    const float x = coord<CLAMP>(kf, g.dx, g.px, hx);
    const float y = coord<CLAMP>(kf, g.dy, g.py, hy);
    const float z = coord<CLAMP>(kf, g.dz, g.pz, hz);
    const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y), fz = __builtin_amdgcn_fractf(z);
    const unsigned o = __umul24((unsigned)z, SZ) + __umul24((unsigned)y, SY) + (unsigned)x;
    if (o != cur) {
      cur = o;
      w[0] = sv[o];
      w[2] = sv[o + SY];
      w[4] = sv[o + SZ];
      w[6] = sv[o + SZ + SY];
      if constexpr (F32) {
        w[1] = sv[o + 1];
        w[3] = sv[o + SY + 1];
        w[5] = sv[o + SZ + 1];
        w[7] = sv[o + SZ + SY + 1];
      }
    }
    float c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (F32) {
        const float lo = __uint_as_float(w[2 * j]), hi = __uint_as_float(w[2 * j + 1]);
        c[j] = fmaf(fx, hi - lo, lo);
      } else if constexpr (FMT == kVolBF16Pairs) {
        const float lo = __uint_as_float(w[2 * j] << 16), hi = __uint_as_float(w[2 * j] & 0xffff0000u);
        c[j] = fmaf(fx, hi - lo, lo);
      } else {
        float d;
        asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(w[2 * j]));
        const float lo = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[2 * j] & 0xffffu));
        c[j] = fmaf(fx, d, lo);
      }
    }
    const float c0 = fmaf(fy, c[1] - c[0], c[0]);
    const float c1 = fmaf(fy, c[3] - c[2], c[2]);
    const float val = fmaf(fz, c1 - c0, c0);
    S = fmaf(S, r_hi, fmaf(S, r_lo, val));
  }
  return S;
}

// March modes of the fixed-point box forward (k_forward_box's MODE).
constexpr int kMarchOne = 1, kMarchPair = 2, kMarchCached = 3;

// Fixed-point forward (the default).  A pixel's value is a sum of segment
// partials pw.w S, each at most (step / n_pupil) n V in magnitude (sample
// weights <= step / n_pupil, attenuation <= 1, trilinear values <= V, the
// volume's largest |value|, n the segment's samples), so the pixel's exact
// sum and every partial sum of it are at most bound = (step / n_pupil)
// pix_samples_max V.  With the power of two scale 2^(61 - e), bound < 2^e,
// every FP32 partial times the scale is exact in FP64 and below 2^61; it is
// rounded to an integer (<= 1/2 off, i.e. <= 2^(e - 62) <= bound 2^-61) and added to the
// pixel's 64-bit integer, which stays below 2^62: integer adds commute, so
// the result does not depend on the order of the atomics.

// vol: the padded working volume, FP32 values or 16-bit pairs (FMT).
// FX = false: partial sums to part[angle][rank][ray] (slots per angle);
// FX = true: fixed-point adds into pfx[angle][pixel].
// MODE: how lanes march a segment.  kMarchOne: one lane, all samples.
// kMarchPair: two neighbouring lanes share a segment, one taking its even
// and the other its odd samples (Horner with r^2 each; the pair's sum is
// S_even + r S_odd); their samples are half a voxel apart, so they often
// read the same LDS words, which the LDS serves as one broadcast.
// kMarchCached: one lane, the current cell's LDS words kept in registers.
template <int B, int FMT, bool FX, int MODE>
__global__ __launch_bounds__(256) void k_forward_box(MarchParams P, BoxParams Bp, const uint32_t* __restrict__ vol,
                                                     float* __restrict__ part, int64_t slots,
                                                     unsigned long long* __restrict__ pfx,
                                                     const unsigned* __restrict__ vmax, double fx_coef) {
  constexpr int SY = Fixed<B>::WXY, SZ = SY * SY, NC = SZ * Fixed<B>::WZ;
  __shared__ uint32_t sv[NC];
  int b, a;
  if (!work_item(Bp.nboxes, Bp.na, Bp.xcd, b, a)) return;
  const double2 cs = P.cs[P.a0 + a];
  const Foot f = footprint(Bp, Bp.box_id[b], cs.x, cs.y, P.cx, P.cy);
  for (int i = threadIdx.x; i < NC; i += blockDim.x) {
    const int z = i / SZ, rem = i - z * SZ, y = rem / SY, x = rem - y * SY;
    uint32_t v = 0u;
    if (x < f.WX && y < f.WY && z < f.WZ)
      v = vol[((int64_t)(f.Z0 + z) * Bp.py + (f.Y0 + y)) * Bp.px + (f.X0 + x)];
    sv[i] = v;
  }
  __syncthreads();
  const float hx = (float)f.WX - 1.001f, hy = (float)f.WY - 1.001f, hz = (float)f.WZ - 1.001f;
  const float c = (float)cs.x, s = (float)cs.y, sc = P.step * c, ss = P.step * s;
  const int s_end = Bp.box_begin[b + 1];
  float* out = part + (int64_t)a * slots;
  double scale = 1.0;
  bool finite = true;
  if constexpr (FX) {
    const unsigned vm = *vmax;
    finite = vm < 0x7f800000u;
    scale = fx_scale(vm, fx_coef);
  }
  unsigned long long* row = pfx + (int64_t)a * Bp.npix;
  const int part_of = MODE == kMarchPair ? (int)(threadIdx.x & 1u) : 0;
  constexpr int LPS = MODE == kMarchPair ? 2 : 1;  // lanes per segment
  for (int si = Bp.box_begin[b] + (int)threadIdx.x / LPS; si < s_end; si += (int)blockDim.x / LPS) {
    const float4 pw = Bp.seg.pw[si], dn = Bp.seg.dn[si];
    const SegPos g = seg_pos(pw, dn, __float_as_int(dn.w), f, c, s, sc, ss, P.step);
    float S;
    if constexpr (MODE == kMarchCached) {
      S = seg_inside(g, hx, hy, hz) ? march_forward_cached<SY, SZ, false, FMT>(sv, g, hx, hy, hz, P.r_hi, P.r_lo)
                                    : march_forward_cached<SY, SZ, true, FMT>(sv, g, hx, hy, hz, P.r_hi, P.r_lo);
    } else if constexpr (MODE == kMarchOne) {
      S = seg_inside(g, hx, hy, hz)
              ? march_forward<SY, SZ, false, FMT, 1>(sv, g, g.k0, g.k1, hx, hy, hz, P.r_hi, P.r_lo)
              : march_forward<SY, SZ, true, FMT, 1>(sv, g, g.k0, g.k1, hx, hy, hz, P.r_hi, P.r_lo);
    } else {
      // this lane's samples: k0 + part_of, then every second one (none if
      // the segment is shorter); both lanes of a pair take the same branch
      const float kfirst = g.k0 + (float)part_of;
      const float klast = kfirst + 2.0f * floorf((g.k1 - kfirst) * 0.5f);
      S = seg_inside(g, hx, hy, hz)
              ? march_forward<SY, SZ, false, FMT, 2>(sv, g, kfirst, klast, hx, hy, hz, P.r2_hi, P.r2_lo)
              : march_forward<SY, SZ, true, FMT, 2>(sv, g, kfirst, klast, hx, hy, hz, P.r2_hi, P.r2_lo);
      const float odd = __shfl_xor(S, 1);
      S = fmaf(odd, P.r_hi, fmaf(odd, P.r_lo, S));
    }
    const float v = pw.w * S;
    if constexpr (FX) {
      // the slot rank * n_rays + pupil * npix + pixel, modulo npix, is the pixel
      if (part_of == 0 && finite && v != 0.0f)
        atomicAdd(row + (unsigned)Bp.seg.idx[si] % (unsigned)Bp.npix,
                  (unsigned long long)__double2ll_rn((double)v * scale));
    } else {
      out[Bp.seg.idx[si]] = v;
    }
  }
}

// Clears the fixed-point projections of a call and the volume maximum.
__global__ void k_fx_clear(unsigned long long* __restrict__ p, int64_t n, unsigned* __restrict__ vmax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
  if (i == 0) *vmax = 0u;
}

// Largest |value| of the padded working volume as FP32 bits (non-negative
// floats order as their bit patterns; a NaN or infinity compares above every
// finite value).
template <int FMT>
__device__ inline unsigned abs_bits(uint32_t w) {
  if constexpr (FMT == kVolF32) {
    return w & 0x7fffffffu;
  } else if constexpr (FMT == kVolBF16Pairs) {
    return max((w << 16) & 0x7fffffffu, w & 0x7fff0000u);
  } else {
    const float lo = (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
    const float hi = (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
    return max(__float_as_uint(lo) & 0x7fffffffu, __float_as_uint(hi) & 0x7fffffffu);
  }
}

template <int FMT>
__global__ __launch_bounds__(256) void k_absmax(const uint32_t* __restrict__ v, int64_t n, unsigned* __restrict__ vmax) {
  unsigned m = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = max(m, abs_bits<FMT>(v[i]));
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(vmax, m);
}

template <typename PT>
__device__ inline void store_proj(PT* p, int64_t i, float x);
template <>
__device__ inline void store_proj<float>(float* p, int64_t i, float x) {
  p[i] = x;
}
template <>
__device__ inline void store_proj<uint16_t>(uint16_t* p, int64_t i, float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    p[i] = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);       // round to nearest even
    p[i] = (uint16_t)(u >> 16);
  }
}
template <>
__device__ inline void store_proj<__half>(__half* p, int64_t i, float x) {
  p[i] = __float2half_rn(x);
}

// Fixed-point projections -> stored projections: the integer over the scale,
// rounded to FP32 (then to BF16 / FP16 on store); all NaN if the volume held
// a NaN or an infinity.
template <typename PT>
__global__ void k_fx_store(const unsigned long long* __restrict__ pfx, PT* __restrict__ proj, int64_t n,
                           const unsigned* __restrict__ vmax, double fx_coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned vm = *vmax;
  const bool finite = vm < 0x7f800000u;
  const float x = finite ? (float)((double)(long long)pfx[i] / fx_scale(vm, fx_coef)) : __uint_as_float(0x7fc00000u);
  store_proj(proj, i, x);
}

template <typename PT>
__global__ void k_reduce_segments(const float* __restrict__ part, const int* __restrict__ nseg,
                                  PT* __restrict__ proj, int npix, int np, int64_t n_rays, int64_t slots,
                                  int na) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)na * npix) return;
  const int a = (int)(i / npix);
  const int pix = (int)(i - (int64_t)a * npix);
  const float* base = part + (int64_t)a * slots;
  float acc = 0.0f;
  for (int j = 0; j < np; ++j) {
    const int64_t r = (int64_t)j * npix + pix;
    const int ns = nseg[r];
    const float* b = base + r;
    // four running sums in a fixed interleave keep four loads in flight;
    // the order is the same on every call
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

// Forward launch arguments beyond the march and box parameters.
struct FwdOut {
  float* part;              // partial sums (fx = false)
  int64_t slots;
  unsigned long long* pfx;  // fixed-point projections (fx = true)
  const unsigned* vmax;
  double fx_coef;
  int mode;                 // march mode (fx = true): kMarchOne, kMarchPair or kMarchCached
};

template <int B, int FMT, bool FX>
static void launch_forward_box_f(dim3 grid, hipStream_t s, const MarchParams& P, const BoxParams& Bp,
                                 const uint32_t* vol, const FwdOut& o) {
  if (FX && o.mode == kMarchCached)
    hipLaunchKernelGGL((k_forward_box<B, FMT, true, kMarchCached>), grid, dim3(256), 0, s, P, Bp, vol, o.part,
                       o.slots, o.pfx, o.vmax, o.fx_coef);
  else if (FX && o.mode == kMarchPair)
    hipLaunchKernelGGL((k_forward_box<B, FMT, true, kMarchPair>), grid, dim3(256), 0, s, P, Bp, vol, o.part, o.slots,
                       o.pfx, o.vmax, o.fx_coef);
  else
    hipLaunchKernelGGL((k_forward_box<B, FMT, FX, kMarchOne>), grid, dim3(256), 0, s, P, Bp, vol, o.part, o.slots,
                       o.pfx, o.vmax, o.fx_coef);
}

template <int B, bool FX>
static void launch_forward_box(dim3 grid, hipStream_t s, const MarchParams& P, const BoxParams& Bp, int fmt,
                               const uint32_t* vol, const FwdOut& o) {
  switch (fmt) {
    case kVolBF16Pairs: launch_forward_box_f<B, kVolBF16Pairs, FX>(grid, s, P, Bp, vol, o); break;
    case kVolF16Pairs: launch_forward_box_f<B, kVolF16Pairs, FX>(grid, s, P, Bp, vol, o); break;
    default: launch_forward_box_f<B, kVolF32, FX>(grid, s, P, Bp, vol, o); break;
  }
}

template <bool FX>
static void launch_forward_box_edge(int edge, dim3 grid, hipStream_t s, const MarchParams& P, const BoxParams& Bp,
                                    int fmt, const uint32_t* vol, const FwdOut& o) {
  switch (edge) {
    case 8: launch_forward_box<8, FX>(grid, s, P, Bp, fmt, vol, o); break;
    case 12: launch_forward_box<12, FX>(grid, s, P, Bp, fmt, vol, o); break;
    default: launch_forward_box<16, FX>(grid, s, P, Bp, fmt, vol, o); break;
  }
}

// Caller volume -> interior of the padded working volume as 16-bit pairs:
// word (z, y, x) holds voxel x (low half) and voxel x + 1 (high half) of the
// padded grid, stored as given (zero in the padding).
__global__ void k_pad_pairs(const uint16_t* __restrict__ vol, uint32_t* __restrict__ vp, int nx, int ny, int nz,
                            int px, int py, int pz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)px * py * pz) return;
  const int x = (int)(i % px), y = (int)((i / px) % py), z = (int)(i / ((int64_t)px * py));
  const int ix = x - kPad, iy = y - kPad, iz = z - kPad;
  uint32_t lo = 0u, hi = 0u;
  if (iy >= 0 && iy < ny && iz >= 0 && iz < nz) {
    const int64_t row = ((int64_t)iz * ny + iy) * nx;
    if (ix >= 0 && ix < nx) lo = vol[row + ix];
    if (ix + 1 >= 0 && ix + 1 < nx) hi = vol[row + ix + 1];
  }
  vp[i] = lo | (hi << 16);
}

// Default forward: every segment adds its partial to its pixel in 64-bit
// fixed point (scale from the volume's largest |value|), then one pass
// rounds the integers to the stored projections.  Variant 2 (below) writes
// FP32 partial sums instead and adds them per pixel in a fixed order.
template <typename PT>
static vam_status forward_box_fx(vam_geometry* h, const MarchParams& P, PT* proj, int na, int fmt, hipStream_t s) {
  const vam_geometry_desc& D = h->desc;
  const int64_t npix = (int64_t)D.n_u * D.n_v;
  if (!h->proj_fx) {
    VAM_HIP_TRY(dev_alloc((void**)&h->proj_fx, (int64_t)D.n_angles * npix * sizeof(int64_t)),
                "allocating the fixed-point projections");
  }
  if (!h->vol_absmax) VAM_HIP_TRY(dev_alloc((void**)&h->vol_absmax, sizeof(unsigned)), "allocating a maximum");
  unsigned long long* pfx = (unsigned long long*)h->proj_fx;
  const int64_t n = (int64_t)na * npix;
  hipLaunchKernelGGL(k_fx_clear, dim3((unsigned)std::max<int64_t>((n + 255) / 256, 1)), dim3(256), 0, s, pfx, n,
                     h->vol_absmax);
  const uint32_t* vol = (const uint32_t*)h->vol_pad;
  const unsigned mb = (unsigned)std::min<int64_t>((h->pad_voxels + 255) / 256, 2048);
  switch (fmt) {
    case kVolBF16Pairs:
      hipLaunchKernelGGL(k_absmax<kVolBF16Pairs>, dim3(mb), dim3(256), 0, s, vol, h->pad_voxels, h->vol_absmax);
      break;
    case kVolF16Pairs:
      hipLaunchKernelGGL(k_absmax<kVolF16Pairs>, dim3(mb), dim3(256), 0, s, vol, h->pad_voxels, h->vol_absmax);
      break;
    default: hipLaunchKernelGGL(k_absmax<kVolF32>, dim3(mb), dim3(256), 0, s, vol, h->pad_voxels, h->vol_absmax);
  }
  const double coef = D.step / D.n_pupil * (double)h->pix_samples_max;
  if (h->n_boxes > 0) {
    const BoxParams Bp = box_params(h, h->seg_fwd, na, h->xcd_forward);
    // the loops are bound by their LDS reads (FP32) or VALU issue (16-bit
    // pairs); keeping the cell's words in registers saves LDS reads for FP32
    // and BF16, while FP16's mixed-precision FMA reads its word directly
    const int mode = h->forward_lanes ? h->forward_lanes : (fmt == kVolF16Pairs ? kMarchOne : kMarchCached);
    const FwdOut o{nullptr, 0, pfx, h->vol_absmax, coef, mode};
    launch_forward_box_edge<true>(h->boxes.B, work_grid(h->n_boxes, na, Bp.xcd), s, P, Bp, fmt, vol, o);
  }
  hipLaunchKernelGGL(k_fx_store<PT>, dim3((unsigned)std::max<int64_t>((n + 255) / 256, 1)), dim3(256), 0, s, pfx,
                     proj, n, h->vol_absmax, coef);
  VAM_HIP_TRY(hipGetLastError(), "launching the fixed-point forward projector");
  return VAM_OK;
}

template <typename PT>
static vam_status forward_box_t(vam_geometry* h, const MarchParams& P0, PT* proj, int na, int fmt, hipStream_t s) {
  if (h->forward_variant != 2) return forward_box_fx(h, P0, proj, na, fmt, s);
  const vam_geometry_desc& D = h->desc;
  const int64_t slots = (int64_t)std::max(h->max_seg_per_ray, 1) * h->n_rays;
  if (!h->seg_part) {
    // partial sums for a chunk of angles, at most 8 GiB (fewer launch tails
    // and reductions than small chunks); if the device cannot hold that
    // much, halve the chunk until the allocation succeeds
    int64_t angles = std::max<int64_t>(1, std::min<int64_t>(D.n_angles, (int64_t(1) << 31) / slots));
    for (;;) {
      const hipError_t e = dev_alloc((void**)&h->seg_part, slots * angles * sizeof(float));
      if (e == hipSuccess) break;
      h->seg_part = nullptr;
      if (e != hipErrorOutOfMemory || angles == 1) return hip_check(e, "allocating segment partial sums");
      (void)hipGetLastError();  // the failed allocation's error is handled here
      angles = (angles + 1) / 2;
    }
    h->seg_part_angles = (int)angles;
  }
  const int npix = D.n_u * D.n_v;
  for (int c0 = 0; c0 < na; c0 += h->seg_part_angles) {
    const int nc = std::min(h->seg_part_angles, na - c0);
    MarchParams P = P0;
    P.a0 = P0.a0 + c0;
    if (h->n_boxes > 0) {
      const BoxParams Bp = box_params(h, h->seg_fwd, nc, h->xcd_forward);
      const FwdOut o{h->seg_part, slots, nullptr, nullptr, 0.0, kMarchOne};
      launch_forward_box_edge<false>(h->boxes.B, work_grid(h->n_boxes, nc, Bp.xcd), s, P, Bp, fmt,
                                     (const uint32_t*)h->vol_pad, o);
    }
    const int64_t n = (int64_t)nc * npix;
    hipLaunchKernelGGL(k_reduce_segments<PT>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->seg_part,
                       h->ray_nseg, proj + (int64_t)c0 * npix, npix, D.n_pupil, h->n_rays, slots, nc);
    VAM_HIP_TRY(hipGetLastError(), "launching the box-tiled forward projector");
  }
  return VAM_OK;
}

// The padded working volume for the box forward: FP32 values (from an FP32
// caller volume) or 16-bit pairs (from a BF16 or FP16 one), in h->vol_pad.
void pad_box_volume(vam_geometry* h, const void* vol, vam_dtype vol_t, hipStream_t s) {
  const vam_geometry_desc& D = h->desc;
  hipLaunchKernelGGL(k_pad_pairs, dim3((unsigned)((h->pad_voxels + 255) / 256)), dim3(256), 0, s,
                     (const uint16_t*)vol, (uint32_t*)h->vol_pad, D.nx, D.ny, D.nz, h->px, h->py, h->pz);
}

vam_status launch_box_forward(vam_geometry* h, const MarchParams& P, void* proj, vam_dtype proj_t, vam_dtype vol_t,
                              int na, hipStream_t s) {
  if (!h->boxes_ready)
    return fail(VAM_ERR_INVALID_ARG, "the box decomposition is not available (a rebuild failed); "
                                     "set the box edge again or create a new geometry");
  const int fmt = vol_t == VAM_BF16 ? kVolBF16Pairs : vol_t == VAM_F16 ? kVolF16Pairs : kVolF32;
  switch (proj_t) {
    case VAM_F32: return forward_box_t(h, P, (float*)proj, na, fmt, s);
    case VAM_BF16: return forward_box_t(h, P, (uint16_t*)proj, na, fmt, s);
    case VAM_F16: return forward_box_t(h, P, (__half*)proj, na, fmt, s);
  }
  return fail(VAM_ERR_INVALID_ARG, "unknown projection dtype");
}

// ------------------------------------------------------------- deposit ---
//
// The deposit adds 8 corner weights per sample into the (box, angle)
// workgroup's LDS footprint in 32-bit fixed point (gfx950 adds 32-bit
// integers in LDS ~45x faster than FP32 and ~2x faster than FP64), then adds
// each touched cell once to its voxel's 64-bit integer (a power-of-two scale
// from the call's largest |projection value|; integer adds commute, so the
// dose is deterministic).  Overflow in LDS is ruled
// out per workgroup: a cell's exact sum is at most bound = n x (step /
// n_pupil) x M, where n is the box's n_supp (the most samples of the box in
// any 4 x 4 x 3 block of lab-frame unit cells, which holds the turned
// support of any voxel), no sample weight exceeds step / n_pupil times |P|,
// and M is the largest |projection value| among the box's segments at this
// angle.  With S = (2^31 - n - 2^12)(1 - 2^-12) / bound, each of the at most
// n adds into a cell rounds a value that is within 2^-12 of exact (the FP32
// run sums of at most a few thousand same-sign terms) to the nearest
// integer, so every partial sum stays below 2^31 in magnitude; the rounding
// error of an add is at most 1/(2S) ~ bound 2^-32.  A non-finite
// projection value makes the whole dose NaN (the workgroups add nothing and
// the dose copy writes NaN).
//
// Run aggregation keeps the 8 corner sums of consecutive samples in one cell
// in registers and adds them to LDS when the cell changes; the sums restart
// through a factor keep in {0, 1} (w <- keep w + q, one FMA) rather than a
// branch, so the loop carries them without register copies.

template <typename PT>
__device__ inline float load_p(const PT* p, int64_t i);
template <>
__device__ inline float load_p<float>(const float* p, int64_t i) {
  return p[i];
}
template <>
__device__ inline float load_p<uint16_t>(const uint16_t* p, int64_t i) {
  return __uint_as_float((uint32_t)p[i] << 16);
}
template <>
__device__ inline float load_p<__half>(const __half* p, int64_t i) {
  return __half2float(p[i]);
}

// Round to the nearest integer, halves upwards (one v_cvt_rpi_i32_f32).
__device__ inline int round_to_int(float v) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

template <int SY, int SZ>
__device__ inline void flush8(int* acc, unsigned cur, const float* w) {
  int* p = (int*)((char*)acc + cur);
  atomicAdd(p, round_to_int(w[0]));
  atomicAdd(p + 1, round_to_int(w[1]));
  atomicAdd(p + SY, round_to_int(w[2]));
  atomicAdd(p + SY + 1, round_to_int(w[3]));
  atomicAdd(p + SZ, round_to_int(w[4]));
  atomicAdd(p + SZ + 1, round_to_int(w[5]));
  atomicAdd(p + SZ + SY, round_to_int(w[6]));
  atomicAdd(p + SZ + SY + 1, round_to_int(w[7]));
}

template <int SY, int SZ, bool CLAMP>
__device__ inline void march_deposit(int* acc, const SegPos& g, float e, float hx, float hy, float hz,
                                     float r_hi, float r_lo) {
  auto cell_bytes = [](float x, float y, float z) {
    return __umul24((unsigned)z, SZ * 4) + __umul24((unsigned)y, SY * 4) + (unsigned)x * 4;
  };
  float w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // byte offset of the cell whose corners w holds, starting at the first
  // sample's (w is zero until its first add)
  unsigned cur = cell_bytes(coord<CLAMP>(g.k0, g.dx, g.px, hx), coord<CLAMP>(g.k0, g.dy, g.py, hy),
                            coord<CLAMP>(g.k0, g.dz, g.pz, hz));
  // exact: a segment has fewer than 2^24 samples
  for (float kf = g.k0; kf <= g.k1; kf += 1.0f) {
    const float x = coord<CLAMP>(kf, g.dx, g.px, hx);
    const float y = coord<CLAMP>(kf, g.dy, g.py, hy);
    const float z = coord<CLAMP>(kf, g.dz, g.pz, hz);
    const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y), fz = __builtin_amdgcn_fractf(z);
    const float z1 = e * fz, z0 = e - z1;
    const float y01 = z0 * fy, y00 = z0 - y01;
    const float y11 = z1 * fy, y10 = z1 - y11;
    const unsigned ob = cell_bytes(x, y, z);
    const bool fl = ob != cur;
    if (fl) flush8<SY, SZ>(acc, cur, w);
    const float keep = fl ? 0.0f : 1.0f;
    cur = ob;
    // w[2j] += yz (1 - fx), w[2j+1] += yz fx, accumulated into w itself
    const float yz[4] = {y00, y01, y10, y11};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      w[2 * j] = fmaf(-yz[j], fx, fmaf(keep, w[2 * j], yz[j]));
      w[2 * j + 1] = fmaf(yz[j], fx, keep * w[2 * j + 1]);
    }
    e = fmaf(e, r_hi, e * r_lo);
  }
  flush8<SY, SZ>(acc, cur, w);  // a segment has at least one sample
}

// acc: the padded dose as 64-bit integers at the scale fx_scale(*pmax,
// dep_coef), pmax the largest |projection value| of the call (FP32 bits;
// a NaN or infinity among them leaves acc untouched: the dose copy then
// writes NaN everywhere).
template <int B, typename PT, int NT>
__global__ __launch_bounds__(NT) void k_back_box(MarchParams P, BoxParams Bp, const PT* __restrict__ proj,
                                                 unsigned long long* __restrict__ acc64,
                                                 const unsigned* __restrict__ pmax, double dep_coef) {
  // slice pitch one word longer than a slice: 3 % faster than SY * SY at
  // edge 12 (the pitch decides which LDS banks the lanes' adds share)
  constexpr int SY = Fixed<B>::WXY, SZ = SY * SY + 1, NC = SZ * Fixed<B>::WZ;
  __shared__ int acc[NC];
  __shared__ unsigned s_pvmax;
  int b, a;
  if (!work_item(Bp.nboxes, Bp.na, Bp.xcd, b, a)) return;
  const unsigned pm = *pmax;
  if (pm >= 0x7f800000u) return;  // a non-finite projection value: the dose is NaN
  const double G = fx_scale(pm, dep_coef);
  const double2 cs = P.cs[P.a0 + a];
  const Foot f = footprint(Bp, Bp.box_id[b], cs.x, cs.y, P.cx, P.cy);
  for (int i = threadIdx.x; i < NC; i += blockDim.x) acc[i] = 0;
  if (threadIdx.x == 0) s_pvmax = 0u;
  __syncthreads();
  const float hx = (float)f.WX - 1.001f, hy = (float)f.WY - 1.001f, hz = (float)f.WZ - 1.001f;
  const int64_t pbase = (int64_t)a * Bp.npix;
  const int s_end = Bp.box_begin[b + 1];
  // the box's largest |projection value| at this angle sets the scale
  float m = 0.0f;
  for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x)
    m = fmaxf(m, fabsf(load_p(proj, pbase + Bp.seg.idx[si])));
  atomicMax(&s_pvmax, __float_as_uint(m));  // non-negative floats order as their bits
  __syncthreads();
  const int nb = Bp.box_supp[b];
  const double bound = (double)nb * Bp.w_coef * (double)__uint_as_float(s_pvmax);
  // capped below FP32's largest value (a smaller S only rounds coarser)
  const float S = bound > 0.0 ? (float)fmin((2147483648.0 - nb - 4096.0) * (1.0 - 1.0 / 4096.0) / bound, 3.0e38)
                              : 1.0f;
  // a cell's integer at the dose scale: raw / S x G, rounded (G a power of two)
  const double toG = G / (double)S;
  const float c = (float)cs.x, s = (float)cs.y, sc = P.step * c, ss = P.step * s;
  for (int si = Bp.box_begin[b] + threadIdx.x; si < s_end; si += blockDim.x) {
    const float pv = load_p(proj, pbase + Bp.seg.idx[si]);
    if (pv == 0.0f) continue;
    const float4 pw = Bp.seg.pw[si], dn = Bp.seg.dn[si];
    const SegPos g = seg_pos(pw, dn, __float_as_int(dn.w), f, c, s, sc, ss, P.step);
    const float e = pw.w * pv * S;  // sample weights in the fixed-point units
    if (seg_inside(g, hx, hy, hz))
      march_deposit<SY, SZ, false>(acc, g, e, hx, hy, hz, P.r_hi, P.r_lo);
    else
      march_deposit<SY, SZ, true>(acc, g, e, hx, hy, hz, P.r_hi, P.r_lo);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NC; i += blockDim.x) {
    const int raw = acc[i];
    if (raw == 0) continue;
    const int z = i / SZ, rem = i - z * SZ, y = rem / SY, x = rem - y * SY;
    if (x >= f.WX || y >= f.WY || z >= f.WZ) continue;
    const int64_t gi = ((int64_t)(f.Z0 + z) * Bp.py + (f.Y0 + y)) * Bp.px + (f.X0 + x);
    atomicAdd(acc64 + gi, (unsigned long long)__double2ll_rn((double)raw * toG));
  }
}

// Largest |value| of the na x npix projections of a call, as FP32 bits
// (a NaN or infinity compares above every finite value).
template <typename PT>
__global__ __launch_bounds__(256) void k_proj_absmax(const PT* __restrict__ proj, int64_t n, unsigned* __restrict__ pmax) {
  unsigned m = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = max(m, __float_as_uint(load_p(proj, i)) & 0x7fffffffu);
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(pmax, m);
}

// Bound on a voxel's dose per unit of the largest |projection value|: per
// angle at most supp_bound samples meet its support, each of weight at most
// step / n_pupil.
double deposit_coef(const vam_geometry* h, int na) {
  return (double)na * (double)std::max<int64_t>(h->supp_bound, 1) * h->desc.step / h->desc.n_pupil;
}

template <int B, typename PT>
static void launch_back_box(vam_geometry* h, const MarchParams& P, const PT* proj, int na, double* acc,
                            hipStream_t s) {
  const BoxParams Bp = box_params(h, h->seg_dep, na, h->xcd_deposit);
  const dim3 grid = work_grid(h->n_boxes, na, Bp.xcd);
  unsigned long long* a64 = (unsigned long long*)acc;
  const unsigned* pm = (const unsigned*)(acc + h->pad_voxels);
  const double coef = deposit_coef(h, na);
  if (h->deposit_threads == 512)
    hipLaunchKernelGGL((k_back_box<B, PT, 512>), grid, dim3(512), 0, s, P, Bp, proj, a64, pm, coef);
  else
    hipLaunchKernelGGL((k_back_box<B, PT, 256>), grid, dim3(256), 0, s, P, Bp, proj, a64, pm, coef);
}

template <typename PT>
static void launch_back_box_t(vam_geometry* h, const MarchParams& P, const PT* proj, int na, double* acc,
                              hipStream_t s) {
  // the largest |projection value| first (its slot was cleared with acc)
  const int64_t n = (int64_t)na * h->desc.n_u * h->desc.n_v;
  hipLaunchKernelGGL(k_proj_absmax<PT>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0, s,
                     proj, n, (unsigned*)(acc + h->pad_voxels));
  switch (h->boxes.B) {
    case 8: launch_back_box<8, PT>(h, P, proj, na, acc, s); break;
    case 12: launch_back_box<12, PT>(h, P, proj, na, acc, s); break;
    default: launch_back_box<16, PT>(h, P, proj, na, acc, s); break;
  }
}

vam_status launch_box_deposit(vam_geometry* h, const MarchParams& P, const void* proj, vam_dtype proj_t, int na,
                              double* acc, hipStream_t s) {
  if (!h->boxes_ready)
    return fail(VAM_ERR_INVALID_ARG, "the box decomposition is not available (a rebuild failed); "
                                     "set the box edge again or create a new geometry");
  if (h->n_boxes == 0) return VAM_OK;
  switch (proj_t) {
    case VAM_F32: launch_back_box_t(h, P, (const float*)proj, na, acc, s); break;
    case VAM_BF16: launch_back_box_t(h, P, (const uint16_t*)proj, na, acc, s); break;
    case VAM_F16: launch_back_box_t(h, P, (const __half*)proj, na, acc, s); break;
  }
  return VAM_OK;
}

}  // namespace vam
