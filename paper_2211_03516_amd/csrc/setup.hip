// Geometry setup: FP64 ray tracing through the projector optics and the
// vial walls, ray-table construction and sample statistics.
//
// Ray tracing follows Sec. 2.1 of Webber et al.: a set of rays per DMD
// pixel, the chief ray fixed by the aperture stop and the others by points
// on the stop; refraction by the vector form of Snell's law at every
// interface; propagation until the far inner wall of the vial.  Interface
// transmission is the unpolarised Fresnel factor of Sec. 2.5.  Projector
// models: ideal thin lens at the stop (Sec. 2.6.1) and a telecentric relay
// (Sec. 2.6.2).  Everything here runs once per geometry, in FP64.

#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "vam_internal.h"

namespace vam {

static thread_local std::string g_last_error;

vam_status fail(vam_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

void clear_error() { g_last_error.clear(); }

vam_status hip_check(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(VAM_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
  return fail(VAM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool valid_handle(const vam_geometry* h) { return h && h->magic == kMagic; }

// Allocation-failure injection (vam_debug_fail_allocations): the countdown
// reaches zero at the allocation that is made to fail.
static int g_fail_alloc = 0;

hipError_t dev_alloc(void** p, size_t bytes) {
  if (g_fail_alloc > 0 && --g_fail_alloc == 0) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

// ------------------------------------------------------------ device math --

struct TraceParams {
  int nu, nv, np;
  double pitch_u, pitch_v;
  int thin_lens;
  double focus, pupil;
  double r_out, r_in;
  double n_air, n_glass, n_resin;
  int matched, fresnel;
  double alpha, step;
  int nx, ny, nz;
  const double* pupil_xy;  // device, may be null
};

struct D3 {
  double x, y, z;
};

__device__ inline D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ inline D3 add(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline D3 scale(D3 a, double s) { return d3(a.x * s, a.y * s, a.z * s); }
__device__ inline double dot3(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Parameter where the line o + t d enters the cylinder x^2 + y^2 = R^2:
// the smaller root of |o_xy + t d_xy|^2 = R^2, from the half-b quadratic in
// its cancellation-free form.  false when the line misses or only touches.
__device__ bool cylinder_entry(D3 o, D3 d, double R, double* t) {
  double a = d.x * d.x + d.y * d.y;
  double hb = o.x * d.x + o.y * d.y;
  double c = o.x * o.x + o.y * o.y - R * R;
  double disc = hb * hb - a * c;
  if (!(disc > 0.0) || !(a > 0.0)) return false;
  double q = -(hb + copysign(sqrt(disc), hb));
  double r1 = q / a;
  double r2 = c / q;
  *t = fmin(r1, r2);
  return true;
}

// Refraction of unit direction d at a wall whose unit normal n points back
// into the incident medium.  Writes the transmitted direction and the
// unpolarised Fresnel power transmission.  false on total internal
// reflection (impossible here: indices grow inward).
__device__ bool refract_wall(D3 d, D3 n, double n1, double n2, int fresnel,
                             D3* out, double* T) {
  double ci = -dot3(n, d);
  double eta = n1 / n2;
  double k = 1.0 - eta * eta * (1.0 - ci * ci);
  if (k < 0.0) return false;
  double ct = sqrt(k);
  *out = add(scale(d, eta), scale(n, eta * ci - ct));
  if (fresnel) {
    double rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct);
    double rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct);
    *T = 1.0 - 0.5 * (rs * rs + rp * rp);
  } else {
    *T = 1.0;
  }
  return true;
}

__device__ inline D3 outward_normal(D3 x) {
  double r = sqrt(x.x * x.x + x.y * x.y);
  return d3(x.x / r, x.y / r, 0.0);
}

// One thread per ray r = (j * nv + v) * nu + u.
__global__ void k_trace(TraceParams P, int64_t n_rays, RayRec* rays, double* ray64) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  int u = (int)(r % P.nu);
  int v = (int)((r / P.nu) % P.nv);
  int j = (int)(r / ((int64_t)P.nu * P.nv));

  // pixel image point on the focus plane and the pupil point
  D3 q = d3((u - 0.5 * (P.nu - 1)) * P.pitch_u, 0.0, (v - 0.5 * (P.nv - 1)) * P.pitch_v);
  double rx = 0.0, ry = 0.0;
  if (P.pupil_xy) {
    rx = P.pupil_xy[2 * j];
    ry = P.pupil_xy[2 * j + 1];
  }
  D3 d;
  if (P.thin_lens) {
    D3 w = d3(q.x - P.pupil * rx, q.y + P.focus, q.z - P.pupil * ry);
    d = scale(w, 1.0 / sqrt(dot3(w, w)));
  } else {
    double sx = P.pupil * rx, sz = P.pupil * ry;
    d = d3(sx, sqrt(1.0 - sx * sx - sz * sz), sz);
  }

  bool hit = false;
  D3 e = q, dr = d;
  double T1 = 1.0, T2 = 1.0, t;
  if (P.matched) {
    if (cylinder_entry(q, d, P.r_in, &t)) {
      e = add(q, scale(d, t));
      hit = true;
    }
  } else if (cylinder_entry(q, d, P.r_out, &t)) {
    D3 x1 = add(q, scale(d, t));
    D3 dg;
    if (refract_wall(d, outward_normal(x1), P.n_air, P.n_glass, P.fresnel, &dg, &T1) &&
        cylinder_entry(x1, dg, P.r_in, &t) && t > 0.0) {
      e = add(x1, scale(dg, t));
      hit = refract_wall(dg, outward_normal(e), P.n_glass, P.n_resin, P.fresnel, &dr, &T2);
    }
  }

  double L = 0.0, K = 0.0, w = 0.0;
  if (hit) {
    // far inner wall: the second root of |e_xy + L dr_xy| = R with e on it
    L = -2.0 * (e.x * dr.x + e.y * dr.y) / (dr.x * dr.x + dr.y * dr.y);
    K = floor(L / P.step + 0.5);
    if (K < 1.0) hit = false;
    else w = T1 * T2 / P.np;
  }

  double* o = ray64 + r * kRay64Fields;
  o[0] = e.x; o[1] = e.y; o[2] = e.z;
  o[3] = dr.x; o[4] = dr.y; o[5] = dr.z;
  o[6] = hit ? L : 0.0;
  o[7] = hit ? K : 0.0;
  o[8] = hit ? w : 0.0;
  o[9] = T1; o[10] = T2;
  o[11] = hit ? 1.0 : 0.0;

  RayRec rec;
  memset(&rec, 0, sizeof rec);
  if (hit) {
    int64_t Ki = (int64_t)K;
    double half = 0.5 * K * P.step;
    D3 m = add(e, scale(dr, half));
    rec.mx = m.x;
    rec.my = m.y;
    rec.dx = dr.x;
    rec.dy = dr.y;
    double gz = m.z + 0.5 * (P.nz - 1) + kPad;
    rec.gz = (float)gz;
    rec.dz = (float)dr.z;
    rec.cw = (float)(w * P.step * exp(-P.alpha * half));
    rec.K = (int32_t)Ki;
    // samples whose padded z coordinate lies in [0.5, nz + 2.5]: a superset
    // of those whose stencil touches the grid, (1, nz + 2) in padded units
    int64_t k_lo = 0, k_hi = Ki;
    if (dr.z != 0.0) {
      double ta = (0.5 - gz) / dr.z;
      double tb = (P.nz + 2.5 - gz) / dr.z;
      double lo = fmin(ta, tb), hi = fmax(ta, tb);
      // t_k = (k + 1/2 - K/2) step  <=>  k = t / step - 1/2 + K/2
      double klo = ceil(lo / P.step - 0.5 + 0.5 * K);
      double khi = floor(hi / P.step - 0.5 + 0.5 * K) + 1.0;
      k_lo = (int64_t)fmax(0.0, fmin(klo, K));
      k_hi = (int64_t)fmax(0.0, fmin(khi, K));
    } else if (!(gz >= 0.5 && gz <= P.nz + 2.5)) {
      k_hi = 0;
    }
    int64_t n = k_hi > k_lo ? k_hi - k_lo : 0;
    rec.k0 = (int32_t)k_lo;
    rec.n = (int32_t)n;
    rec.t0 = (float)((k_lo + 0.5 - 0.5 * K) * P.step);
  }
  rays[r] = rec;
}

// Samples whose anti-aliasing stencil touches the grid, summed over rays and
// the given angles: per axis the open interval -1 < g < n in unpadded grid
// coordinates, intersected, and the integer k inside counted exactly.
__global__ void k_count(TraceParams P, int64_t n_rays, const double* ray64,
                        const double2* cs, int n_angles, unsigned long long* total) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long cnt = 0;
  if (r < n_rays) {
    const double* o = ray64 + r * kRay64Fields;
    if (o[11] != 0.0) {
      double K = o[7];
      double cx = 0.5 * (P.nx - 1), cy = 0.5 * (P.ny - 1), cz = 0.5 * (P.nz - 1);
      for (int a = 0; a < n_angles; ++a) {
        double c = cs[a].x, s = cs[a].y;
        // volume-frame entry point and direction; s_k = (k + 1/2) step
        double ex = c * o[0] + s * o[1] + cx, ey = -s * o[0] + c * o[1] + cy, ez = o[2] + cz;
        double dx = c * o[3] + s * o[4], dy = -s * o[3] + c * o[4], dz = o[5];
        double lo = -1e300, hi = 1e300;
        double gs[3] = {ex, ey, ez}, ds[3] = {dx, dy, dz};
        double ns[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
        bool empty = false;
        for (int ax = 0; ax < 3; ++ax) {
          if (ds[ax] == 0.0) {
            if (!(gs[ax] > -1.0 && gs[ax] < ns[ax])) empty = true;
            continue;
          }
          double ta = (-1.0 - gs[ax]) / ds[ax], tb = (ns[ax] - gs[ax]) / ds[ax];
          lo = fmax(lo, fmin(ta, tb));
          hi = fmin(hi, fmax(ta, tb));
        }
        if (empty || !(hi > lo)) continue;
        // k with lo < (k + 1/2) step < hi
        double klo = floor(lo / P.step - 0.5) + 1.0;
        double khi = ceil(hi / P.step - 0.5) - 1.0;
        klo = fmax(klo, 0.0);
        khi = fmin(khi, K - 1.0);
        if (khi >= klo) cnt += (unsigned long long)(khi - klo + 1.0);
      }
    }
  }
  // wave reduction, one atomic per wave
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(total, cnt);
}

static TraceParams make_params(const vam_geometry* h, const double* pupil_dev) {
  const vam_geometry_desc& D = h->desc;
  TraceParams P;
  P.nu = D.n_u;
  P.nv = D.n_v;
  P.np = D.n_pupil;
  P.pitch_u = D.pitch_u;
  P.pitch_v = D.pitch_v;
  P.thin_lens = D.projector == VAM_THIN_LENS;
  P.focus = D.focus_distance;
  P.pupil = D.pupil;
  P.r_out = D.r_outer;
  P.r_in = D.r_inner;
  P.n_air = D.n_air;
  P.n_glass = D.n_glass;
  P.n_resin = D.n_resin;
  P.matched = D.r_outer == D.r_inner;
  P.fresnel = !(D.flags & VAM_NO_FRESNEL);
  P.alpha = D.alpha;
  P.step = D.step;
  P.nx = D.nx;
  P.ny = D.ny;
  P.nz = D.nz;
  P.pupil_xy = pupil_dev;
  return P;
}

static vam_status validate(const vam_geometry_desc* d) {
  if (!d) return fail(VAM_ERR_INVALID_ARG, "descriptor is NULL");
  auto bad = [](const char* what) { return fail(VAM_ERR_INVALID_ARG, "invalid descriptor: %s", what); };
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > 2048 || d->ny > 2048 || d->nz > 2048)
    return bad("volume size must be in [1, 2048]");
  if (d->n_u < 1 || d->n_v < 1 || d->n_u > 8192 || d->n_v > 8192)
    return bad("pixel counts must be in [1, 8192]");
  if (!(d->pitch_u > 0) || !(d->pitch_v > 0) || !std::isfinite(d->pitch_u) || !std::isfinite(d->pitch_v))
    return bad("pixel pitch must be finite and > 0");
  if (d->n_angles < 1 || d->n_angles > 65535) return bad("n_angles must be in [1, 65535]");
  if (d->angles_rad)
    for (int a = 0; a < d->n_angles; ++a)
      if (!std::isfinite(d->angles_rad[a])) return bad("angle is not finite");
  if (d->projector != VAM_TELECENTRIC && d->projector != VAM_THIN_LENS) return bad("unknown projector");
  if (d->n_pupil < 1 || d->n_pupil > 1024) return bad("n_pupil must be in [1, 1024]");
  if (!d->pupil_xy && d->n_pupil != 1) return bad("pupil_xy is NULL but n_pupil > 1");
  if (d->pupil_xy)
    for (int j = 0; j < d->n_pupil; ++j) {
      double x = d->pupil_xy[2 * j], y = d->pupil_xy[2 * j + 1];
      if (!std::isfinite(x) || !std::isfinite(y) || x * x + y * y > 1.0 + 1e-12)
        return bad("pupil point outside the unit disk");
    }
  if (!(d->pupil >= 0) || !std::isfinite(d->pupil)) return bad("pupil must be finite and >= 0");
  if (d->projector == VAM_TELECENTRIC && !(d->pupil < 1.0)) return bad("telecentric pupil (a sine) must be < 1");
  if (!(d->r_inner > 0) || !(d->r_outer >= d->r_inner) || !std::isfinite(d->r_outer))
    return bad("vial radii need r_outer >= r_inner > 0");
  if (d->projector == VAM_THIN_LENS && !(d->focus_distance > d->r_outer) )
    return bad("thin-lens focus distance must exceed r_outer (lens outside the vial)");
  if (!(d->n_air >= 1) || !(d->n_glass >= 1) || !(d->n_resin >= 1) || !std::isfinite(d->n_air) ||
      !std::isfinite(d->n_glass) || !std::isfinite(d->n_resin))
    return bad("refractive indices must be finite and >= 1");
  if (!(d->alpha >= 0) || !std::isfinite(d->alpha)) return bad("alpha must be finite and >= 0");
  if (!(d->step > 0) || !std::isfinite(d->step)) return bad("step must be finite and > 0");
  if (!(2.0 * d->r_inner / d->step < 1e6)) return bad("more than 1e6 samples per ray (2 r_inner / step)");
  if (!(d->step >= 1e-3)) return bad("step must be >= 0.001");
  if (d->flags & ~(uint32_t)VAM_NO_FRESNEL) return bad("unknown flag bits");
  if ((int64_t)d->n_u * d->n_v * d->n_pupil >= 0x7fffffffLL) return bad("n_u n_v n_pupil must be below 2^31");
  return VAM_OK;
}

static void free_handle(vam_geometry* h) {
  if (!h) return;
  for (int i = 0; i < 4; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  free_boxes(h);
  free_gather(h);
  void* ptrs[] = {h->rays, h->ray64, h->angle_cs, h->vol_pad, h->dose_pad64,
                  h->resid, h->grad, h->dose_tmp, h->loss_part, h->proj_fx, h->vol_absmax};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->magic = 0;
  delete h;
}

}  // namespace vam

using namespace vam;

extern "C" {

int32_t vam_version(void) { return 10000; }

const char* vam_last_error(void) { return g_last_error.c_str(); }

vam_status vam_setup_geometry(const vam_geometry_desc* desc, hipStream_t stream,
                              vam_geometry_t* out) {
  clear_error();
  if (!out) return fail(VAM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  vam_status st = validate(desc);
  if (st != VAM_OK) return st;

  vam_geometry* h = new (std::nothrow) vam_geometry();
  if (!h) return fail(VAM_ERR_OUT_OF_MEMORY, "host allocation failed");
  h->magic = kMagic;
  h->desc = *desc;
  h->adjoint_variant = 0;
  h->seg_order = 11;  // pixel classes (u mod 3, v mod 2), length-sorted runs (fastest measured)
  h->seg_order_fwd = 16;  // ray order, then the box by length in steps of two samples (fastest measured)
  h->deposit_threads = 256;
  h->xcd_deposit = 8;  // XCD-aware deposit order, angles in blocks of 8 (fastest measured)
  h->xcd_forward = 16;  // the same for the forward, in blocks of 16: its segment records come from the XCD's L2
  h->forward_lanes = 0;  // by volume format: cached cell words for FP32 and BF16, one lane for FP16 (fastest measured)
  h->angles.resize(desc->n_angles);
  for (int a = 0; a < desc->n_angles; ++a)
    h->angles[a] = desc->angles_rad ? desc->angles_rad[a] : 2.0 * M_PI * a / desc->n_angles;
  h->pupil.assign(2 * desc->n_pupil, 0.0);
  if (desc->pupil_xy) std::memcpy(h->pupil.data(), desc->pupil_xy, 2 * desc->n_pupil * sizeof(double));
  h->desc.angles_rad = nullptr;
  h->desc.pupil_xy = nullptr;
  h->n_rays = (int64_t)desc->n_u * desc->n_v * desc->n_pupil;
  h->px = desc->nx + 2 * kPad;
  h->py = desc->ny + 2 * kPad;
  h->pz = desc->nz + 2 * kPad;
  h->pad_voxels = (int64_t)h->px * h->py * h->pz;

  auto cleanup = [&](vam_status s) {
    free_handle(h);
    return s;
  };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return cleanup(hip_check(e, "hipGetDevice"));

  double* pupil_dev = nullptr;
  unsigned long long* count_dev = nullptr;
  std::vector<double2> cs(desc->n_angles);
  for (int a = 0; a < desc->n_angles; ++a) cs[a] = make_double2(cos(h->angles[a]), sin(h->angles[a]));

#define SETUP_TRY(expr, what)                        \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) {                          \
      if (pupil_dev) (void)hipFree(pupil_dev);       \
      if (count_dev) (void)hipFree(count_dev);       \
      return cleanup(hip_check(e_, what));           \
    }                                                \
  } while (0)

  for (int i = 0; i < 4; ++i) SETUP_TRY(hipEventCreate(&h->ev[i]), "creating events");
  SETUP_TRY(dev_alloc((void**)&h->rays, h->n_rays * sizeof(RayRec)), "allocating the ray table");
  SETUP_TRY(dev_alloc((void**)&h->ray64, h->n_rays * kRay64Fields * sizeof(double)), "allocating FP64 rays");
  SETUP_TRY(dev_alloc((void**)&h->angle_cs, desc->n_angles * sizeof(double2)), "allocating angles");
  SETUP_TRY(dev_alloc((void**)&h->vol_pad, h->pad_voxels * sizeof(float)), "allocating the padded volume");
  SETUP_TRY(dev_alloc((void**)&pupil_dev, h->pupil.size() * sizeof(double)), "allocating the pupil table");
  SETUP_TRY(dev_alloc((void**)&count_dev, sizeof(unsigned long long)), "allocating a counter");
  SETUP_TRY(hipMemcpyAsync(pupil_dev, h->pupil.data(), h->pupil.size() * sizeof(double),
                           hipMemcpyHostToDevice, stream), "copying the pupil table");
  SETUP_TRY(hipMemcpyAsync(h->angle_cs, cs.data(), cs.size() * sizeof(double2),
                           hipMemcpyHostToDevice, stream), "copying angles");
  SETUP_TRY(hipMemsetAsync(count_dev, 0, sizeof(unsigned long long), stream), "clearing a counter");

  TraceParams P = make_params(h, desc->pupil_xy ? pupil_dev : nullptr);
  int threads = 256;
  int64_t blocks = (h->n_rays + threads - 1) / threads;
  hipLaunchKernelGGL(k_trace, dim3((unsigned)blocks), dim3(threads), 0, stream, P, h->n_rays, h->rays, h->ray64);
  SETUP_TRY(hipGetLastError(), "launching the ray tracer");
  hipLaunchKernelGGL(k_count, dim3((unsigned)blocks), dim3(threads), 0, stream, P, h->n_rays, h->ray64,
                     h->angle_cs, desc->n_angles, count_dev);
  SETUP_TRY(hipGetLastError(), "launching the sample counter");

  unsigned long long total = 0;
  SETUP_TRY(hipMemcpyAsync(&total, count_dev, sizeof total, hipMemcpyDeviceToHost, stream), "reading the count");
  SETUP_TRY(hipStreamSynchronize(stream), "synchronising setup");
  h->samples_per_pass = (int64_t)total;

  // rays that reach the resin
  std::vector<double> hitflags;
  {
    std::vector<double> r64(h->n_rays * kRay64Fields);
    SETUP_TRY(hipMemcpy(r64.data(), h->ray64, r64.size() * sizeof(double), hipMemcpyDeviceToHost),
              "reading the FP64 rays");
    int64_t hits = 0;
    for (int64_t r = 0; r < h->n_rays; ++r) hits += r64[r * kRay64Fields + 11] != 0.0;
    h->rays_hit = hits;
  }
  (void)hipFree(pupil_dev);
  (void)hipFree(count_dev);
  pupil_dev = nullptr;
  count_dev = nullptr;
  {
    vam_status bs = build_boxes(h, stream);
    if (bs != VAM_OK) {
      free_handle(h);
      return bs;
    }
  }
#undef SETUP_TRY
  *out = h;
  return VAM_OK;
}

vam_status vam_destroy_geometry(vam_geometry_t h) {
  clear_error();
  if (!h) return VAM_OK;
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  free_handle(h);
  return VAM_OK;
}

vam_status vam_ray_table_stats(vam_geometry_t h, int64_t* rays_hit, int64_t* samples_per_pass) {
  clear_error();
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  if (rays_hit) *rays_hit = h->rays_hit;
  if (samples_per_pass) *samples_per_pass = h->samples_per_pass;
  return VAM_OK;
}

vam_status vam_export_rays(vam_geometry_t h, double* out) {
  clear_error();
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  if (!out) return fail(VAM_ERR_INVALID_ARG, "out is NULL");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  VAM_HIP_TRY(hipMemcpy(out, h->ray64, h->n_rays * kRay64Fields * sizeof(double), hipMemcpyDeviceToHost),
              "copying rays to the host");
  return VAM_OK;
}

vam_status vam_set_variant(vam_geometry_t h, int32_t op, int32_t variant) {
  clear_error();
  if (!valid_handle(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live geometry handle");
  if (op == 0) {
    if (variant < 0 || variant > 2) return fail(VAM_ERR_INVALID_ARG, "unknown forward variant %d", variant);
    h->forward_variant = variant;
  } else if (op == 1) {
    if (variant < 0 || variant > 2) return fail(VAM_ERR_INVALID_ARG, "unknown deposit variant %d", variant);
    h->adjoint_variant = variant;
  } else if (op == 2 || op == 4 || op == 7) {
    if (op == 2 && !supported_box_edge(variant))
      return fail(VAM_ERR_INVALID_ARG, "box edge %d is not one of 8, 12, 16", variant);
    if (op != 2 && (variant < 0 || variant > 16))
      return fail(VAM_ERR_INVALID_ARG, "segment order must be in [0, 16]");
    VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    VAM_HIP_TRY(hipDeviceSynchronize(), "synchronising before rebuilding boxes");
    (op == 2 ? h->box_edge : op == 4 ? h->seg_order : h->seg_order_fwd) = variant;
    return build_boxes(h, nullptr);
  } else if (op == 5) {
    if (variant != 256 && variant != 512) return fail(VAM_ERR_INVALID_ARG, "deposit workgroup size must be 256 or 512");
    h->deposit_threads = variant;
  } else if (op == 8 || op == 9) {
    if (variant < 0 || variant > 4096) return fail(VAM_ERR_INVALID_ARG, "angle block must be in [0, 4096]");
    (op == 8 ? h->xcd_deposit : h->xcd_forward) = variant;
  } else if (op == 10) {
    if (variant < 0 || variant > 3) return fail(VAM_ERR_INVALID_ARG, "forward march mode must be 0, 1, 2 or 3");
    h->forward_lanes = variant;
  } else {
    return fail(VAM_ERR_INVALID_ARG, "unknown operator %d", op);
  }
  return VAM_OK;
}

vam_status vam_debug_fail_allocations(int32_t n) {
  clear_error();
  if (n < 0) return fail(VAM_ERR_INVALID_ARG, "n must be >= 0");
  g_fail_alloc = n;
  return VAM_OK;
}

}  // extern "C"
