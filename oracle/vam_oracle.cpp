// FP64 CPU oracle for the 3D ray-traced tomographic VAM projector pair.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// HIP library is checked against.  Only the test suite, the smoke check and
// the benchmark's CPU-baseline leg may load it.  It shares no code, header,
// table or constant with the HIP library: its own descriptor struct, its own
// tracing, sampling and interpolation, written straight from the paper.
//
// What it computes (Webber et al., "Versatile volumetric additive
// manufacturing with 3D ray tracing"):
//   * rays per DMD pixel, chief ray set by the aperture stop, non-chief rays
//     from points on the stop (Sec. 2.1; ideal thin lens at the stop,
//     Sec. 2.6.1; telecentric relay, Sec. 2.6.2);
//   * vector Snell refraction at the air-glass and glass-resin vial walls,
//     stopping at the far inner wall (Sec. 2.1);
//   * anti-aliasing weights (1-dx)(1-dy)(1-dz) over the voxels around each
//     ray sample (Sec. 2.2, "Anti-aliasing");
//   * projection = weighted sum of voxel values along every ray of a pixel,
//     for every angle (Sec. 2.4);
//   * dose = pixel intensity x anti-aliasing weight x Fresnel transmission x
//     Beer-Lambert transmission, summed over rays and angles (Sec. 2.5).
//
// Readings where the paper is silent (each is listed in the design notes):
//   * the projection carries the same Fresnel and Beer-Lambert factors as the
//     dose, so that projection and dose are exact transposes; the paper's
//     plain voxel sum is the alpha = 0, T = 1 special case;
//   * samples at fixed step ds from the resin entry, s_k = (k + 1/2) ds,
//     K = floor(L/ds + 1/2), each weighted by ds; attenuation exp(-alpha s_k)
//     at the sample;
//   * the two-voxel weight formula is the trilinear tent over the 8 voxel
//     centres around the sample; voxels outside the grid read as 0 and
//     receive nothing;
//   * each of the n_pupil rays of a pixel carries 1/n_pupil of its power;
//   * unpolarised Fresnel transmission at both refracting interfaces;
//   * the vial turns by +theta about +z: volume-frame point = Rz(-theta) lab.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

extern "C" {

// Geometry, lengths in voxels.  Lab frame: vial axis +z through the origin,
// light travels +y, focus plane y = 0 at the rotation axis.
struct OracleGeometry {
  int32_t nx, ny, nz;       // volume [z][y][x], x fastest
  int32_t nu, nv;           // DMD pixels, projection [angle][v][u]
  int32_t n_angles;
  int32_t projector;        // 0 telecentric, 1 ideal thin lens at the stop
  int32_t n_pupil;
  int32_t flags;            // bit 0: no Fresnel loss (T = 1)
  int32_t reserved;
  double pitch_u, pitch_v;  // pixel pitch on the focus plane
  double focus;             // thin lens: lens (= stop) plane at y = -focus
  double pupil;             // thin lens: stop radius; telecentric: sin(half divergence)
  double r_outer, r_inner;  // vial radii; equal radii = index-matched, no walls
  double n_air, n_glass, n_resin;
  double alpha;             // absorption per voxel length in the resin
  double step;              // sample spacing along the ray
  const double* angles;     // [n_angles] radians, or NULL for 2*pi*a/n_angles
  const double* pupil_xy;   // [n_pupil][2] points in the unit disk, or NULL
};

// Per-ray record, all FP64.
enum {
  R_O = 0,      // point on the air ray (the pixel's image point Q), 3
  R_D0 = 3,     // air direction, 3
  R_X1 = 6,     // outer-wall entry point, 3
  R_D1 = 9,     // direction in the glass, 3
  R_E = 12,     // resin entry point, 3
  R_DR = 15,    // direction in the resin, 3
  R_T1 = 18, R_T2 = 19, R_L = 20, R_K = 21, R_W = 22, R_HIT = 23,
  R_COS1 = 24, R_COS2 = 25,
  R_SIZE = 26
};

int oracle_record_size(void) { return R_SIZE; }

// ---------------------------------------------------------------- optics --

// Unpolarised Fresnel transmission from medium n1 into n2 for incidence
// cosine cos_i and transmission cosine cos_t: T = 1 - (rs^2 + rp^2) / 2.
double oracle_fresnel(double n1, double n2, double cos_i, double cos_t,
                      double* rs_out, double* rp_out) {
  double rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
  double rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
  if (rs_out) *rs_out = rs;
  if (rp_out) *rp_out = rp;
  return 1.0 - 0.5 * (rs * rs + rp * rp);
}

// Vector form of Snell's law.  `nrm` is the unit surface normal on the
// incident side, `d` the unit incident direction.  Returns 0 and the
// refracted unit direction, or -1 on total internal reflection.
int oracle_refract(double n1, double n2, const double* d, const double* nrm,
                   double* out, double* cos_i_out, double* cos_t_out) {
  double cos_i = -(nrm[0] * d[0] + nrm[1] * d[1] + nrm[2] * d[2]);
  double eta = n1 / n2;
  double k = 1.0 - eta * eta * (1.0 - cos_i * cos_i);
  if (k < 0.0) return -1;
  double cos_t = std::sqrt(k);
  for (int i = 0; i < 3; ++i) out[i] = eta * d[i] + (eta * cos_i - cos_t) * nrm[i];
  if (cos_i_out) *cos_i_out = cos_i;
  if (cos_t_out) *cos_t_out = cos_t;
  return 0;
}

// Both parameters t at which the line o + t d meets the infinite cylinder
// x^2 + y^2 = R^2 (axis +z).  Uses the cancellation-free form of the
// quadratic.  Returns 0 when the line misses or touches it (disc <= 0).
int oracle_cylinder_roots(const double* o, const double* d, double R,
                          double* t_lo, double* t_hi) {
  double a = d[0] * d[0] + d[1] * d[1];
  double b = 2.0 * (o[0] * d[0] + o[1] * d[1]);
  double c = o[0] * o[0] + o[1] * o[1] - R * R;
  double disc = b * b - 4.0 * a * c;
  if (!(disc > 0.0) || a == 0.0) return 0;
  double sq = std::sqrt(disc);
  double q = -0.5 * (b + (b >= 0.0 ? sq : -sq));
  double r1 = q / a, r2 = c / q;
  *t_lo = std::min(r1, r2);
  *t_hi = std::max(r1, r2);
  return 1;
}

static void radial_normal(const double* x, double* n) {
  double r = std::sqrt(x[0] * x[0] + x[1] * x[1]);
  n[0] = x[0] / r;
  n[1] = x[1] / r;
  n[2] = 0.0;
}

// Air ray of pixel (u, v) and pupil point j: a point on the line (the image
// point Q on the focus plane) and the unit direction.
void oracle_air_ray(const OracleGeometry* g, int u, int v, int j, double* o,
                    double* d) {
  double Q[3] = {(u - 0.5 * (g->nu - 1)) * g->pitch_u, 0.0,
                 (v - 0.5 * (g->nv - 1)) * g->pitch_v};
  double rx = 0.0, ry = 0.0;
  if (g->pupil_xy) {
    rx = g->pupil_xy[2 * j];
    ry = g->pupil_xy[2 * j + 1];
  }
  if (g->projector == 1) {
    // ideal lens at the stop: every ray of the pixel leaves its stop point
    // and is imaged onto Q; the chief ray crosses the stop centre.
    double P[3] = {g->pupil * rx, -g->focus, g->pupil * ry};
    double len = 0.0;
    for (int i = 0; i < 3; ++i) {
      d[i] = Q[i] - P[i];
      len += d[i] * d[i];
    }
    len = std::sqrt(len);
    for (int i = 0; i < 3; ++i) d[i] /= len;
  } else {
    // telecentric: chief ray along +y, stop points give direction cosines
    // spread uniformly over a disk of radius sin(half divergence).
    double s = g->pupil;
    d[0] = s * rx;
    d[2] = s * ry;
    d[1] = std::sqrt(1.0 - d[0] * d[0] - d[2] * d[2]);
  }
  for (int i = 0; i < 3; ++i) o[i] = Q[i];
}

// Trace one ray through the vial to the far inner wall.
void oracle_trace_ray(const OracleGeometry* g, int u, int v, int j,
                      double* rec) {
  for (int i = 0; i < R_SIZE; ++i) rec[i] = 0.0;
  double* o = rec + R_O;
  double* d0 = rec + R_D0;
  oracle_air_ray(g, u, v, j, o, d0);
  bool fresnel = !(g->flags & 1);
  double e[3], dr[3], T1 = 1.0, T2 = 1.0;
  double tl, th;
  if (g->r_outer == g->r_inner) {
    // index-matched: straight through, no walls
    if (!oracle_cylinder_roots(o, d0, g->r_inner, &tl, &th)) return;
    for (int i = 0; i < 3; ++i) {
      e[i] = o[i] + tl * d0[i];
      dr[i] = d0[i];
      rec[R_X1 + i] = e[i];
      rec[R_D1 + i] = d0[i];
    }
  } else {
    if (!oracle_cylinder_roots(o, d0, g->r_outer, &tl, &th)) return;
    double* x1 = rec + R_X1;
    for (int i = 0; i < 3; ++i) x1[i] = o[i] + tl * d0[i];
    double n1[3];
    radial_normal(x1, n1);
    double* d1 = rec + R_D1;
    double ci, ct;
    if (oracle_refract(g->n_air, g->n_glass, d0, n1, d1, &ci, &ct)) return;
    rec[R_COS1] = ci;
    if (fresnel) T1 = oracle_fresnel(g->n_air, g->n_glass, ci, ct, 0, 0);
    if (!oracle_cylinder_roots(x1, d1, g->r_inner, &tl, &th)) return;
    if (!(tl > 0.0)) return;
    for (int i = 0; i < 3; ++i) e[i] = x1[i] + tl * d1[i];
    double n2[3];
    radial_normal(e, n2);
    if (oracle_refract(g->n_glass, g->n_resin, d1, n2, dr, &ci, &ct)) return;
    rec[R_COS2] = ci;
    if (fresnel) T2 = oracle_fresnel(g->n_glass, g->n_resin, ci, ct, 0, 0);
  }
  // resin chord: from the entry e to the far inner wall
  double L = -2.0 * (e[0] * dr[0] + e[1] * dr[1]) / (dr[0] * dr[0] + dr[1] * dr[1]);
  double K = std::floor(L / g->step + 0.5);
  for (int i = 0; i < 3; ++i) {
    rec[R_E + i] = e[i];
    rec[R_DR + i] = dr[i];
  }
  rec[R_T1] = T1;
  rec[R_T2] = T2;
  rec[R_L] = L;
  if (K < 1.0) return;
  rec[R_K] = K;
  rec[R_W] = T1 * T2 / g->n_pupil;
  rec[R_HIT] = 1.0;
}

// Ray index of (u, v, j) in the oracle's own ordering.
static inline int64_t ray_id(const OracleGeometry* g, int u, int v, int j) {
  return ((int64_t)v * g->nu + u) * g->n_pupil + j;
}

static int clamp_threads(int nthreads) {
  if (nthreads <= 0) nthreads = (int)std::thread::hardware_concurrency();
  return std::max(1, nthreads);
}

}  // extern "C"

template <class F>
static void parallel_for(int64_t n, int nthreads, F f) {
  nthreads = (int)std::min<int64_t>(clamp_threads(nthreads), std::max<int64_t>(n, 1));
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([=]() {
      for (int64_t i = t; i < n; i += nthreads) f(i, t);
    });
  for (auto& th : pool) th.join();
}

extern "C" {

void oracle_trace(const OracleGeometry* g, double* recs, int nthreads) {
  parallel_for((int64_t)g->nv, nthreads, [=](int64_t v, int) {
    for (int u = 0; u < g->nu; ++u)
      for (int j = 0; j < g->n_pupil; ++j)
        oracle_trace_ray(g, u, (int)v, j, recs + R_SIZE * ray_id(g, u, (int)v, j));
  });
}

static double angle_of(const OracleGeometry* g, int a) {
  if (g->angles) return g->angles[a];
  return 2.0 * M_PI * a / g->n_angles;
}

// ------------------------------------------------------------- sampling --

// Anti-aliasing stencil of one volume-frame point: the 8 voxel centres of
// the cell containing it and their weights (1-dx)(1-dy)(1-dz), where d is
// the per-axis distance from the point to the voxel centre.  Voxels outside
// the grid get index -1.
static void stencil(const OracleGeometry* g, const double* p, int64_t* idx,
                    double* wt) {
  double gx = p[0] + 0.5 * (g->nx - 1);
  double gy = p[1] + 0.5 * (g->ny - 1);
  double gz = p[2] + 0.5 * (g->nz - 1);
  double fx0 = std::floor(gx), fy0 = std::floor(gy), fz0 = std::floor(gz);
  int c = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx, ++c) {
        double vx = fx0 + dx, vy = fy0 + dy, vz = fz0 + dz;
        double w = (1.0 - std::fabs(gx - vx)) * (1.0 - std::fabs(gy - vy)) *
                   (1.0 - std::fabs(gz - vz));
        wt[c] = w;
        if (vx < 0 || vy < 0 || vz < 0 || vx > g->nx - 1 || vy > g->ny - 1 ||
            vz > g->nz - 1)
          idx[c] = -1;
        else
          idx[c] = ((int64_t)vz * g->ny + (int64_t)vy) * g->nx + (int64_t)vx;
      }
}

// Calls f(k, weight c_k, stencil) for every sample of ray `rec` at angle
// theta: q_k = e + s_k d_r in the lab frame, p = Rz(-theta) q_k in the
// volume frame, c_k = w ds exp(-alpha s_k).
}  // extern "C"

template <class F>
static void for_each_sample(const OracleGeometry* g, const double* rec,
                            double theta, F f) {
  if (rec[R_HIT] == 0.0) return;
  const double* e = rec + R_E;
  const double* dr = rec + R_DR;
  int64_t K = (int64_t)rec[R_K];
  double ct = std::cos(theta), st = std::sin(theta);
  int64_t idx[8];
  double wt[8];
  for (int64_t k = 0; k < K; ++k) {
    double s = (k + 0.5) * g->step;
    double q[3] = {e[0] + s * dr[0], e[1] + s * dr[1], e[2] + s * dr[2]};
    double p[3] = {ct * q[0] + st * q[1], -st * q[0] + ct * q[1], q[2]};
    stencil(g, p, idx, wt);
    double c = rec[R_W] * g->step * std::exp(-g->alpha * s);
    f(k, c, idx, wt);
  }
}

extern "C" {

// ------------------------------------------------------------- operators --

// Forward projection (Sec. 2.4 with the Sec. 2.5 transmission factors):
// proj[a][v][u] for angles a0 .. a0+na-1.
void oracle_forward(const OracleGeometry* g, const double* vol, int a0, int na,
                    double* proj, int nthreads) {
  int64_t nray = (int64_t)g->nu * g->nv * g->n_pupil;
  std::vector<double> recs(nray * R_SIZE);
  oracle_trace(g, recs.data(), nthreads);
  const double* R = recs.data();
  parallel_for((int64_t)na * g->nv, nthreads, [=](int64_t row, int) {
    int a = (int)(row / g->nv), v = (int)(row % g->nv);
    double theta = angle_of(g, a0 + a);
    for (int u = 0; u < g->nu; ++u) {
      double acc = 0.0;
      for (int j = 0; j < g->n_pupil; ++j)
        for_each_sample(g, R + R_SIZE * ray_id(g, u, v, j), theta,
                        [&](int64_t, double c, const int64_t* idx, const double* wt) {
                          double val = 0.0;
                          for (int q = 0; q < 8; ++q)
                            if (idx[q] >= 0) val += wt[q] * vol[idx[q]];
                          acc += c * val;
                        });
      proj[((int64_t)a * g->nv + v) * g->nu + u] = acc;
    }
  });
}

// Forward projection of selected pixels only: out[i] = proj at
// (angle[i], v[i], u[i]).
void oracle_forward_pixels(const OracleGeometry* g, const double* vol,
                           int64_t n, const int32_t* ang, const int32_t* vv,
                           const int32_t* uu, double* out, int nthreads) {
  parallel_for(n, nthreads, [=](int64_t i, int) {
    double rec[R_SIZE];
    double theta = angle_of(g, ang[i]);
    double acc = 0.0;
    for (int j = 0; j < g->n_pupil; ++j) {
      oracle_trace_ray(g, uu[i], vv[i], j, rec);
      for_each_sample(g, rec, theta,
                      [&](int64_t, double c, const int64_t* idx, const double* wt) {
                        double val = 0.0;
                        for (int q = 0; q < 8; ++q)
                          if (idx[q] >= 0) val += wt[q] * vol[idx[q]];
                        acc += c * val;
                      });
    }
    out[i] = acc;
  });
}

// Dose deposit (Sec. 2.5), the transpose of oracle_forward:
// dose = sum over angles a0..a0+na-1 of A_a^T proj[a].  Each worker sums
// into its own buffer; the buffers are added in worker order.
void oracle_adjoint(const OracleGeometry* g, const double* proj, int a0, int na,
                    double* dose, int nthreads) {
  int64_t nray = (int64_t)g->nu * g->nv * g->n_pupil;
  int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
  std::vector<double> recs(nray * R_SIZE);
  oracle_trace(g, recs.data(), nthreads);
  const double* R = recs.data();
  int64_t rows = (int64_t)na * g->nv;
  int nt = (int)std::min<int64_t>(clamp_threads(nthreads), std::max<int64_t>(rows, 1));
  std::vector<std::vector<double>> part(nt);
  parallel_for(nt, nt, [&](int64_t t, int) {
    part[t].assign(nvox, 0.0);
    double* D = part[t].data();
    for (int64_t row = t; row < rows; row += nt) {
      int a = (int)(row / g->nv), v = (int)(row % g->nv);
      double theta = angle_of(g, a0 + a);
      for (int u = 0; u < g->nu; ++u) {
        double pv = proj[((int64_t)a * g->nv + v) * g->nu + u];
        if (pv == 0.0) continue;
        for (int j = 0; j < g->n_pupil; ++j)
          for_each_sample(g, R + R_SIZE * ray_id(g, u, v, j), theta,
                          [&](int64_t, double c, const int64_t* idx, const double* wt) {
                            for (int q = 0; q < 8; ++q)
                              if (idx[q] >= 0) D[idx[q]] += c * wt[q] * pv;
                          });
      }
    }
  });
  for (int64_t i = 0; i < nvox; ++i) dose[i] = 0.0;
  for (int t = 0; t < nt; ++t)
    for (int64_t i = 0; i < nvox; ++i) dose[i] += part[t][i];
}

// Number of samples (angles a0..a0+na-1) whose stencil touches the grid.
int64_t oracle_count_samples(const OracleGeometry* g, int a0, int na,
                             int nthreads) {
  int64_t nray = (int64_t)g->nu * g->nv * g->n_pupil;
  std::vector<double> recs(nray * R_SIZE);
  oracle_trace(g, recs.data(), nthreads);
  int nt = clamp_threads(nthreads);
  std::vector<int64_t> cnt(nt, 0);
  const double* R = recs.data();
  parallel_for((int64_t)na * nray, nt, [&](int64_t i, int t) {
    int a = (int)(i / nray);
    int64_t r = i % nray;
    for_each_sample(g, R + R_SIZE * r, angle_of(g, a0 + a),
                    [&](int64_t, double, const int64_t* idx, const double*) {
                      for (int q = 0; q < 8; ++q)
                        if (idx[q] >= 0) {
                          ++cnt[t];
                          break;
                        }
                    });
  });
  int64_t s = 0;
  for (auto c : cnt) s += c;
  return s;
}

// ------------------------------------------------- loss and its gradient --

// Dose-threshold loss of projections `proj` (all angles) against a binary
// target: d = A^T proj, sig = 1/(1 + exp(-kappa (d - thr))),
// loss = mean (sig - t)^2 over all voxels; grad = A r with
// r = (2/N) (sig - t) sig (1 - sig) kappa.  dose and grad may be NULL.
double oracle_loss_grad(const OracleGeometry* g, const double* target,
                        const double* proj, double kappa, double thr,
                        double* dose_out, double* grad_out, int nthreads) {
  int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
  std::vector<double> dose(nvox), r(nvox);
  oracle_adjoint(g, proj, 0, g->n_angles, dose.data(), nthreads);
  double loss = 0.0;
  for (int64_t i = 0; i < nvox; ++i) {
    double sig = 1.0 / (1.0 + std::exp(-kappa * (dose[i] - thr)));
    double diff = sig - target[i];
    loss += diff * diff;
    r[i] = (2.0 / nvox) * diff * sig * (1.0 - sig) * kappa;
  }
  loss /= nvox;
  if (dose_out) std::memcpy(dose_out, dose.data(), nvox * sizeof(double));
  if (grad_out) oracle_forward(g, r.data(), 0, g->n_angles, grad_out, nthreads);
  return loss;
}

// ------------------------------------------------ paper geometry helpers --

// Ideal thin lens: magnification of an image at distance s_i for focal
// length f (1/s_o + 1/s_i = 1/f, m = s_i / s_o).
double oracle_thin_lens_magnification(double f, double s_i) {
  double s_o = 1.0 / (1.0 / f - 1.0 / s_i);
  return s_i / s_o;
}

// Paraxial etendue of one pixel: area x solid angle of a cone with half
// angle theta = full divergence / 2, Omega = pi theta^2.
double oracle_paraxial_etendue(double pixel, double full_divergence_deg) {
  double theta = 0.5 * full_divergence_deg * M_PI / 180.0;
  return pixel * pixel * M_PI * theta * theta;
}

// Full axial divergence (degrees) behind a relay lens of focal length f with
// an iris of diameter `iris` at its focal plane.
double oracle_iris_divergence_deg(double iris, double f) {
  return 2.0 * std::atan(0.5 * iris / f) * 180.0 / M_PI;
}

}  // extern "C"
