/*
 * vam.h -- C ABI of libvam, the MI355X (gfx950) 3D ray-traced projector pair
 * for tomographic volumetric additive manufacturing.
 *
 * Method: Webber et al., "Versatile volumetric additive manufacturing with
 * 3D ray tracing".  Rays are cast per DMD pixel across the projector's
 * aperture stop (Sec. 2.1), refracted by vector Snell's law at the
 * air-glass and glass-resin vial walls and stopped at the far inner wall
 * (Sec. 2.1), sampled with the anti-aliasing weights of Sec. 2.2
 * ("Anti-aliasing"), and used both for the tomographic projection
 * (Sec. 2.4) and for the dose deposit with Fresnel and Beer-Lambert
 * transmission (Sec. 2.5), for every rotation angle.
 *
 * Conventions (all lengths in voxel units):
 *   lab frame   vial axis +z through the origin, light travels +y, the
 *               projector's focus plane is y = 0 (rotation axis at best
 *               focus, Sec. 2.8);
 *   volume      V[z][y][x], x fastest; voxel (i,j,k) is centred at
 *               (i-(nx-1)/2, j-(ny-1)/2, k-(nz-1)/2) in the volume frame;
 *   rotation    at angle theta the vial has turned by +theta about +z, so a
 *               lab point q is at Rz(-theta) q in the volume frame;
 *   projections P[angle][v][u], u fastest; pixel (u,v) images to
 *               Q = ((u-(n_u-1)/2) pitch_u, 0, (v-(n_v-1)/2) pitch_v);
 *   samples     s_k = (k+1/2) step from the resin entry, k < K =
 *               floor(L/step + 1/2), L the resin chord; sample weight
 *               c_k = (T1 T2 / n_pupil) step exp(-alpha s_k);
 *   weights     trilinear tent over the 8 voxel centres around a sample;
 *               voxels outside the grid read 0 and receive nothing.
 *
 * The forward operator A maps a volume to projections,
 *   P[a][v][u] = sum_j sum_k c_k sum_corners W V,
 * and the dose deposit is its exact transpose, D = A^T P.
 *
 * Memory and streams: every volume, projection and dose pointer is a DEVICE
 * pointer owned by the caller, contiguous, 16-byte aligned, on the device
 * that was current at vam_setup_geometry.  Calls are asynchronous and
 * stream-ordered on the given stream; a handle may be used from one stream
 * at a time.  No call throws; each returns a vam_status and, on failure,
 * sets a thread-local message readable with vam_last_error().
 */
#ifndef VAM_H
#define VAM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VAM_OK = 0,
  VAM_ERR_INVALID_ARG = -1,   /* bad descriptor, pointer, size or range    */
  VAM_ERR_UNSUPPORTED = -2,   /* valid request the library does not handle */
  VAM_ERR_OUT_OF_MEMORY = -3, /* a device allocation failed                */
  VAM_ERR_HIP = -4,           /* a HIP runtime call or launch failed       */
  VAM_ERR_BAD_HANDLE = -5     /* NULL or destroyed geometry handle         */
} vam_status;

/* Element type of caller buffers.  Reduced types are rounded to nearest
 * even on store; all ray sums accumulate in FP32. */
typedef enum { VAM_F32 = 0, VAM_BF16 = 1, VAM_F16 = 2 } vam_dtype;

/* Projector models (Sec. 2.6.1 and 2.6.2). */
typedef enum {
  VAM_TELECENTRIC = 0, /* chief rays along +y; pupil = sin(half divergence) */
  VAM_THIN_LENS = 1    /* ideal lens at the stop, plane y = -focus_distance;
                          pupil = stop radius                                */
} vam_projector;

enum {
  VAM_NO_FRESNEL = 1u  /* refract at the walls but transmit all power */
};

/* Printer and volume geometry.  Host arrays are copied at setup. */
typedef struct {
  int32_t nx, ny, nz;        /* volume size, each in [1, 2048]              */
  int32_t n_u, n_v;          /* DMD pixels, each in [1, 8192]               */
  double pitch_u, pitch_v;   /* pixel pitch on the focus plane, > 0         */
  int32_t n_angles;          /* >= 1                                        */
  const double* angles_rad;  /* [n_angles], or NULL for 2 pi a / n_angles   */
  int32_t projector;         /* vam_projector                               */
  double focus_distance;     /* thin lens: > r_outer                        */
  double pupil;              /* see vam_projector; >= 0 (< 1 telecentric)   */
  int32_t n_pupil;           /* rays per pixel, in [1, 1024]                */
  const double* pupil_xy;    /* [n_pupil][2] points in the unit disk, or
                                NULL when n_pupil == 1 (chief ray)          */
  double r_outer, r_inner;   /* vial radii, r_outer >= r_inner > 0; equal
                                radii mean an index-matched vial (no walls,
                                no refraction, T = 1)                       */
  double n_air, n_glass, n_resin; /* refractive indices, each >= 1          */
  double alpha;              /* absorption per voxel length in resin, >= 0  */
  double step;               /* sample spacing along the ray, > 0           */
  uint32_t flags;            /* VAM_NO_FRESNEL                              */
} vam_geometry_desc;

typedef struct vam_geometry* vam_geometry_t;

/* Trace every ray of every pixel and pupil point through the optics and the
 * vial walls (Sec. 2.1; Fresnel factors of Sec. 2.5) in FP64 on the device
 * and keep the resin segments as the handle's ray table.  Allocates the ray
 * table and the padded working volumes (owned by the handle).  Synchronises
 * `stream` before returning.  Errors: VAM_ERR_INVALID_ARG for a descriptor
 * outside the ranges above or a NULL `out`; VAM_ERR_OUT_OF_MEMORY;
 * VAM_ERR_HIP. */
vam_status vam_setup_geometry(const vam_geometry_desc* desc, hipStream_t stream,
                              vam_geometry_t* out);

/* Free the handle and everything it owns.  NULL is accepted.  The caller
 * must ensure no call using the handle is still running on the device. */
vam_status vam_destroy_geometry(vam_geometry_t h);

/* Forward projection (Sec. 2.4, with the Sec. 2.5 transmission factors):
 * writes proj[a - angle_begin][v][u] for angles angle_begin ..
 * angle_begin+angle_count-1 from vol[nz][ny][nx].  vol_t and proj_t select
 * the element types.  Deterministic: the same inputs give the same bits.
 * Each pixel's segment sums are added in 64-bit fixed point (rounding
 * <= 2^-61 of a bound per add, see vam_set_variant, op 0) and the total is
 * rounded once; a NaN or infinity anywhere in the volume makes every
 * projection value of the call NaN.  The first call allocates
 * n_angles x n_u x n_v x 8 bytes in the handle.
 * Errors: VAM_ERR_BAD_HANDLE; VAM_ERR_INVALID_ARG for NULL pointers, bad
 * dtypes, angle_count < 1 or an angle range outside [0, n_angles);
 * VAM_ERR_OUT_OF_MEMORY; VAM_ERR_HIP. */
vam_status vam_forward_project(vam_geometry_t h, const void* vol, vam_dtype vol_t,
                               void* proj, vam_dtype proj_t,
                               int32_t angle_begin, int32_t angle_count,
                               hipStream_t stream);

/* Dose deposit (Sec. 2.5), the exact transpose of vam_forward_project over
 * the same angle range: dose[nz][ny][nx] (FP32) receives
 * sum_a A_a^T proj[a - angle_begin].  accumulate != 0 adds to dose,
 * otherwise dose is overwritten.  Rays whose projection value is exactly 0
 * are skipped (they add nothing).  The default kernel sums each (box of the
 * lab frame, angle) in 32-bit fixed point, scaled per box and angle so that
 * no partial sum can overflow (rounding <= 2^-31 of a bound on the box's
 * largest cell sum per add), then adds each cell to the voxel's 64-bit
 * integer at a power-of-two scale set by the call's largest |projection
 * value| (rounding <= 2^-61 of a bound on the voxel's dose per add); the
 * integer adds commute, so the result is deterministic (the same bits on
 * every run and for every segment order).  A NaN or infinity among the
 * projection values makes the whole dose NaN.  The angle range selects
 * which projections proj holds (one GPU's share of the angles when the
 * work is split).  The first call allocates (nx+4)(ny+4)(nz+4) + 32 eight-
 * byte words in the handle.  Errors as for vam_forward_project. */
vam_status vam_back_project(vam_geometry_t h, const void* proj, vam_dtype proj_t,
                            float* dose, int32_t accumulate,
                            int32_t angle_begin, int32_t angle_count,
                            hipStream_t stream);

/* vam_back_project without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it).  Same arguments, operator and result as
 * vam_back_project; the padded accumulator of the deposit comes from a
 * file-scope device array of the library (136 MiB per device, held by every
 * device the library runs on until the process ends) instead of the
 * handle.  Limit: the padded grid (nx+4)(ny+4)(nz+4) must be at most
 * 17,825,760 voxels (cubes up to 257^3), else VAM_ERR_UNSUPPORTED; the
 * gather variant (vam_set_variant op 1 = 2) is refused the same way.  All
 * calls on one device share the array and it keeps the last call's
 * contents (each call clears it first, with a kernel): calls that overlap
 * on one device race.  Errors as for vam_back_project. */
vam_status vam_back_project_noalloc(vam_geometry_t h, const void* proj, vam_dtype proj_t,
                                    float* dose, int32_t accumulate,
                                    int32_t angle_begin, int32_t angle_count,
                                    hipStream_t stream);

/* One projected gradient step of the dose-threshold loss, standing in for
 * the paper's iterative projection optimisation (Sec. 2.7), over all
 * angles:
 *   d = A^T g,  sig = 1/(1+exp(-sharpness (d - threshold))),
 *   loss = mean over voxels of (sig - target)^2,
 *   grad = A [ (2/N)(sig - target) sig (1-sig) sharpness ],
 *   g <- g - lr grad, then g <- max(g, 0) if clamp_nonneg.
 * target: FP32 [nz][ny][nx]; proj: [n_angles][n_v][n_u] of element type
 * proj_t (FP32, BF16 or FP16), updated in place: the deposit reads the
 * stored values, the gradient is FP32 and the updated value is rounded to
 * nearest even on store; dose (optional, may be NULL): FP32 [nz][ny][nx]
 * receives d; the loss is reduced in FP64.  loss_out (optional) receives the
 * loss of the projections BEFORE the update; passing it synchronises
 * `stream`.  The first call allocates the step's buffers (two volumes and
 * an FP32 gradient of the projections' shape, and the forward
 * projection's) in the handle.  Errors:
 * VAM_ERR_BAD_HANDLE; VAM_ERR_INVALID_ARG for NULL pointers, an unknown
 * dtype or parameters outside the ranges below; VAM_ERR_OUT_OF_MEMORY;
 * VAM_ERR_HIP. */
typedef struct {
  double threshold;     /* gelation dose threshold, e.g. 0.8 */
  double sharpness;     /* sigmoid slope kappa, > 0          */
  double lr;            /* step size, >= 0                   */
  int32_t clamp_nonneg; /* 1: project onto g >= 0            */
} vam_opt_params;

vam_status vam_optimize_step(vam_geometry_t h, const float* target, void* proj, vam_dtype proj_t,
                             float* dose, const vam_opt_params* params,
                             double* loss_out, hipStream_t stream);

/* Ram-Lak filtering of projection rows, for the plain (filtered
 * parallel-beam) initialisation of Sec. 2.3: each of the n_rows rows of n_u
 * FP32 values (device, row-major) is convolved along u with the discrete
 * band-limited ramp kernel for pixel pitch `pitch` (h[0] = 1/(4 pitch^2),
 * h[n] = -1/(n^2 pi^2 pitch^2) for odd n, 0 for even n != 0, times pitch),
 * then clipped at zero when clip_negative != 0.  proj_out must not alias
 * proj_in.  Asynchronous on `stream`.  Errors: VAM_ERR_INVALID_ARG for NULL
 * or aliased buffers, n_u outside [1, 8192], pitch <= 0. */
vam_status vam_ramlak_filter(const float* proj_in, float* proj_out, int32_t n_rows, int32_t n_u,
                             double pitch, int32_t clip_negative, hipStream_t stream);

/* Dose error of Sec. 2.7's termination test, reduced in FP64 over n
 * voxels of device arrays dose and target (FP32):
 *   out2[0] = ||sigmoid(sharpness (dose - threshold)) - target||_1 / ||target||_1,
 *   out2[1] = fraction of voxels where (dose >= threshold) != (target >= 0.5).
 * out2 is host memory; the call synchronises `stream`. */
vam_status vam_dose_error(const float* dose, const float* target, int64_t n, double threshold,
                          double sharpness, double* out2, hipStream_t stream);

/* 8-bit export of projections (Sec. 2.7): over all n FP32 values (device),
 * mean and population standard deviation in FP64; clip = mean + 3 std;
 * out[i] = round-half-even(255 * min(max(proj[i], 0), clip) / clip), the
 * product formed in FP64 (0 everywhere if clip <= 0).  out: n bytes
 * (device).  stats3 (host, optional): mean, std, clip; passing it
 * synchronises `stream`. */
vam_status vam_equalize_u8(const float* proj, int64_t n, uint8_t* out, double* stats3,
                           hipStream_t stream);

/* Ray-table statistics: rays that reach the resin, and ray-voxel samples
 * over all angles whose anti-aliasing stencil touches the grid (one pass of
 * vam_forward_project or vam_back_project over all angles processes this
 * many samples).  Either pointer may be NULL. */
vam_status vam_ray_table_stats(vam_geometry_t h, int64_t* rays_hit,
                               int64_t* samples_per_pass);

/* Copy the FP64 resin segments to host memory: for every ray in order
 * ((j * n_v + v) * n_u + u), 12 doubles: entry point e (3), resin direction
 * (3), chord length L, sample count K, weight T1 T2 / n_pupil, T1, T2,
 * hit flag (1 or 0).  `out` holds n_u * n_v * n_pupil * 12 doubles.
 * Synchronises the handle's setup stream. */
vam_status vam_export_rays(vam_geometry_t h, double* out);

/* Select the kernel variant of an operator for this handle (measurement
 * and testing; every variant computes the same operator).
 *   op 0, forward:  0 = default: lab-box tiled, volume footprint staged in
 *                   LDS, each segment's partial added to its pixel as a
 *                   64-bit integer (scale: a power of two from the volume's
 *                   largest |value| and the most samples of a pixel;
 *                   rounding <= 2^-61 of that bound per add; integer adds
 *                   make it deterministic); a NaN or infinity anywhere in
 *                   the volume makes every projection value NaN.  Needs
 *                   n_angles x n_u x n_v x 8 bytes, allocated on first use;
 *                   1 = ray-driven reference (one lane per pixel and angle,
 *                   buffer gathers from the padded volume);
 *                   2 = lab-box tiled, per-segment FP32 partial sums in a
 *                   buffer of up to 8 GiB (allocated on first use), added
 *                   per pixel in a fixed order by a second kernel.
 *   op 1, deposit:  0 = default: lab-box tiled, footprint summed in LDS in
 *                   32-bit fixed point (the scale of each box and angle
 *                   bounds every partial sum below 2^31; rounding <= 2^-31
 *                   of that bound per add), then 64-bit integer adds into
 *                   the voxels (deterministic; a non-finite projection
 *                   value makes the whole dose NaN);
 *                   1 = ray-driven reference with FP64 global atomics;
 *                   2 = voxel-driven gather through an inverse ray map
 *                   (lab-frame unit cells -> sample runs; built on first
 *                   use, ~32 bytes per run; no atomics, fixed order).
 *   op 2, tiling:   lab-box edge in voxels: 8, 12 (default) or 16; rebuilds
 *                   the box decomposition (synchronises the device).
 *   op 4, order:    order of the segments inside a box for the deposit:
 *                   0 = by ray, 1 = by decreasing length, 2 = by pixel
 *                   parity class (u mod 2, v mod 2) then ray, 3, 4 = by
 *                   class (u mod m, v mod m), m = 3, 4, then ray, 5 = by a
 *                   hash of the ray index, 6 = by pixel, then pupil sample,
 *                   7, 8 = order 3, then each run of 1024 (7) or 2048 (8)
 *                   segments by decreasing length, 9 = by pupil sample,
 *                   then pixel column, then row, 10 = by class (u mod 3,
 *                   v mod 2), then ray, 11, 12, 13 = order 10, then each
 *                   run of 1024 (11, default), 512 (12) or 2048 (13)
 *                   segments by decreasing length, 14, 15, 16 = by ray,
 *                   then each run of 256 (14) or 1024 (15) segments, or the
 *                   whole box (16), by decreasing length in steps of two
 *                   samples; rebuilds the boxes.
 *   op 5, threads:  workgroup size of the box deposit, 256 (default) or 512.
 *   op 7, order:    as op 4, for the forward projection (default 16).
 *   op 8, 9:        work order of the deposit (8) or forward (9) box
 *                   kernels: 0 = boxes fastest, 1 = XCD-aware with all
 *                   angles of a box on one XCD, A >= 2 = XCD-aware with the
 *                   angles of a box in blocks of A (up to 4096; default 8
 *                   for the deposit, 16 for the forward).
 *   op 10, mode:    how the default (fixed-point) box forward marches a
 *                   segment: 1 = one lane; 2 = two lanes take alternate
 *                   samples, each summing with r^2 (their samples are half
 *                   a voxel apart, so they often read the same LDS words);
 *                   3 = one lane that keeps the current cell's LDS words in
 *                   registers and reads LDS only when its cell changes
 *                   (the same bits as 1); 0 = default: 3 for FP32 and BF16
 *                   volumes, 1 for FP16.
 * A failed rebuild (ops 2, 4, 7) leaves the handle without a box
 * decomposition: the box kernels then return VAM_ERR_INVALID_ARG until a
 * rebuild succeeds.  Errors: VAM_ERR_BAD_HANDLE, VAM_ERR_INVALID_ARG for an
 * unknown op or variant, VAM_ERR_OUT_OF_MEMORY, VAM_ERR_HIP. */
vam_status vam_set_variant(vam_geometry_t h, int32_t op, int32_t variant);

/* Test hook for error paths: the n-th device allocation the library makes
 * after this call (n >= 1) fails as if the device were out of memory; n = 0
 * switches the hook off.  Process-wide, not thread-safe; for tests only. */
vam_status vam_debug_fail_allocations(int32_t n);

/* Instrumentation: device time (ms) of the main kernel of the last
 * vam_forward_project and of the last vam_back_project on this handle,
 * from HIP events recorded on the caller's stream right around that kernel
 * (the small copy kernels around it are excluded).  -1 if no such call has
 * been made.  The caller must have synchronised the stream.  Either pointer
 * may be NULL. */
vam_status vam_kernel_times(vam_geometry_t h, float* forward_ms, float* back_ms);

/* Thread-local description of the last failure on this thread ("" if
 * none).  The string stays valid until the next vam_* call on the thread. */
const char* vam_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t vam_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VAM_H */
