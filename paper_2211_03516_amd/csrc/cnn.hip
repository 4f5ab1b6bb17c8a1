// Learned initialiser: a small 3x3 convolutional network trained and run on
// MFMA matrix cores (gfx950 v_mfma_f32_32x32x16_bf16).
//
// Every convolution is one GEMM over the im2col matrix of its input:
//   forward          z[p][co]     = sum_kc col(a)[p][kc]   W[co][kc]
//   data gradient    da[p][ci]    = sum_kc col(g)[p][kc]   Wflip[ci][kc]
//   weight gradient  dW^T[kc][co] = sum_p  col(a)[p][kc]   g[p][co]
// Every GEMM gathers its col tiles straight from the NHWC activations (or
// gradients) while staging them in LDS: no im2col matrix is written to
// memory.  The weight gradient stages both operands transposed (pixels
// along k).
// with p a pixel of the batch, kc = (tap, channel) and Wflip the kernel
// turned by 180 degrees with input and output channels swapped (the
// transposed convolution as a convolution).  Activations are NHWC BF16 with
// channels padded to a multiple of 8; K of every GEMM is padded to the
// 32-element k-tile with zeros.  The weight-gradient GEMM splits its pixel
// sum over workgroups into FP32 partials that a second kernel adds in a
// fixed order, so training is deterministic.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "vam_cnn.h"
#include "vam_internal.h"

namespace vam {
namespace cnn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr uint64_t kCnnMagic = 0x56414d434e4e3031ull;  // "VAMCNN01"
constexpr int BM = 128, BN = 64, BK = 32, LDK = BK + 8;
constexpr int kMaxSplits = 256;

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline bool bf_positive(uint16_t h) { return h != 0 && !(h & 0x8000u); }

enum Epi { EPI_RELU_BF16 = 0, EPI_BIAS_F32 = 1, EPI_MASK_BF16 = 2, EPI_PART_F32 = 3 };

struct GemmArgs {
  const uint16_t* B;   // !CONVT: [N][ldb] (B^T rows: the packed weights)
  int M, N, K;         // K per split (multiple of BK)
  int ldb;
  void* C;
  int ldc;
  int64_t split_stride;      // EPI_PART_F32: elements between split partials
  const float* bias;         // EPI_RELU_BF16, EPI_BIAS_F32
  const uint16_t* mask;      // EPI_MASK_BF16: [M][ldm]
  int ldm;
  const uint16_t* X;         // !CONVT: A = col(X), X NHWC [M pixels][cp]; CONVT: A = col(X)^T
  int H, W, cp;              // image size, padded channels of X
  const uint16_t* G;         // CONVT: B = G^T, G NHWC [pixels][cpg]
  int cpg;
  int ones_row;              // CONVT: A row of ones (the bias gradient's column sums)
};

// Transposed staging (CONVT) of 8 rows x 2 pixels: fetch_t loads the
// 8-channel chunk `c` of pixels k0 + pp and k0 + pp + 1 of `src` (channels
// per pixel `cp`) shifted by (dy, dx), zero where `ok` is false or the
// shifted pixel leaves the image; store_t writes element j of both as one
// 32-bit word at tile[(8 rc + j) LDK + pp].
__device__ inline void fetch_t(uint4 (&v)[2], const uint16_t* src, int64_t k0, int pp, int cp, int c, int dy, int dx,
                               bool ok, int H, int W) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    v[e] = make_uint4(0, 0, 0, 0);
    const int p = (int)k0 + pp + e;  // pixel indices fit 31 bits (checked at creation)
    if (ok) {
      const int x = p % W, y = (p / W) % H;
      if (y + dy >= 0 && y + dy < H && x + dx >= 0 && x + dx < W)
        v[e] = *(const uint4*)(src + ((int64_t)p + dy * W + dx) * cp + c);
    }
  }
}

__device__ inline void store_t(uint16_t* tile, int rc, int pp, const uint4 (&v)[2]) {
  const uint32_t w0[4] = {v[0].x, v[0].y, v[0].z, v[0].w}, w1[4] = {v[1].x, v[1].y, v[1].z, v[1].w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    *(uint32_t*)(tile + (8 * rc + 2 * q) * LDK + pp) = (w0[q] & 0xffffu) | (w1[q] << 16);
    *(uint32_t*)(tile + (8 * rc + 2 * q + 1) * LDK + pp) = (w0[q] >> 16) | (w1[q] & 0xffff0000u);
  }
}

// C = epilogue(sum_k A(m, k) B(k, n)), 128 x 64 output tile per workgroup,
// four waves of 32 rows x 64 columns (two 32 x 32 MFMA blocks each).  In
// the !CONVT GEMMs the next k-tile's global loads are issued into registers
// before the current tile's MFMAs and written to LDS after them (10 %
// faster); the CONVT GEMM stages each tile just before its MFMAs (its
// prefetching form needs more registers and ran 37 % slower).
//  !CONVT: A(m, k) = X[pixel m shifted by tap][c], k = tap cp + c (tap =
//   3 (dy + 1) + dx + 1), zero outside the image and for k >= 9 cp: the
//   im2col matrix, gathered 8 channels (16 bytes) at a time; B(k, n) =
//   B[n][k] (packed weights, ldb per row).
//  CONVT: A(m, k) = the same with m = tap cp + c and k the pixel, and
//   B(k, n) = G[pixel k][n] (the weight gradient's operands); row ones_row
//   of A is all ones, so that row of C is the column sums of G (the bias
//   gradient).
template <int EPI, bool CONVT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDK];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int64_t kbase = (int64_t)blockIdx.z * g.K;
  f32x16 acc0, acc1;
  for (int r = 0; r < 16; ++r) {
    acc0[r] = 0.0f;
    acc1[r] = 0.0f;
  }
  auto mma = [&]() {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      const bf16x8 a = *(const bf16x8*)(As + (wave * 32 + (lane & 31)) * LDK + kk);
      const bf16x8 b0 = *(const bf16x8*)(Bs + (lane & 31) * LDK + kk);
      const bf16x8 b1 = *(const bf16x8*)(Bs + (32 + (lane & 31)) * LDK + kk);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
    }
  };
  if constexpr (CONVT) {
    // each tile staged right before its MFMAs: work item (rc, pp) moves an
    // 8-row chunk of two pixels of A (and, t < 128, of B)
    const int rc = t >> 4, pp = (t & 15) * 2, kc = m0 + 8 * rc, co = n0 + 8 * rc;
    for (int kt = 0; kt < g.K; kt += BK) {
      const int64_t k0 = kbase + kt;
      uint4 v[2];
      if (kc == g.ones_row) {
        // rows ones_row .. + 7: ones, then zeros (bf16 1.0 = 0x3f80)
        *(uint32_t*)(As + (8 * rc) * LDK + pp) = 0x3f803f80u;
#pragma unroll
        for (int j = 1; j < 8; ++j) *(uint32_t*)(As + (8 * rc + j) * LDK + pp) = 0u;
      } else {
        const int tap = kc / g.cp, c = kc - tap * g.cp;
        fetch_t(v, g.X, k0, pp, g.cp, c, tap / 3 - 1, tap % 3 - 1, kc < g.M && tap < 9, g.H, g.W);
        store_t(As, rc, pp, v);
      }
      if (t < 128) {
        fetch_t(v, g.G, k0, pp, g.cpg, co, 0, 0, co < g.cpg, g.H, g.W);
        store_t(Bs, rc, pp, v);
      }
      __syncthreads();
      mma();
      __syncthreads();
    }
  } else {
    // the next tile's global loads are issued before the current tile's
    // MFMAs and written to LDS after them
    int cy[2], cx[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int p = m0 + (t >> 2) + 64 * i;
      cx[i] = p % g.W;
      cy[i] = (p / g.W) % g.H;
    }
    uint4 ra[2], rb;
    auto fetch = [&](int64_t k0) {
      const int kc = (int)k0 + (t & 3) * 8;
      const int tap = kc / g.cp, c = kc - tap * g.cp;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int p = m0 + (t >> 2) + 64 * i;
        const int yy = cy[i] + dy, xx = cx[i] + dx;
        ra[i] = make_uint4(0, 0, 0, 0);
        if (p < g.M && tap < 9 && yy >= 0 && yy < g.H && xx >= 0 && xx < g.W)
          ra[i] = *(const uint4*)(g.X + ((int64_t)p + dy * g.W + dx) * g.cp + c);
      }
      const int row = t >> 2;
      rb = make_uint4(0, 0, 0, 0);
      if (n0 + row < g.N) rb = *(const uint4*)(g.B + (int64_t)(n0 + row) * g.ldb + k0 + (t & 3) * 8);
    };
    fetch(kbase);
    for (int kt = 0; kt < g.K; kt += BK) {
#pragma unroll
      for (int i = 0; i < 2; ++i) *(uint4*)(As + ((t >> 2) + 64 * i) * LDK + (t & 3) * 8) = ra[i];
      *(uint4*)(Bs + (t >> 2) * LDK + (t & 3) * 8) = rb;
      __syncthreads();
      if (kt + BK < g.K) fetch(kbase + kt + BK);
      mma();
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      // accumulator layout: register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
      const int m = m0 + wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int n = n0 + 32 * j + (lane & 31);
      if (m >= g.M || n >= g.N) continue;
      const float v = j ? acc1[r] : acc0[r];
      const int64_t o = (int64_t)m * g.ldc + n;
      if (EPI == EPI_RELU_BF16) {
        ((uint16_t*)g.C)[o] = f2bf(fmaxf(v + g.bias[n], 0.0f));
      } else if (EPI == EPI_BIAS_F32) {
        ((float*)g.C)[o] = v + g.bias[n];
      } else if (EPI == EPI_MASK_BF16) {
        ((uint16_t*)g.C)[o] = bf_positive(g.mask[(int64_t)m * g.ldm + n]) ? f2bf(v) : (uint16_t)0;
      } else {
        ((float*)g.C)[(int64_t)blockIdx.z * g.split_stride + o] = v;
      }
    }
  }
}

// a0[p][c] = bf16(s_c x[img][c][h][w]) for c < 2, zero for 2 <= c < 8.
__global__ void k_pack_input(const float* __restrict__ x, int64_t npix, int hw, float s0, float s1,
                             uint16_t* __restrict__ a0) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const int64_t img = p / hw, off = p - img * hw;
  const float x0 = x[img * 2 * hw + off], x1 = x[img * 2 * hw + hw + off];
  uint4 v;
  v.x = (uint32_t)f2bf(s0 * x0) | ((uint32_t)f2bf(s1 * x1) << 16);
  v.y = v.z = v.w = 0;
  *(uint4*)(a0 + p * 8) = v;
}

// y = x1 + z / s1
__global__ void k_output(const float* __restrict__ z, int ldz, const float* __restrict__ x, int64_t npix, int hw,
                         float s1, float* __restrict__ y) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const int64_t img = p / hw, off = p - img * hw;
  y[p] = x[img * 2 * hw + hw + off] + z[p * ldz] / s1;
}

// Residual r = z + s1 x1 - s1 t; g[p][0] = bf16(2 r / npix), other channels
// 0; per-block sum of r^2 in FP64 (fixed-order tree).
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ z, int ldz, const float* __restrict__ x,
                                              const float* __restrict__ tgt, int64_t npix, int hw, float s1,
                                              uint16_t* __restrict__ g, double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double r2 = 0.0;
  if (p < npix) {
    const int64_t img = p / hw, off = p - img * hw;
    const float r = z[p * ldz] + s1 * x[img * 2 * hw + hw + off] - s1 * tgt[p];
    r2 = (double)r * r;
    uint4 v;
    v.x = f2bf(2.0f * r / (float)npix);
    v.y = v.z = v.w = 0;
    *(uint4*)(g + p * 8) = v;
  }
  sh[threadIdx.x] = r2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// *out = scale * sum of part[0 .. n): thread j adds part[j], part[j + 256],
// ... in order, then a fixed-shape tree adds the 256 sums (one workgroup of
// 256 threads; the same order on every call).
__global__ __launch_bounds__(256) void k_sum_in_order(const double* part, int n, double scale, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

// grad W[co][tap][ci] = sum over splits of part[z][tap * cinp + ci][co]
// and grad b[co] = sum over splits of part[z][kp][co] (the row of ones)
// (part entry o = kc * ldc + co).  A workgroup takes 64 consecutive entries
// o; its four waves add the splits z = w, w + 4, ... (w = wave) in order,
// reading 64 consecutive floats per split, and the four sums are added in
// wave order: a fixed order on every call.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* part, int splits, int64_t stride, int ldc, int cinp,
                                                      int cin, int cout, int kp, float* grad, float* bgrad) {
  __shared__ double sh[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t o = (int64_t)blockIdx.x * 64 + l;
  double s = 0.0;
  if (o < stride)
    for (int z = w; z < splits; z += 4) s += part[z * stride + o];
  sh[w][l] = s;
  __syncthreads();
  if (w != 0 || o >= stride) return;
  const int kc = (int)(o / ldc), co = (int)(o - (int64_t)kc * ldc);
  const int tap = kc / cinp, ci = kc - tap * cinp;
  const float v = (float)(((sh[0][l] + sh[1][l]) + sh[2][l]) + sh[3][l]);
  if (co >= cout) return;  // padding
  if (kc == kp)
    bgrad[co] = v;
  else if (tap < 9 && ci < cin)
    grad[(co * 9 + tap) * cin + ci] = v;
}

// Forward weights wb[co][kc] (kc = tap * cinp + ci) and, for the data
// gradient, wf[ci][kc'] (kc' = tap' * coutp + co) = W[co][8 - tap'][ci].
__global__ void k_pack_weights(const float* __restrict__ W, int cin, int cout, int cinp, int coutp, int kp, int kpb,
                               uint16_t* __restrict__ wb, uint16_t* __restrict__ wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < coutp * kp) {
    const int co = i / kp, kc = i % kp, tap = kc / cinp, ci = kc % cinp;
    const float v = (co < cout && tap < 9 && ci < cin) ? W[(co * 9 + tap) * cin + ci] : 0.0f;
    wb[i] = f2bf(v);
  }
  if (wf && i < cinp * kpb) {
    const int ci = i / kpb, kc = i % kpb, tap = kc / coutp, co = kc % coutp;
    const float v = (ci < cin && co < cout && tap < 9) ? W[(co * 9 + (8 - tap)) * cin + ci] : 0.0f;
    wf[i] = f2bf(v);
  }
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace cnn
}  // namespace vam

struct vam_cnn {
  uint64_t magic;
  int device;
  int L, C, H, W, maxn;
  float s0, s1;
  std::vector<int> cin, cout, cinp, coutp, kp, kpb;
  std::vector<int64_t> woff, boff;
  int64_t nparam;
  float *master, *m1, *m2, *grad;
  std::vector<uint16_t*> wb, wf;   // per layer (index l - 1)
  std::vector<uint16_t*> act;      // a_0 .. a_{L-1}
  float* z;
  uint16_t* g[2];
  float* part;
  double* lpart;
  double* loss;
  int adam_t;
};

namespace vam {
namespace cnn {

static inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

static bool valid(const vam_cnn* h) { return h && h->magic == kCnnMagic; }

static void free_cnn(vam_cnn* h) {
  std::vector<void*> ptrs = {h->master, h->m1, h->m2, h->grad, h->z, h->g[0], h->g[1],
                             h->part, h->lpart, h->loss};
  for (auto p : h->wb) ptrs.push_back(p);
  for (auto p : h->wf) ptrs.push_back(p);
  for (auto p : h->act) ptrs.push_back(p);
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->magic = 0;
  delete h;
}

template <int EPI, bool CONVT>
static vam_status gemm(const GemmArgs& a, int splits, hipStream_t s) {
  const dim3 grid((unsigned)((a.M + BM - 1) / BM), (unsigned)((a.N + BN - 1) / BN), (unsigned)splits);
  hipLaunchKernelGGL((k_gemm<EPI, CONVT>), grid, dim3(256), 0, s, a);
  VAM_HIP_TRY(hipGetLastError(), "launching a CNN GEMM");
  return VAM_OK;
}

static vam_status pack_all(vam_cnn* h, hipStream_t s) {
  for (int l = 1; l <= h->L; ++l) {
    const int i = l - 1;
    const int n = std::max(h->coutp[i] * h->kp[i], h->cinp[i] * h->kpb[i]);
    hipLaunchKernelGGL(k_pack_weights, dim3(nblocks(n, 256)), dim3(256), 0, s, h->master + h->woff[i], h->cin[i],
                       h->cout[i], h->cinp[i], h->coutp[i], h->kp[i], h->kpb[i], h->wb[i], h->wf[i]);
  }
  VAM_HIP_TRY(hipGetLastError(), "launching the weight packing");
  return VAM_OK;
}

#define CNN_TRY(expr)                   \
  do {                                  \
    vam_status st_ = (expr);            \
    if (st_ != VAM_OK) return st_;      \
  } while (0)

// Forward pass of n images; leaves a_0 .. a_{L-1} and z in the workspace.
static vam_status forward(vam_cnn* h, const float* x, int n, hipStream_t s) {
  const int64_t npix = (int64_t)n * h->H * h->W;
  hipLaunchKernelGGL(k_pack_input, dim3(nblocks(npix, 256)), dim3(256), 0, s, x, npix, h->H * h->W, h->s0, h->s1,
                     h->act[0]);
  VAM_HIP_TRY(hipGetLastError(), "launching the input packing");
  for (int l = 1; l <= h->L; ++l) {
    const int i = l - 1;
    GemmArgs a = {};
    a.X = h->act[i];
    a.H = h->H;
    a.W = h->W;
    a.cp = h->cinp[i];
    a.B = h->wb[i];
    a.ldb = h->kp[i];
    a.M = (int)npix;
    a.N = h->cout[i];
    a.K = h->kp[i];
    a.bias = h->master + h->boff[i];
    if (l < h->L) {
      a.C = h->act[l];
      a.ldc = h->coutp[i];
      CNN_TRY((gemm<EPI_RELU_BF16, false>(a, 1, s)));
    } else {
      a.C = h->z;
      a.ldc = h->coutp[i];
      CNN_TRY((gemm<EPI_BIAS_F32, false>(a, 1, s)));
    }
  }
  return VAM_OK;
}

static int choose_splits(int64_t npix) {
  // the pixel sum of the weight gradient, in equal multiples of BK
  const int64_t tiles = npix / BK;
  int best = 1;
  for (int s = 1; s <= kMaxSplits; ++s)
    if (tiles % s == 0 && tiles / s >= 16) best = s;
  return best;
}

}  // namespace cnn
}  // namespace vam

using namespace vam;
using namespace vam::cnn;

extern "C" {

vam_status vam_cnn_create(int32_t layers, int32_t channels, int32_t height, int32_t width, int32_t max_batch,
                          float in_scale0, float in_scale1, vam_cnn_t* out) {
  clear_error();
  if (!out) return fail(VAM_ERR_INVALID_ARG, "NULL output handle");
  *out = nullptr;
  if (layers < 2 || layers > 32) return fail(VAM_ERR_INVALID_ARG, "layers must be in [2, 32]");
  if (channels < 8 || channels > 64 || channels % 8) return fail(VAM_ERR_INVALID_ARG, "channels must be 8..64, a multiple of 8");
  if (height < 1 || width < 1 || width > 1024 || height > 1024) return fail(VAM_ERR_INVALID_ARG, "image size outside [1, 1024]");
  if (max_batch < 1) return fail(VAM_ERR_INVALID_ARG, "max_batch must be positive");
  const int64_t npix = (int64_t)max_batch * height * width;
  if (npix % BK) return fail(VAM_ERR_INVALID_ARG, "max_batch * height * width must be a multiple of 32");
  if (npix * 576 >= (1LL << 40) || npix >= 0x7fffffffLL) return fail(VAM_ERR_INVALID_ARG, "batch too large");
  if (!(in_scale0 > 0.0f) || !(in_scale1 > 0.0f)) return fail(VAM_ERR_INVALID_ARG, "input scales must be positive");
  vam_cnn* h = new (std::nothrow) vam_cnn();
  if (!h) return fail(VAM_ERR_OUT_OF_MEMORY, "allocating the CNN handle");
  h->magic = kCnnMagic;
  (void)hipGetDevice(&h->device);
  h->L = layers;
  h->C = channels;
  h->H = height;
  h->W = width;
  h->maxn = max_batch;
  h->s0 = in_scale0;
  h->s1 = in_scale1;
  int64_t off = 0;
  int kmax = 0, cmax = 8;
  for (int l = 1; l <= layers; ++l) {
    const int ci = l == 1 ? 2 : channels, co = l == layers ? 1 : channels;
    h->cin.push_back(ci);
    h->cout.push_back(co);
    h->cinp.push_back(round_up(ci, 8));
    h->coutp.push_back(round_up(co, 8));
    h->kp.push_back(round_up(9 * round_up(ci, 8), BK));
    h->kpb.push_back(round_up(9 * round_up(co, 8), BK));
    h->woff.push_back(off);
    off += (int64_t)co * 9 * ci;
    h->boff.push_back(off);
    off += co;
    kmax = std::max({kmax, h->kp.back(), h->kpb.back()});
    cmax = std::max(cmax, round_up(co, 8));
  }
  h->nparam = off;
  const unsigned lblocks = nblocks(npix, 256);
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
  };
  alloc((void**)&h->master, h->nparam * 4);
  alloc((void**)&h->m1, h->nparam * 4);
  alloc((void**)&h->m2, h->nparam * 4);
  alloc((void**)&h->grad, h->nparam * 4);
  h->wb.assign(layers, nullptr);
  h->wf.assign(layers, nullptr);
  h->act.assign(layers, nullptr);
  for (int i = 0; i < layers; ++i) {
    alloc((void**)&h->wb[i], (size_t)h->coutp[i] * h->kp[i] * 2);
    if (i > 0) alloc((void**)&h->wf[i], (size_t)h->cinp[i] * h->kpb[i] * 2);
    alloc((void**)&h->act[i], (size_t)npix * h->cinp[i] * 2);
  }
  alloc((void**)&h->z, (size_t)npix * h->coutp[layers - 1] * 4);
  alloc((void**)&h->g[0], (size_t)npix * cmax * 2);
  alloc((void**)&h->g[1], (size_t)npix * cmax * 2);
  alloc((void**)&h->part, (size_t)kMaxSplits * (kmax + 1) * cmax * 4);  // choose_splits() <= kMaxSplits
  alloc((void**)&h->lpart, (size_t)lblocks * 8);
  alloc((void**)&h->loss, 8);
  if (e == hipSuccess) e = hipMemset(h->master, 0, h->nparam * 4);
  if (e == hipSuccess) e = hipMemset(h->m1, 0, h->nparam * 4);
  if (e == hipSuccess) e = hipMemset(h->m2, 0, h->nparam * 4);
  if (e == hipSuccess) e = hipMemset(h->grad, 0, h->nparam * 4);
  if (e != hipSuccess) {
    vam_status st = hip_check(e, "allocating the CNN workspace");
    free_cnn(h);
    return st;
  }
  vam_status st = pack_all(h, nullptr);
  if (st == VAM_OK && hipDeviceSynchronize() != hipSuccess) st = fail(VAM_ERR_HIP, "initialising the CNN");
  if (st != VAM_OK) {
    free_cnn(h);
    return st;
  }
  *out = h;
  return VAM_OK;
}

vam_status vam_cnn_destroy(vam_cnn_t h) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  free_cnn(h);
  return VAM_OK;
}

int64_t vam_cnn_param_count(vam_cnn_t h) { return valid(h) ? h->nparam : -1; }

vam_status vam_cnn_set_params(vam_cnn_t h, const float* params) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!params) return fail(VAM_ERR_INVALID_ARG, "NULL parameters");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  VAM_HIP_TRY(hipMemcpy(h->master, params, h->nparam * 4, hipMemcpyHostToDevice), "copying parameters");
  VAM_HIP_TRY(hipMemset(h->m1, 0, h->nparam * 4), "clearing Adam moments");
  VAM_HIP_TRY(hipMemset(h->m2, 0, h->nparam * 4), "clearing Adam moments");
  h->adam_t = 0;
  CNN_TRY(pack_all(h, nullptr));
  VAM_HIP_TRY(hipDeviceSynchronize(), "packing weights");
  return VAM_OK;
}

vam_status vam_cnn_get_params(vam_cnn_t h, float* params) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!params) return fail(VAM_ERR_INVALID_ARG, "NULL parameters");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  VAM_HIP_TRY(hipDeviceSynchronize(), "synchronising");
  VAM_HIP_TRY(hipMemcpy(params, h->master, h->nparam * 4, hipMemcpyDeviceToHost), "copying parameters");
  return VAM_OK;
}

vam_status vam_cnn_get_state(vam_cnn_t h, float* state, int64_t* adam_steps) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!state || !adam_steps) return fail(VAM_ERR_INVALID_ARG, "NULL argument");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  VAM_HIP_TRY(hipDeviceSynchronize(), "synchronising");
  VAM_HIP_TRY(hipMemcpy(state, h->master, h->nparam * 4, hipMemcpyDeviceToHost), "copying parameters");
  VAM_HIP_TRY(hipMemcpy(state + h->nparam, h->m1, h->nparam * 4, hipMemcpyDeviceToHost), "copying moments");
  VAM_HIP_TRY(hipMemcpy(state + 2 * h->nparam, h->m2, h->nparam * 4, hipMemcpyDeviceToHost), "copying moments");
  *adam_steps = h->adam_t;
  return VAM_OK;
}

vam_status vam_cnn_set_state(vam_cnn_t h, const float* state, int64_t adam_steps) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!state) return fail(VAM_ERR_INVALID_ARG, "NULL state");
  if (adam_steps < 0 || adam_steps > (int64_t)1 << 40) return fail(VAM_ERR_INVALID_ARG, "bad Adam step count");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  VAM_HIP_TRY(hipDeviceSynchronize(), "synchronising");
  VAM_HIP_TRY(hipMemcpy(h->master, state, h->nparam * 4, hipMemcpyHostToDevice), "copying parameters");
  VAM_HIP_TRY(hipMemcpy(h->m1, state + h->nparam, h->nparam * 4, hipMemcpyHostToDevice), "copying moments");
  VAM_HIP_TRY(hipMemcpy(h->m2, state + 2 * h->nparam, h->nparam * 4, hipMemcpyHostToDevice), "copying moments");
  h->adam_t = (int)adam_steps;
  CNN_TRY(pack_all(h, nullptr));
  VAM_HIP_TRY(hipDeviceSynchronize(), "packing weights");
  return VAM_OK;
}

vam_status vam_cnn_get_grads(vam_cnn_t h, float* grads) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!grads) return fail(VAM_ERR_INVALID_ARG, "NULL gradients");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  VAM_HIP_TRY(hipDeviceSynchronize(), "synchronising");
  VAM_HIP_TRY(hipMemcpy(grads, h->grad, h->nparam * 4, hipMemcpyDeviceToHost), "copying gradients");
  return VAM_OK;
}

vam_status vam_cnn_forward(vam_cnn_t h, const float* x, int32_t n, float* y, hipStream_t s) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!x || !y) return fail(VAM_ERR_INVALID_ARG, "NULL buffer");
  if (n < 1 || n > h->maxn) return fail(VAM_ERR_INVALID_ARG, "batch %d outside [1, %d]", n, h->maxn);
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  CNN_TRY(forward(h, x, n, s));
  const int64_t npix = (int64_t)n * h->H * h->W;
  hipLaunchKernelGGL(k_output, dim3(nblocks(npix, 256)), dim3(256), 0, s, h->z, h->coutp[h->L - 1], x, npix,
                     h->H * h->W, h->s1, y);
  VAM_HIP_TRY(hipGetLastError(), "launching the CNN output");
  return VAM_OK;
}

vam_status vam_cnn_loss_grad(vam_cnn_t h, const float* x, const float* t, int32_t n, double* loss_out,
                             hipStream_t s) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!x || !t) return fail(VAM_ERR_INVALID_ARG, "NULL buffer");
  if (n < 1 || n > h->maxn) return fail(VAM_ERR_INVALID_ARG, "batch %d outside [1, %d]", n, h->maxn);
  const int64_t npix = (int64_t)n * h->H * h->W;
  if (npix % BK) return fail(VAM_ERR_INVALID_ARG, "n * height * width must be a multiple of 32");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  CNN_TRY(forward(h, x, n, s));
  const int L = h->L;
  const unsigned lblocks = nblocks(npix, 256);
  // g_L = d loss / d z (8 channels, channel 0 used)
  uint16_t* gcur = h->g[0];
  uint16_t* gnext = h->g[1];
  hipLaunchKernelGGL(k_loss, dim3(lblocks), dim3(256), 0, s, h->z, h->coutp[L - 1], x, t, npix, h->H * h->W, h->s1,
                     gcur, h->lpart);
  hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(256), 0, s, h->lpart, (int)lblocks, 1.0 / (double)npix, h->loss);
  VAM_HIP_TRY(hipGetLastError(), "launching the CNN loss");
  const int splits = choose_splits(npix);
  const int ksplit = (int)(npix / splits);
  for (int l = L; l >= 1; --l) {
    const int i = l - 1;
    // weight gradient: dW^T[kc][co] = sum_p col(a_{l-1})[p][kc] g_l[p][co],
    // both operands staged along the pixel sum straight from a_{l-1} and g_l
    GemmArgs a = {};
    a.X = h->act[i];
    a.H = h->H;
    a.W = h->W;
    a.cp = h->cinp[i];
    a.G = gcur;
    a.cpg = h->coutp[i];
    // rows 0 .. kp - 1 of dW^T, then row kp = sum_p g_l[p][co] (the bias
    // gradient, from a row of ones in A)
    a.M = h->kp[i] + 1;
    a.ones_row = h->kp[i];
    a.N = h->cout[i];
    a.K = ksplit;
    a.C = h->part;
    a.ldc = h->coutp[i];
    a.split_stride = (int64_t)(h->kp[i] + 1) * h->coutp[i];
    CNN_TRY((gemm<EPI_PART_F32, true>(a, splits, s)));
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblocks(a.split_stride, 64)), dim3(256), 0, s, h->part, splits, a.split_stride,
                       h->coutp[i], h->cinp[i], h->cin[i], h->cout[i], h->kp[i], h->grad + h->woff[i],
                       h->grad + h->boff[i]);
    VAM_HIP_TRY(hipGetLastError(), "launching the gradient reductions");
    if (l == 1) break;
    // data gradient through the ReLU of a_{l-1}
    GemmArgs d = {};
    d.X = gcur;
    d.H = h->H;
    d.W = h->W;
    d.cp = h->coutp[i];
    d.B = h->wf[i];
    d.ldb = h->kpb[i];
    d.M = (int)npix;
    d.N = h->cinp[i];
    d.K = h->kpb[i];
    d.C = gnext;
    d.ldc = h->cinp[i];
    d.mask = h->act[i];
    d.ldm = h->cinp[i];
    CNN_TRY((gemm<EPI_MASK_BF16, false>(d, 1, s)));
    std::swap(gcur, gnext);
  }
  if (loss_out) {
    VAM_HIP_TRY(hipMemcpyAsync(loss_out, h->loss, 8, hipMemcpyDeviceToHost, s), "reading the loss");
    VAM_HIP_TRY(hipStreamSynchronize(s), "synchronising");
  }
  return VAM_OK;
}

vam_status vam_cnn_adam_step(vam_cnn_t h, float lr, float beta1, float beta2, float eps, hipStream_t s) {
  clear_error();
  if (!valid(h)) return fail(VAM_ERR_BAD_HANDLE, "not a live CNN handle");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(VAM_ERR_INVALID_ARG, "Adam parameters out of range");
  VAM_HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  h->adam_t += 1;
  const float c1 = 1.0f - (float)std::pow((double)beta1, h->adam_t);
  const float c2 = 1.0f - (float)std::pow((double)beta2, h->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(nblocks(h->nparam, 256)), dim3(256), 0, s, h->master, h->m1, h->m2, h->grad,
                     h->nparam, lr, beta1, beta2, eps, c1, c2);
  VAM_HIP_TRY(hipGetLastError(), "launching Adam");
  return pack_all(h, s);
}

}  // extern "C"
