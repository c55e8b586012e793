// Mean structural similarity (MSSIM) of each image's reconstruction against
// its source: the paper's third quality measure (§4.1, from the SSIM of Wang
// et al. 2004: 11 x 11 Gaussian window, standard deviation 1.5, C1 =
// (0.01 * 255)^2, C2 = (0.03 * 255)^2, every window position inside the
// image, averaged).
//
// rklt_ssim_tiles_kernel: a workgroup codes output tiles of 32 x 64 window
// positions.  It stages the 42 x 74 source and reconstruction pixels the
// tile needs in LDS (minus 128, which keeps the second moments small), runs
// the horizontal 11-tap pass of the five quantities x, y, x^2, y^2, xy from
// registers into LDS, then each thread runs the vertical pass for 8 positions of one column
// in registers, evaluates SSIM and adds it up.  Each tile's sum goes to its
// own slot (double), and rklt_ssim_mean_kernel adds an image's slots in a
// fixed order and divides by the number of positions, so the result does
// not depend on scheduling.  FP32 arithmetic, double sums.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.h"
#include "rklt_internal.h"

namespace rklt {
namespace {

constexpr int kTW = kMsTileW, kTH = kMsTileH;  // window positions per tile
constexpr int kIW = kTW + 10, kIH = kTH + 10;  // pixels the tile reads
constexpr int kQuality = 0x00020000;        // raw buffer resource flags
static_assert(kTH == 32 && kTW == 64, "the work split below assumes 32 x 64 tiles of 256 threads");

// normalised 1D Gaussian taps (the 2D window is their outer product)
__device__ __forceinline__ float gtap(int k) {
  // exp(-(k - 5)^2 / (2 * 1.5^2)) / sum; computed once per thread
  float s = 0.0f;
  for (int i = 0; i < 11; ++i) s += expf(-static_cast<float>((i - 5) * (i - 5)) / 4.5f);
  return expf(-static_cast<float>((k - 5) * (k - 5)) / 4.5f) / s;
}

// W horizontal-pass outputs of row r from column c0: the 11-tap weighted
// sums of x, y, x^2, y^2 and xy; the products are formed once per pixel
template <int W>
__device__ __forceinline__ void hpass(const float (*sx)[kIW + 1], const float (*sy)[kIW + 1],
                                      float (*sh)[kIH][kTW + 1], int r, int c0, const float* g) {
  float vx[W + 10], vy[W + 10], vxx[W + 10], vyy[W + 10], vxy[W + 10];
#pragma unroll
  for (int k = 0; k < W + 10; ++k) {
    vx[k] = sx[r][c0 + k];
    vy[k] = sy[r][c0 + k];
    vxx[k] = vx[k] * vx[k];
    vyy[k] = vy[k] * vy[k];
    vxy[k] = vx[k] * vy[k];
  }
#pragma unroll
  for (int c = 0; c < W; ++c) {
    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f, m4 = 0.0f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      m0 = fmaf(g[k], vx[c + k], m0);
      m1 = fmaf(g[k], vy[c + k], m1);
      m2 = fmaf(g[k], vxx[c + k], m2);
      m3 = fmaf(g[k], vyy[c + k], m3);
      m4 = fmaf(g[k], vxy[c + k], m4);
    }
    sh[0][r][c0 + c] = m0;
    sh[1][r][c0 + c] = m1;
    sh[2][r][c0 + c] = m2;
    sh[3][r][c0 + c] = m3;
    sh[4][r][c0 + c] = m4;
  }
}

__global__ __launch_bounds__(256) void rklt_ssim_tiles_kernel(MsArgs a) {
  __shared__ float sx[kIH][kIW + 1];
  __shared__ float sy[kIH][kIW + 1];
  __shared__ float sh[5][kIH][kTW + 1];  // horizontal pass: mu_x, mu_y, x^2, y^2, xy
  __shared__ double red[4];
  float g[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) g[k] = gtap(k);
  const ConstMsImage imgs = (ConstMsImage)(a.imgs);
  for (int t = blockIdx.x; t < a.total; t += gridDim.x) {
    // the image of tile t: the last k with tile0 <= t (binary search)
    int lo = 0, hi = a.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (imgs[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const ConstMsImage im = imgs + lo;
    const int H = im->H, W = im->W, across = im->across;
    const int lt = t - im->tile0;
    const int y0 = (lt / across) * kTH, x0 = (lt % across) * kTW;
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(im->x), 0, (H - 1) * im->px + W, kQuality);
    const __amdgpu_buffer_rsrc_t ry =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(im->y), 0, (H - 1) * im->py + W, kQuality);
    __syncthreads();  // the previous tile's LDS reads are done
    // stage the pixels, four per load: image rows start on 8-byte boundaries
    // and W and x0 are multiples of 4, so each word is aligned and lies
    // wholly inside or wholly past its row (past the last row it reads zero);
    // pixels outside the image only feed positions that are not evaluated
    constexpr int kWords = (kIW + 3) / 4;
    for (int e = threadIdx.x; e < kIH * kWords; e += blockDim.x) {
      const int r = e / kWords, w = e % kWords;
      const bool in = y0 + r < H;
      const uint32_t ox = in ? static_cast<uint32_t>(y0 + r) * im->px + (x0 + 4 * w) : 0x80000000u;
      const uint32_t oy = in ? static_cast<uint32_t>(y0 + r) * im->py + (x0 + 4 * w) : 0x80000000u;
      const uint32_t vx = __builtin_amdgcn_raw_buffer_load_b32(rx, ox, 0, 0);
      const uint32_t vy = __builtin_amdgcn_raw_buffer_load_b32(ry, oy, 0, 0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (4 * w + b < kIW) {
          sx[r][4 * w + b] = static_cast<float>((vx >> (8 * b)) & 0xffu) - 128.0f;
          sy[r][4 * w + b] = static_cast<float>((vy >> (8 * b)) & 0xffu) - 128.0f;
        }
      }
    }
    __syncthreads();
    // horizontal pass: rows 0 .. 31 in items of 8 outputs (256 items, one
    // per thread), the last 10 rows in items of 4 (160 items), so no wave
    // runs more than 12 outputs
    hpass<8>(sx, sy, sh, threadIdx.x / (kTW / 8), (threadIdx.x % (kTW / 8)) * 8, g);
    if (threadIdx.x < (kIH - 32) * (kTW / 4))
      hpass<4>(sx, sy, sh, 32 + threadIdx.x / (kTW / 4), (threadIdx.x % (kTW / 4)) * 4, g);
    __syncthreads();
    // vertical pass and SSIM: column c, rows r0 .. r0 + 7
    const int c = threadIdx.x % kTW, r0 = (threadIdx.x / kTW) * 8;
    const int vh = H - 10 - y0, vw = W - 10 - x0;  // valid positions in this tile
    float sum = 0.0f;
    if (c < vw) {
      float col[5][18];
#pragma unroll
      for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int k = 0; k < 18; ++k) col[q][k] = sh[q][r0 + k][c];
      const float C1 = 6.5025f, C2 = 58.5225f;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 11; ++k)
#pragma unroll
          for (int q = 0; q < 5; ++q) m[q] = fmaf(g[k], col[q][i + k], m[q]);
        // m[0], m[1]: means of x - 128, y - 128
        const float mx = m[0] + 128.0f, my = m[1] + 128.0f;
        const float vxx = m[2] - m[0] * m[0], vyy = m[3] - m[1] * m[1], cxy = m[4] - m[0] * m[1];
        const float num = (2.0f * mx * my + C1) * (2.0f * cxy + C2);
        const float den = (mx * mx + my * my + C1) * (vxx + vyy + C2);
        // one rounding of the reciprocal (1 ulp) instead of a correctly
        // rounded division; den > 0 (the variances are negative only by
        // rounding, far less than C2)
        if (r0 + i < vh) sum += num * __builtin_amdgcn_rcpf(den);
      }
    }
    // workgroup sum in double, one slot per tile
    double s = static_cast<double>(sum);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) a.partials[t] = red[0] + red[1] + red[2] + red[3];
  }
}

// One workgroup per image: the image's tile sums in a fixed order, divided
// by the number of window positions; NaN for an image without a
// reconstruction or smaller than the window.
__global__ __launch_bounds__(256) void rklt_ssim_mean_kernel(MsArgs a) {
  __shared__ double red[4];
  const ConstMsImage im = (ConstMsImage)(a.imgs) + blockIdx.x;
  const int t0 = im->tile0, nt = im->ntiles;
  double s = 0.0;
  for (int k = threadIdx.x; k < nt; k += blockDim.x) s += a.partials[t0 + k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double total = red[0] + red[1] + red[2] + red[3];
    const double count = static_cast<double>(im->H - 10) * static_cast<double>(im->W - 10);
    a.out[im->slot] = nt > 0 ? total / count : __builtin_nan("");
  }
}

}  // namespace

rklt_status launch_mssim(const MsArgs& a, int grid, void* stream) {
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.total > 0) hipLaunchKernelGGL(rklt_ssim_tiles_kernel, dim3(grid), dim3(256), 0, st, a);
  hipLaunchKernelGGL(rklt_ssim_mean_kernel, dim3(a.n), dim3(256), 0, st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RKLT_E_HIP, "rklt_ssim kernels: launch failed: %s", hipGetErrorString(e));
  return RKLT_OK;
}

}  // namespace rklt
