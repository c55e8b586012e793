// Mean structural similarity (MSSIM) of each image's reconstruction against
// its source: the paper's third quality measure (§4.1, from the SSIM of Wang
// et al. 2004: 11 x 11 Gaussian window, standard deviation 1.5, C1 =
// (0.01 * 255)^2, C2 = (0.03 * 255)^2, every window position inside the
// image, averaged).
//
// rklt_ssim_tiles_kernel: a workgroup codes output tiles of 32 x 64 window
// positions.  It stages the 42 x 74 source and reconstruction pixels the
// tile needs in LDS (minus 128, which keeps the second moments small), runs
// the horizontal 11-tap pass of the five quantities x, y, x^2, y^2, xy into
// LDS, then each thread runs the vertical pass for 8 positions of one column
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

// normalised 1D Gaussian taps (the 2D window is their outer product)
__device__ __forceinline__ float gtap(int k) {
  // exp(-(k - 5)^2 / (2 * 1.5^2)) / sum; computed once per thread
  float s = 0.0f;
  for (int i = 0; i < 11; ++i) s += expf(-static_cast<float>((i - 5) * (i - 5)) / 4.5f);
  return expf(-static_cast<float>((k - 5) * (k - 5)) / 4.5f) / s;
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
    // stage the pixels (outside the image: zero; they only feed positions
    // that are not evaluated)
    for (int e = threadIdx.x; e < kIH * kIW; e += blockDim.x) {
      const int r = e / kIW, c = e % kIW;
      const bool in = y0 + r < H && x0 + c < W;
      const uint32_t ox = in ? static_cast<uint32_t>(y0 + r) * im->px + (x0 + c) : 0x80000000u;
      const uint32_t oy = in ? static_cast<uint32_t>(y0 + r) * im->py + (x0 + c) : 0x80000000u;
      sx[r][c] = static_cast<float>(__builtin_amdgcn_raw_buffer_load_b8(rx, ox, 0, 0)) - 128.0f;
      sy[r][c] = static_cast<float>(__builtin_amdgcn_raw_buffer_load_b8(ry, oy, 0, 0)) - 128.0f;
    }
    __syncthreads();
    // horizontal pass: (row r, 16 columns from c0) per work item
    for (int e = threadIdx.x; e < kIH * (kTW / 16); e += blockDim.x) {
      const int r = e / (kTW / 16), c0 = (e % (kTW / 16)) * 16;
      float vx[26], vy[26];
#pragma unroll
      for (int k = 0; k < 26; ++k) {
        vx[k] = sx[r][c0 + k];
        vy[k] = sy[r][c0 + k];
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f, m4 = 0.0f;
#pragma unroll
        for (int k = 0; k < 11; ++k) {
          const float X = vx[c + k], Y = vy[c + k];
          m0 = fmaf(g[k], X, m0);
          m1 = fmaf(g[k], Y, m1);
          m2 = fmaf(g[k], X * X, m2);
          m3 = fmaf(g[k], Y * Y, m3);
          m4 = fmaf(g[k], X * Y, m4);
        }
        sh[0][r][c0 + c] = m0;
        sh[1][r][c0 + c] = m1;
        sh[2][r][c0 + c] = m2;
        sh[3][r][c0 + c] = m3;
        sh[4][r][c0 + c] = m4;
      }
    }
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
        if (r0 + i < vh) sum += num / den;
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
