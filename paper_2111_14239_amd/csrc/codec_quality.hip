// Mean structural similarity (MSSIM) of each image's reconstruction against
// its source: the paper's third quality measure (§4.1, from the SSIM of Wang
// et al. 2004: 11 x 11 Gaussian window, standard deviation 1.5, C1 =
// (0.01 * 255)^2, C2 = (0.03 * 255)^2, every window position inside the
// image, averaged).
//
// rklt_ssim_tiles_kernel: a workgroup codes output tiles of 32 x 64 window
// positions.  It runs the horizontal 11-tap pass of the five quantities x,
// y, x^2, y^2, xy over the 42 x 74 source and reconstruction pixels the tile
// needs (read from the images into registers, minus 128, which keeps the
// second moments small) into LDS, then each thread runs the vertical pass
// for 8 positions of one column in registers, evaluates SSIM and adds it
// up.  Each tile's sum goes to its
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

// W horizontal-pass outputs of tile row r from tile column c0: the 11-tap
// weighted sums of x, y, x^2, y^2 and xy, one quantity after another.  The
// W + 10 pixels of x and y are read from the images as 32-bit words (rows
// start on 8-byte boundaries and W, x0 and c0 are multiples of 4, so each
// word is aligned and lies wholly inside or wholly past its row; past the
// last row the buffer reads zero); pixels outside the image only feed
// positions that are not evaluated.  Pixels are taken minus 128, which keeps
// the second moments below 128^2 and the FP32 cancellation in E[x^2] - mu^2
// small.
template <int W>
__device__ __forceinline__ void hpass(__amdgpu_buffer_rsrc_t rx, __amdgpu_buffer_rsrc_t ry, uint32_t ox,
                                      uint32_t oy, float (*sh)[kIH][kTW + 1], int r, int c0, const float* g) {
  constexpr int kN = W + 10, kWords = (kN + 3) / 4;
  float vx[kN], vy[kN];
#pragma unroll
  for (int w = 0; w < kWords; ++w) {
    const uint32_t wx = __builtin_amdgcn_raw_buffer_load_b32(rx, ox + (ox == 0x80000000u ? 0u : 4u * w), 0, 0);
    const uint32_t wy = __builtin_amdgcn_raw_buffer_load_b32(ry, oy + (oy == 0x80000000u ? 0u : 4u * w), 0, 0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (4 * w + b < kN) {
        vx[4 * w + b] = static_cast<float>((wx >> (8 * b)) & 0xffu) - 128.0f;
        vy[4 * w + b] = static_cast<float>((wy >> (8 * b)) & 0xffu) - 128.0f;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    float v[kN];
#pragma unroll
    for (int k = 0; k < kN; ++k)
      v[k] = q == 0 ? vx[k] : q == 1 ? vy[k] : q == 2 ? vx[k] * vx[k] : q == 3 ? vy[k] * vy[k] : vx[k] * vy[k];
#pragma unroll
    for (int c = 0; c < W; ++c) {
      float m = 0.0f;
#pragma unroll
      for (int k = 0; k < 11; ++k) m = fmaf(g[k], v[c + k], m);
      sh[q][r][c0 + c] = m;
    }
  }
}

__global__ __launch_bounds__(256) void rklt_ssim_tiles_kernel(MsArgs a) {
  // horizontal pass: mu_x, mu_y, x^2, y^2, xy (54600 bytes: three
  // workgroups fit a CU's LDS; the workgroup sums reuse its first bytes)
  __shared__ float sh[5][kIH][kTW + 1];
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
    auto row_offset = [&](int r, int c0, int pitch) {
      return y0 + r < H ? static_cast<uint32_t>(y0 + r) * pitch + (x0 + c0) : 0x80000000u;
    };
    __syncthreads();  // the previous tile's LDS reads are done
    // horizontal pass: rows 0 .. 31 in items of 8 outputs (256 items, one
    // per thread), the last 10 rows in items of 4 (160 items), so no wave
    // runs more than 12 outputs
    {
      const int r = threadIdx.x / (kTW / 8), c0 = (threadIdx.x % (kTW / 8)) * 8;
      hpass<8>(rx, ry, row_offset(r, c0, im->px), row_offset(r, c0, im->py), sh, r, c0, g);
    }
    if (threadIdx.x < (kIH - 32) * (kTW / 4)) {
      const int r = 32 + threadIdx.x / (kTW / 4), c0 = (threadIdx.x % (kTW / 4)) * 4;
      hpass<4>(rx, ry, row_offset(r, c0, im->px), row_offset(r, c0, im->py), sh, r, c0, g);
    }
    __syncthreads();
    // vertical pass and SSIM: column c, rows r0 .. r0 + 7, one quantity
    // after another (m[q][i] in the same tap order as before)
    const int c = threadIdx.x % kTW, r0 = (threadIdx.x / kTW) * 8;
    const int vh = H - 10 - y0, vw = W - 10 - x0;  // valid positions in this tile
    float sum = 0.0f;
    if (c < vw) {
      float m[5][8];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float col[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) col[k] = sh[q][r0 + k][c];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          float acc = 0.0f;
#pragma unroll
          for (int k = 0; k < 11; ++k) acc = fmaf(g[k], col[i + k], acc);
          m[q][i] = acc;
        }
      }
      const float C1 = 6.5025f, C2 = 58.5225f;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        // m[0], m[1]: means of x - 128, y - 128
        const float mx = m[0][i] + 128.0f, my = m[1][i] + 128.0f;
        const float vxx = m[2][i] - m[0][i] * m[0][i], vyy = m[3][i] - m[1][i] * m[1][i];
        const float cxy = m[4][i] - m[0][i] * m[1][i];
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
    __syncthreads();  // every read of sh is done: its first bytes take the wave sums
    double* const red = reinterpret_cast<double*>(&sh[0][0][0]);
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
