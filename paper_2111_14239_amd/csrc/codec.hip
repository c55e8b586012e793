// HIP kernels of the rounded-KLT block codec for gfx950 (§4.1, Appendix A):
// forward B = T (A - ell) T^T in exact integers, scaling by s_i s_j and
// zig-zag zonal truncation in FP32, inverse with T_hat^-1 in FP32, rounding
// floor(x + 1/2), clipping, and the per-image squared error with PSNR.
//
// The register kernel below shares the tile / result protocol with the
// matrix-core kernel (codec_mfma.hip) and the panel kernel (codec_panel.hip):
//   * rklt_block8_kernel: N = 8, level shift 128, int8-range T.  One thread codes whole
//     8 x 8 blocks in registers: pixels arrive as two 32-bit words per row
//     (coalesced across the wave: 64 lanes read 512 contiguous bytes per
//     row), the row transform is v_dot4 on int8 (pixel xor 0x80 = pixel -
//     128), the column transform v_dot2 on int16 pairs.  Only the
//     anti-diagonals i + j < D that hold kept coefficients are computed
//     (D is a template parameter), so truncation removes work instead of
//     masking it.
//
// Work list: a tile is a run of consecutive blocks of one image.  A
// workgroup loops over tiles (persistent grid for a plan, one tile per
// workgroup for the plain path), reduces its squared error, adds it to the
// image's accumulator and counts the tile done; the workgroup that finishes
// an image's last tile writes SSE, MSE and PSNR and resets the accumulators.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.h"
#include "rklt_internal.h"

namespace rklt {
namespace {

// Code one 8 x 8 block with level shift 128.  s/d point at its top-left
// pixel; sxx accumulates sum(x^2) + sum(y^2) and sxy sum(x y) over the
// original x and the reconstruction y.
//
// The scaling and the inverse merge: T_hat^-1 = T^-1 S^-1, so
//   T_hat^-1 (mask (.) (s s^T) (.) B) T_hat^-T = T^-1 (mask (.) B) T^-T,
// and with T^-1 = adj / den (integer adj) the reconstruction is
//   A' - 128 = Out / den^2,   Out = adj (mask (.) B) adj^T.
// Both inverse stages run as FP32 FMAs on integer values; the host checked
// that every product and partial sum stays below 2^24 in magnitude, so each
// FMA is exact and Out is the exact integer.  The scaled coefficients
// s_i s_j B_ij are written only by the verification dump.  Pixels are
// floor(Out / den^2 + 1/2) + 128, clipped: Out * inv_den2 + (128 + delta)
// lies within 4e-5 of the exact value plus delta, half the 1/den^2 spacing
// of the rationals away from every rounding boundary, so the saturating
// round-to-nearest byte conversion returns the exact result, ties included.
//
// Loop order keeps few table words live: rows i of B outer in the forward
// column stage (one row of T and one column of adj at a time), output
// columns n outer in the last inverse stage (one row of adj at a time).
template <int D, bool DUMP>
__device__ __forceinline__ void block8(const uint8_t* __restrict__ s, int ps, uint8_t* __restrict__ d,
                                       int pd, const DevTransform* __restrict__ table, int tid, int r,
                                       int32_t* __restrict__ coef, float* __restrict__ scaled,
                                       uint32_t& sxx, uint32_t& sxy) {
  constexpr int C = D < 8 ? D : 8;  // columns j (and rows i) that hold a kept coefficient
  // Opaque transform index: the table is read from the scalar cache where it
  // is used, and loads are not shared (and kept live) across the D variants
  // or across consecutive blocks.
  asm volatile("" : "+s"(tid));
  const ConstTransform tf = as_constant(table + tid);

  u32x2 px[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) px[m] = *as_global(reinterpret_cast<const u32x2*>(s + static_cast<size_t>(m) * ps));

  // Rows: Y[m][j] = sum_n X[m][n] T[j][n], X = pixel - 128 = pixel xor 0x80
  // (int8 dots), kept as int16 pairs P[p][j] = (Y[2p][j], Y[2p+1][j]).
  int P[4][C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int t0 = tf->t8[j][0], t1 = tf->t8[j][1];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int m0 = 2 * p, m1 = 2 * p + 1;
      const int y0 = __builtin_amdgcn_sdot4(static_cast<int>(px[m0].y ^ 0x80808080u), t1,
                                            __builtin_amdgcn_sdot4(static_cast<int>(px[m0].x ^ 0x80808080u), t0, 0, false),
                                            false);
      const int y1 = __builtin_amdgcn_sdot4(static_cast<int>(px[m1].y ^ 0x80808080u), t1,
                                            __builtin_amdgcn_sdot4(static_cast<int>(px[m1].x ^ 0x80808080u), t0, 0, false),
                                            false);
      P[p][j] = static_cast<int>(__builtin_amdgcn_perm(static_cast<uint32_t>(y1), static_cast<uint32_t>(y0), 0x05040100u));
    }
  }

  // Columns and first inverse stage:
  //   B[i][j] = sum_m T[i][m] Y[m][j]                      (int16 dots)
  //   W[m][j] = sum_{i : (i, j) kept} adj[m][i] B[i][j]    (exact FP32)
  float W[8][C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int jmax = (D - i) < 8 ? (D - i) : 8;
#pragma unroll
    for (int j = 0; j < jmax; ++j) {
      int B = dot2(tf->t16[i][0], P[0][j], 0);
#pragma unroll
      for (int p = 1; p < 4; ++p) B = dot2(tf->t16[i][p], P[p][j], B);
      if (DUMP) {
        if (coef) as_global(coef)[i * 8 + j] = B;
        if (scaled) as_global(scaled)[i * 8 + j] = static_cast<float>(B) * tf->w[i * 8 + j];
      }
      float c = static_cast<float>(B);
      // Zonal mask.  With D from r, every position on the anti-diagonals
      // before D - 1 has zig-zag rank < r, so only the last one is tested;
      // the dump computes all 64 coefficients and tests every position.
      if ((DUMP || i + j == D - 1) && zz_rank(8, i, j) >= r) c = 0.0f;
#pragma unroll
      for (int m = 0; m < 8; ++m)
        W[m][j] = (i == 0) ? tf->fadj[m * 8 + i] * c : fmaf(tf->fadj[m * 8 + i], c, W[m][j]);
    }
  }

  // Second inverse stage, output column n outer:
  //   Out[m][n] = sum_j W[m][j] adj[n][j];  pixel = RNE(Out * inv_den2 + bias)
  const float inv = tf->inv_den2, bias = tf->bias;
  uint32_t out[8][2];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      float acc = W[m][0] * tf->fadj[n * 8 + 0];
#pragma unroll
      for (int j = 1; j < C; ++j) acc = fmaf(W[m][j], tf->fadj[n * 8 + j], acc);
      const float y = fmaf(acc, inv, bias);
      out[m][n >> 2] = __builtin_amdgcn_cvt_pk_u8_f32(y, n & 3, (n & 3) ? out[m][n >> 2] : 0u);
    }
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const uint32_t lo = out[m][0], hi = out[m][1];
    if (d) {
      u32x2 o;
      o.x = lo;
      o.y = hi;
      *as_global(reinterpret_cast<u32x2*>(d + static_cast<size_t>(m) * pd)) = o;
    }
    sxx = __builtin_amdgcn_udot4(px[m].x, px[m].x, sxx, false);
    sxx = __builtin_amdgcn_udot4(px[m].y, px[m].y, sxx, false);
    sxx = __builtin_amdgcn_udot4(lo, lo, sxx, false);
    sxx = __builtin_amdgcn_udot4(hi, hi, sxx, false);
    sxy = __builtin_amdgcn_udot4(px[m].x, lo, sxy, false);
    sxy = __builtin_amdgcn_udot4(px[m].y, hi, sxy, false);
  }
}

template <bool DUMP>
__device__ __forceinline__ void block8_dispatch(int D, const uint8_t* s, int ps, uint8_t* d, int pd,
                                                const DevTransform* table, int tid, int r,
                                                int32_t* coef, float* scaled, uint32_t& sxx,
                                                uint32_t& sxy) {
#define RKLT_CASE(DD) \
  case DD:            \
    block8<DD, DUMP>(s, ps, d, pd, table, tid, r, coef, scaled, sxx, sxy); \
    break;
  switch (D) {
    RKLT_CASE(1) RKLT_CASE(2) RKLT_CASE(3) RKLT_CASE(4) RKLT_CASE(5) RKLT_CASE(6) RKLT_CASE(7)
    RKLT_CASE(8) RKLT_CASE(9) RKLT_CASE(10) RKLT_CASE(11) RKLT_CASE(12) RKLT_CASE(13)
    RKLT_CASE(14)
    default:
      block8<15, DUMP>(s, ps, d, pd, table, tid, r, coef, scaled, sxx, sxy);
      break;
  }
#undef RKLT_CASE
}

// PLAN: a batch plan's work list (persistent grid); otherwise the plain
// path's single image from the kernel argument, one tile per workgroup.
template <bool PLAN>
__global__ __launch_bounds__(256) void rklt_block8_kernel(KArgs a) {
  __shared__ unsigned long long red[4];
  for (int tile = tile_begin(a.total_tiles); tile < tile_end_of(a.total_tiles); ++tile) {
    const int ii = PLAN ? __builtin_amdgcn_readfirstlane(a.tile_img[tile]) : 0;
    const DevImage* im = PLAN ? a.imgs + ii : &a.one;
    const int tid = __builtin_amdgcn_readfirstlane(im->tid);
    const int tile_blocks = im->tile_blocks;
    const int b0 = (tile - im->tile0) * tile_blocks;
    const int nblocks = im->nblocks, bw = im->bw, ps = im->ps, pd = im->pd;
    const int r = im->r, D = a.dump ? 15 : im->D;
    uint32_t sxx = 0, sxy = 0;
    for (int k = 0; k * static_cast<int>(blockDim.x) < tile_blocks; ++k) {
      const int b = b0 + k * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
      if (b < nblocks) {
        const int by = b / bw, bx = b - by * bw;
        const uint8_t* s = im->src + static_cast<size_t>(by) * 8 * ps + bx * 8;
        uint8_t* d = im->dst ? im->dst + static_cast<size_t>(by) * 8 * pd + bx * 8 : nullptr;
        if (a.dump) {
          int32_t* coef = im->coef ? im->coef + static_cast<size_t>(b) * 64 : nullptr;
          float* scaled = im->scaled ? im->scaled + static_cast<size_t>(b) * 64 : nullptr;
          block8<15, true>(s, ps, d, pd, a.tf, tid, r, coef, scaled, sxx, sxy);
        } else {
          block8_dispatch<false>(D, s, ps, d, pd, a.tf, tid, r, nullptr, nullptr, sxx, sxy);
        }
      }
    }
    const uint32_t mine = sxx - 2u * sxy;
    reduce_and_finish(mine, red, a.res + im->slot, 1, im->ntiles, static_cast<long long>(im->H) * im->W);
  }
}

__global__ __launch_bounds__(256) void rklt_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

rklt_status launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RKLT_E_HIP, "%s: launch failed: %s", what, hipGetErrorString(e));
  return RKLT_OK;
}

}  // namespace

rklt_status launch_block8(const KArgs& a, int grid, int wg, void* stream) {
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.imgs) hipLaunchKernelGGL(rklt_block8_kernel<true>, dim3(grid), dim3(wg), 0, st, a);
  else hipLaunchKernelGGL(rklt_block8_kernel<false>, dim3(grid), dim3(wg), 0, st, a);
  return launched("rklt_block8_kernel");
}

rklt_status launch_copy(const void* src, void* dst, size_t nbytes, void* stream) {
  const size_t n = nbytes / 16;
  if (n == 0) return RKLT_OK;
  size_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(rklt_copy_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  return launched("rklt_copy_kernel");
}

}  // namespace rklt
