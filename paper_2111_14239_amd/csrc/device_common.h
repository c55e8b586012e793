// Device helpers shared by the codec kernels: address-space casts, the
// zig-zag rank, and the per-tile squared-error reduction with the fence-free
// per-image finalisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "rklt_internal.h"

namespace rklt {
namespace {

typedef short short2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// The transform table never changes while a kernel runs: reading it through
// the constant address space lets every wave-uniform read become a scalar
// load into SGPRs, even after the kernel has stored pixels.
typedef const __attribute__((address_space(4))) DevTransform* ConstTransform;
__device__ __forceinline__ ConstTransform as_constant(const DevTransform* p) {
  return (ConstTransform)(p);
}

// The plan's work list is written before the launch and only read by the
// kernels: constant-address-space reads become scalar loads that no pixel
// store can invalidate, and the values they give are wave-uniform.
typedef const __attribute__((address_space(4))) DevImage* ConstImage;
typedef const __attribute__((address_space(4))) int32_t* ConstInt;
typedef const __attribute__((address_space(4))) MsImage* ConstMsImage;

// Image pointers always address global memory; saying so gives global_load /
// global_store instead of flat accesses.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}

// Position of coefficient (i, j) in the zig-zag scan of an n x n block
// (§4.1): anti-diagonals t = i + j in order; odd t runs with the row rising,
// even t with the row falling.
__host__ __device__ constexpr int zz_rank(int n, int i, int j) {
  const int t = i + j;
  const int before = t < n ? t * (t + 1) / 2 : n * n - (2 * n - 1 - t) * (2 * n - t) / 2;
  const int ilo = t < n ? 0 : t - (n - 1);
  const int ihi = t < n ? t : n - 1;
  return before + ((t & 1) ? i - ilo : ihi - i);
}

// Appendix A quantiser: code c = round(B / Q~), Q~ = Q / (s s^T), with
// t = fl32(B * fl32(1 / Q~)) and round = floor(t + 1/2), evaluated exactly as
// floor(t) + [t - floor(t) >= 1/2]; returns the dequantised coefficient of
// T_hat A T_hat^T, Q c.  Contraction is off so that t is rounded once and
// the decision is taken on that FP32 value, not on an FMA's exact product.
// B is an integer held exactly in FP32 (|B| < 2^24).
__device__ __forceinline__ float quantise(float B, float qinv, float qstep) {
#pragma clang fp contract(off)
  const float t = B * qinv;
  const float f = floorf(t);
  const float c = f + (t - f >= 0.5f ? 1.0f : 0.0f);
  return c * qstep;
}
__device__ __forceinline__ float quantise(int B, float qinv, float qstep) {
  return quantise(static_cast<float>(B), qinv, qstep);
}

__device__ __forceinline__ int dot2(int a, int b, int acc) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, a), __builtin_bit_cast(short2v, b), acc,
                                false);
}

// Static schedule of a persistent grid: workgroup w takes the contiguous run
// of tiles [w T / G, (w + 1) T / G).  Consecutive tiles of a workgroup then
// mostly belong to one image, so per-image state (transform tables staged in
// LDS, operands in registers) is rarely reloaded.
__device__ __forceinline__ int tile_begin(int total) {
  return static_cast<int>(static_cast<long long>(total) * blockIdx.x / gridDim.x);
}
__device__ __forceinline__ int tile_end_of(int total) {
  return static_cast<int>(static_cast<long long>(total) * (blockIdx.x + 1) / gridDim.x);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Add the squared error of `tiles` finished tiles to an image and finalise
// the image when its last tiles are in.  Called by one thread.
//
// res->acc packs the tile count above bit 48 and the running SSE below it
// (SSE < 2^31 pixels * 255^2 < 2^48; the host keeps an image's tiles below
// 2^16).  One relaxed atomic add returns the previous value, so the caller
// that brings the count to ntiles holds the whole sum in its own result: no
// fence and no second read are needed, and no L2 write-back is forced while
// other workgroups still stream pixels through it.
__device__ void finish_tiles(rklt_result* res, unsigned long long sum, int tiles, int ntiles, long long npix) {
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(&res->acc);
  const unsigned long long mine = sum + (static_cast<unsigned long long>(tiles) << 48);
  const unsigned long long now = atomicAdd(acc, mine) + mine;
  if ((now >> 48) == static_cast<unsigned long long>(ntiles)) {
    const unsigned long long sse = now & ((1ull << 48) - 1);
    atomicExch(acc, 0ull);
    const float mse = static_cast<float>(sse) / static_cast<float>(npix);
    res->sse = sse;
    res->mse = mse;
    res->psnr_db = sse == 0 ? INFINITY : 10.0f * log10f(65025.0f / mse);
    res->tiles = static_cast<uint32_t>(ntiles);
  }
}

// Workgroup-wide sum of a per-thread value, then finish_tiles.
__device__ __forceinline__ void reduce_and_finish(unsigned long long mine, unsigned long long* red,
                                                  rklt_result* res, int tiles, int ntiles, long long npix) {
  const unsigned long long w = wave_sum(mine);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) t += red[k];
    finish_tiles(res, t, tiles, ntiles, npix);
  }
  __syncthreads();
}

}  // namespace
}  // namespace rklt
