// Matrix-core kernel of the N = 8 codec (level shift 128, int8-range T): the
// same computation as the register kernel, with both 2D transforms as
// products over the 64 pixels of a block:
//   forward   vec(B)   = (T (x) T) vec(A - 128)           v_mfma_i32_32x32x32_i8
//   inverse   vec(Out) = (adj (x) adj) vec(mask (.) B)    v_mfma_f32_32x32x16_f16
// where (x) is the Kronecker product (so B = T (A - 128) T^T, exact int32),
// T^-1 = adj / den and Out = den^2 (A' - 128) as in the register kernel.
//
// A wave codes 32 blocks per step: block = lane % 32.  The forward product
// takes 32 zig-zag ranks per instruction pair (two K-chunks of 32 pixels);
// rows of ranks >= r are zeroed in the operand, so truncation costs nothing
// and only ceil(r / 8) coefficient chunks enter the inverse.  The inverse of
// an image takes one of three forms, chosen on the host per (transform, r):
//   1  each coefficient enters as two exact fp16 halves B = hi + lo (hi = B
//      rounded toward zero, |lo| < 16); the weights are integers
//      |adj adj| <= 2048 and every partial sum stays below 2^24, so the FP32
//      accumulation is exact and Out is the exact integer;
//   3  hi = B rounded to a multiple of 64 and lo = B - hi go to separate
//      accumulators (the hi sums are multiples of 64 below 2^30, the lo sums
//      small), and their sum is exact because |Out| < 2^24 is certified;
//   2  no exact inverse fits: vec(A' - 128) in FP32 with
//      v_mfma_f32_32x32x2_f32, like the register kernel's fallback.
//
// Operand layouts (checked on gfx950 with a lane-layout probe): A lane l holds
// row l % 32 and K elements 16 (l / 32) + e (int8) or 8 (l / 32) + e (fp16);
// B lane l holds column l % 32 with the same K elements; accumulator register
// 4g + v of lane l holds row 8g + 4 (l / 32) + v, column l % 32.  With
// h = l / 32, lane l loads pixel rows 4c + 2h and 4c + 2h + 1 of its block for
// K-chunk c, and receives exactly those pixels back from pixel chunk mu = c,
// so reconstruction, store and squared error stay in the lane that loaded.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "rklt_internal.h"

namespace rklt {
namespace {

// Occupancy target (waves per SIMD the register allocation must allow) and
// depth of the pixel prefetch ring (steps in flight per wave, 2 or 3).  Four
// waves with two steps each in flight (128 VGPRs) beat three waves with
// three steps each by 3% back to back.
#ifndef RKLT_MFMA_WAVES_PER_EU
#define RKLT_MFMA_WAVES_PER_EU 4
#endif
#ifndef RKLT_MFMA_RING
#define RKLT_MFMA_RING 2
#endif
// Cache-policy bits of the pixel loads and reconstruction stores.  The
// reconstruction is written once and not read again by the kernel:
// non-temporal stores (bit 1) keep it from lingering dirty in L2, which
// otherwise costs a write-back at the end of every launch.
#ifndef RKLT_MFMA_LOAD_AUX
#define RKLT_MFMA_LOAD_AUX 0
#endif
#ifndef RKLT_MFMA_STORE_AUX
#define RKLT_MFMA_STORE_AUX 2
#endif

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Exact fp16 halves of four int32 coefficients (|B| < 32768): hi = B rounded
// toward zero to fp16, lo = B - hi (|lo| < 16, an exact fp16 integer).  The
// words are [hi0 hi1] [lo0 lo1] [hi2 hi3] [lo2 lo3]; lo comes from one
// mixed-precision FMA per coefficient, lo = fma(hi, -1, B) rounded to fp16.
__device__ __forceinline__ v8h split_fp16(int b0, int b1, int b2, int b3) {
  const float f0 = static_cast<float>(b0), f1 = static_cast<float>(b1);
  const float f2 = static_cast<float>(b2), f3 = static_cast<float>(b3);
  v4u w;
  w[0] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(f0, f1));
  w[2] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(f2, f3));
  uint32_t lo01, lo23;
  // the trailing s_nop keeps two wait states between these VALU writes and a
  // matrix instruction that reads them
  asm("v_fma_mixlo_f16 %0, %2, -1.0, %4 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %0, %2, -1.0, %5 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixlo_f16 %1, %3, -1.0, %6 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %1, %3, -1.0, %7 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
      "s_nop 1"
      : "=&v"(lo01), "=&v"(lo23)
      : "v"(w[0]), "v"(w[2]), "v"(f0), "v"(f1), "v"(f2), "v"(f3));
  w[1] = lo01;
  w[3] = lo23;
  return __builtin_bit_cast(v8h, w);
}

// Exact fp16 halves of four int32 coefficients for the two-accumulator
// inverse: hi = B rounded to a multiple of 64 (exact in fp16 for |B| < 65504),
// lo = B - hi in [-32, 31].  Bh holds the hi parts in the hi slots of the
// operand layout and zeros in the lo slots; Bl the reverse.
__device__ __forceinline__ void split_fp16_64(int b0, int b1, int b2, int b3, v8h& Bh, v8h& Bl) {
  const int h0 = (b0 + 32) & ~63, h1 = (b1 + 32) & ~63, h2 = (b2 + 32) & ~63, h3 = (b3 + 32) & ~63;
  v4u wh, wl;
  wh[0] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(static_cast<float>(h0), static_cast<float>(h1)));
  wh[2] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(static_cast<float>(h2), static_cast<float>(h3)));
  wl[1] = __builtin_bit_cast(uint32_t,
                             __builtin_amdgcn_cvt_pkrtz(static_cast<float>(b0 - h0), static_cast<float>(b1 - h1)));
  wl[3] = __builtin_bit_cast(uint32_t,
                             __builtin_amdgcn_cvt_pkrtz(static_cast<float>(b2 - h2), static_cast<float>(b3 - h3)));
  wh[1] = wh[3] = 0u;
  wl[0] = wl[2] = 0u;
  Bh = __builtin_bit_cast(v8h, wh);
  Bl = __builtin_bit_cast(v8h, wl);
}

// One step: 32 blocks of one image.  px[c][rr] are pixel rows 4c + 2h + rr
// (8 bytes each) of this lane's block; sF the forward operand (ranks >= r
// zeroed) and sV the inverse operand, both in LDS.  Writes the
// reconstruction rows through the buffer resource rd at lane offset od (rows
// 4 mu + rr at pitch pd) and accumulates the squared-error terms of valid
// blocks.  PATH is the inverse form (1 and 3 exact, 2 FP32).
template <int R8, int PATH>
__device__ __forceinline__ void mfma_step(const u32x2 (&px)[2][2], const v4i* sF, const void* sVraw, int lane,
                                          float inv, float bias, __amdgpu_buffer_rsrc_t rd, uint32_t od, int pd,
                                          bool valid, uint32_t& sxx, uint32_t& sxy) {
  v4i X[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    X[c][0] = static_cast<int>(px[c][0].x ^ 0x80808080u);
    X[c][1] = static_cast<int>(px[c][0].y ^ 0x80808080u);
    X[c][2] = static_cast<int>(px[c][1].x ^ 0x80808080u);
    X[c][3] = static_cast<int>(px[c][1].y ^ 0x80808080u);
  }
  v16i acc[2];
  auto forward = [&]() {
    const v16i zi = {};
    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(sF[(0 * 2 + 0) * 64 + lane], X[0], zi, 0, 0, 0);
    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(sF[(0 * 2 + 1) * 64 + lane], X[1], acc[0], 0, 0, 0);
    if (R8 > 4) {
      acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(sF[(1 * 2 + 0) * 64 + lane], X[0], zi, 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(sF[(1 * 2 + 1) * 64 + lane], X[1], acc[1], 0, 0, 0);
    }
  };
  if (PATH != 3) forward();
  // Reconstruction of pixel chunk mu: register 4g + v is pixel row
  // 4 mu + 2h + g / 2, column 4 (g % 2) + v of this lane's block.
  auto finish = [&](const v16f& o, int mu) {
    uint32_t w[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      uint32_t word = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) word = __builtin_amdgcn_cvt_pk_u8_f32(fmaf(o[4 * g + v], inv, bias), v, word);
      w[g] = word;
    }
    // unconditional stores: lanes without a block carry an out-of-range
    // offset and the buffer unit drops their writes
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      u32x2 ow;
      ow.x = w[2 * rr];
      ow.y = w[2 * rr + 1];
      __builtin_amdgcn_raw_buffer_store_b64(ow, rd, od, (4 * mu + rr) * pd, RKLT_MFMA_STORE_AUX);
    }
    if (valid) {
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        sxx = __builtin_amdgcn_udot4(px[mu][rr].x, px[mu][rr].x, sxx, false);
        sxx = __builtin_amdgcn_udot4(px[mu][rr].y, px[mu][rr].y, sxx, false);
        sxx = __builtin_amdgcn_udot4(w[2 * rr], w[2 * rr], sxx, false);
        sxx = __builtin_amdgcn_udot4(w[2 * rr + 1], w[2 * rr + 1], sxx, false);
        sxy = __builtin_amdgcn_udot4(px[mu][rr].x, w[2 * rr], sxy, false);
        sxy = __builtin_amdgcn_udot4(px[mu][rr].y, w[2 * rr + 1], sxy, false);
      }
    }
  };
  const v16f zf = {};
  if (PATH == 1) {
    // exact fp16 inverse: each coefficient as two exact halves B = hi + lo
    const v8h* sV = static_cast<const v8h*>(sVraw);
    v16f out[2] = {zf, zf};
#pragma unroll
    for (int kappa = 0; kappa < R8; ++kappa) {
      const int g = kappa & 3;
      const v16i& A = acc[kappa >> 2];
      const v8h Bop = split_fp16(A[4 * g], A[4 * g + 1], A[4 * g + 2], A[4 * g + 3]);
#pragma unroll
      for (int mu = 0; mu < 2; ++mu)
        out[mu] = __builtin_amdgcn_mfma_f32_32x32x16_f16(sV[(mu * 8 + kappa) * 64 + lane], Bop, out[mu], 0, 0, 0);
      // keep each chunk's operand reads next to its use (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    finish(out[0], 0);
    finish(out[1], 1);
  } else if (PATH == 3) {
    // exact fp16 inverse with the hi parts (multiples of 64) and the lo parts
    // summed in separate accumulators, one pixel chunk at a time; the forward
    // product is recomputed per chunk so that only two accumulators and the
    // coefficients are live at once (register pressure)
    const v8h* sV = static_cast<const v8h*>(sVraw);
#pragma unroll
    for (int mu = 0; mu < 2; ++mu) {
      forward();
      v16f oh = zf, ol = zf;
#pragma unroll
      for (int kappa = 0; kappa < R8; ++kappa) {
        const int g = kappa & 3;
        const v16i& A = acc[kappa >> 2];
        v8h Bh, Bl;
        split_fp16_64(A[4 * g], A[4 * g + 1], A[4 * g + 2], A[4 * g + 3], Bh, Bl);
        const v8h Wt = sV[(mu * 8 + kappa) * 64 + lane];
        oh = __builtin_amdgcn_mfma_f32_32x32x16_f16(Wt, Bh, oh, 0, 0, 0);
        ol = __builtin_amdgcn_mfma_f32_32x32x16_f16(Wt, Bl, ol, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      // one pixel chunk's accumulators live at a time (register pressure)
      __builtin_amdgcn_sched_barrier(0);
      finish(oh + ol, mu);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // FP32 inverse: one coefficient per lane and instruction (K = lane / 32)
    const float* sVf = static_cast<const float*>(sVraw);
    v16f out[2] = {zf, zf};
#pragma unroll
    for (int kappa = 0; kappa < R8; ++kappa) {
      const int g = kappa & 3;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float fb = static_cast<float>(acc[kappa >> 2][4 * g + v]);
#pragma unroll
        for (int mu = 0; mu < 2; ++mu)
          out[mu] = __builtin_amdgcn_mfma_f32_32x32x2f32(sVf[((mu * 8 + kappa) * 4 + v) * 64 + lane], fb, out[mu], 0, 0,
                                                         0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    finish(out[0], 0);
    finish(out[1], 1);
  }
}

// Pixels and reconstructions go through raw buffer resources: a lane whose
// block lies past the segment end gets this offset, which is beyond every
// image (the host keeps image spans below 2^31 bytes), so its loads return
// zero and its stores are dropped without a branch.  Every step then issues
// the same memory operations on every path, which keeps the wait counts of
// the prefetch ring exact.
constexpr uint32_t kOutOfRange = 0x80000000u;
constexpr int kRawBufferFlags = 0x00020000;

// Wave-uniform fields of the image a segment codes (held in SGPRs): bw
// blocks per row, bwp blocks per row of the block index space.
struct SegImage {
  __amdgpu_buffer_rsrc_t rs, rd;
  int ps, pd, bw, bwp;
};

// Block row and column of the first block of a wave's step, wave-uniform:
// a step covers 32 consecutive blocks in raster order and the next step of
// the same wave starts `stride` blocks later.
struct Cursor {
  int by, bx;
};

// Steps [base0, be) of one image segment, 32 blocks per step, strided by
// the workgroup's waves.  A ring of RKLT_MFMA_RING pixel buffers keeps the
// loads of the next steps in flight while a step is computed.  WIDE images
// (at least 32 blocks per row) have block rows padded to bwp, a multiple of
// 32, and steps start at multiples of 32, so a step's 32 blocks lie in one
// block row: a wave-uniform cursor (block row, first column) gives every
// lane's offset as the cursor's plus a lane constant, and lanes in the
// padding are out of range.  Narrower images divide per lane.
template <int R8, int PATH, bool WIDE>
__device__ __forceinline__ void segment(const SegImage& im, int base0, int be, int stride, const v4i* sF,
                                        const void* sV, int lane, int q, int h, float inv, float bias,
                                        uint32_t& sxx, uint32_t& sxy) {
  const int bw = im.bw, bwp = im.bwp, ps = im.ps, pd = im.pd;
  const uint32_t Ls = 8u * q + 2u * h * ps, Ld = 8u * q + 2u * h * pd;
  // lanes of step `base` (cursor c) that hold a block of the segment
  auto lanes = [&](const Cursor& c, int base) {
    const int n = be - base;
    return WIDE ? (n < bw - c.bx ? n : bw - c.bx) : n;
  };
  // byte offset of this lane's block of step `base` from the image start,
  // rows 2h and up; out of range for lanes without a block
  auto offset = [&](const Cursor& c, int base, int pitch, uint32_t L) -> uint32_t {
    uint32_t off;
    if (WIDE) {
      off = static_cast<uint32_t>(c.by * 8 * pitch + c.bx * 8) + L;
    } else {
      const int b = base + q;
      const int by = b / bw, bx = b - by * bw;
      off = static_cast<uint32_t>(by * 8 + 2 * h) * pitch + static_cast<uint32_t>(bx) * 8;
    }
    return q < lanes(c, base) ? off : kOutOfRange;
  };
  auto advance = [&](Cursor& c) {
    if (WIDE) {
      c.bx += stride;
      while (c.bx >= bwp) {
        c.bx -= bwp;
        ++c.by;
      }
    }
  };
  // pixel rows 4c + 2h + rr of this lane's block of step `base`
  auto load = [&](u32x2 (&px)[2][2], const Cursor& c, int base) {
    const uint32_t off = offset(c, base, ps, Ls);
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
      for (int rr = 0; rr < 2; ++rr)
        px[cc][rr] = __builtin_amdgcn_raw_buffer_load_b64(im.rs, off, (4 * cc + rr) * ps, RKLT_MFMA_LOAD_AUX);
  };
  Cursor cl{0, 0};
  if (WIDE) {
    cl.by = base0 / bwp;
    cl.bx = base0 - cl.by * bwp;
  }
  Cursor cs = cl;
#if RKLT_MFMA_RING == 3
  u32x2 p0[2][2], p1[2][2], p2[2][2];
  load(p0, cl, base0);
  advance(cl);
  load(p1, cl, base0 + stride);
  advance(cl);
  load(p2, cl, base0 + 2 * stride);
  advance(cl);
#else
  u32x2 p0[2][2], p1[2][2];
  load(p0, cl, base0);
  advance(cl);
  load(p1, cl, base0 + stride);
  advance(cl);
#endif
  auto run = [&](u32x2 (&px)[2][2], int base) {
    const bool valid = q < lanes(cs, base);
    const uint32_t od = offset(cs, base, pd, Ld);
    mfma_step<R8, PATH>(px, sF, sV, lane, inv, bias, im.rd, od, pd, valid, sxx, sxy);
    advance(cs);
    load(px, cl, base + RKLT_MFMA_RING * stride);
    advance(cl);
  };
  // Whole rounds of the ring, then the remaining steps.  No step exits the
  // loop early, so the memory operations between a load and its use are the
  // same on every path and the load's wait leaves the later loads in flight.
  const int nsteps = base0 < be ? (be - base0 + stride - 1) / stride : 0;
  int base = base0;
  for (int g = nsteps / RKLT_MFMA_RING; g > 0; --g) {
    run(p0, base);
    run(p1, base + stride);
#if RKLT_MFMA_RING == 3
    run(p2, base + 2 * stride);
#endif
    base += RKLT_MFMA_RING * stride;
  }
  const int rem = nsteps % RKLT_MFMA_RING;
  if (rem > 0) run(p0, base);
#if RKLT_MFMA_RING == 3
  if (rem > 1) run(p1, base + stride);
#endif
}

template <int R8, int PATH>
__device__ __forceinline__ void segment_any(const SegImage& im, int base0, int be, int stride, const v4i* sF,
                                            const void* sV, int lane, int q, int h, float inv, float bias,
                                            uint32_t& sxx, uint32_t& sxy) {
  if (im.bw >= 32) segment<R8, PATH, true>(im, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy);
  else segment<R8, PATH, false>(im, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy);
}

// PLAN: a batch plan's work list; otherwise the plain path's single image.
// The grid is sized to the resident capacity.  Workgroup w codes a
// contiguous tile range (the plan balances the ranges by estimated cost;
// otherwise [w T / G, (w + 1) T / G)) as segments of consecutive tiles of one
// image: per segment it sets up the image (forward operand with
// ranks >= r zeroed; the inverse operand staged in LDS when the transform
// changes), lets its waves stride over the segment's steps, and adds the
// segment's squared error and tile count to the image's accumulator.
template <bool PLAN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RKLT_MFMA_WAVES_PER_EU)))
void rklt_mfma8_kernel(KArgs a) {
  __shared__ unsigned long long red[4];
  __shared__ uint4 sV[2 * 8 * 64];  // inverse operand of the current transform (16 KB)
  __shared__ v4i sF[2 * 2 * 64];  // forward operand of the current (transform, r) (4 KB)
  const int lane = threadIdx.x & 63;
  // the wave index is wave-uniform; saying so keeps every per-step block
  // cursor in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int nwaves = static_cast<int>(blockDim.x >> 6);
  const int q = lane & 31, h = lane >> 5;
  const int stride = nwaves * 32;
  int loaded = -1, loaded_r = -1;
  const ConstInt wg_tiles = (ConstInt)(a.wg_tiles);
  const ConstInt tile_img = (ConstInt)(a.tile_img);
  // contiguous tile range of this workgroup (cost-balanced by the plan, or an
  // equal share of the tiles), or, for a round-robin plan, tiles blockIdx.x,
  // blockIdx.x + gridDim.x, ... each as a segment of its own (the whole grid
  // then sweeps the batch together; which schedule is faster depends on the
  // batch, and the autotuner tries both)
  const bool strided = PLAN && a.strided;
  const int t_end = strided              ? a.total_tiles
                    : PLAN && a.wg_tiles ? wg_tiles[blockIdx.x + 1]
                                         : tile_end_of(a.total_tiles);
  for (int t = strided                ? static_cast<int>(blockIdx.x)
               : PLAN && a.wg_tiles ? wg_tiles[blockIdx.x]
                                    : tile_begin(a.total_tiles);
       t < t_end;) {
    const int ii = PLAN ? __builtin_amdgcn_readfirstlane(tile_img[t]) : 0;
    const ConstImage im = PLAN ? (ConstImage)(a.imgs + ii) : (ConstImage)(&a.one);
    const int tile0 = im->tile0, ntiles = im->ntiles;
    const int seg_end = strided ? t + 1 : tile0 + ntiles < t_end ? tile0 + ntiles : t_end;
    const int tid = __builtin_amdgcn_readfirstlane(im->tid);
    const int r = __builtin_amdgcn_readfirstlane(im->r);
    const DevTransform* tf = a.tf + tid;
    const int path = __builtin_amdgcn_readfirstlane(mfma8_path(*tf, r));
    // the inverse operand in LDS: fp16 (forms 1 and 3) or FP32 (form 2)
    const int operand = 2 * tid + (path == 2);
    if (operand != loaded || r != loaded_r) {
      __syncthreads();
      if (operand != loaded) {
        // 16 KB either way
        const uint4* srcv = path != 2 ? reinterpret_cast<const uint4*>(&tf->mV[0][0][0][0])
                                      : reinterpret_cast<const uint4*>(&tf->mVf[0][0][0][0]);
        for (int k = threadIdx.x; k < 2 * 8 * 64; k += blockDim.x) sV[k] = srcv[k];
      }
      // forward operand: rows (zig-zag ranks) >= r zeroed
      for (int k = threadIdx.x; k < 2 * 2 * 64; k += blockDim.x) {
        const int mu = k >> 7, l = k & 63;
        const int4 f = *reinterpret_cast<const int4*>(&tf->mF[0][0][0][0] + 4 * k);
        const bool keep = 32 * mu + (l & 31) < r;
        sF[k] = keep ? v4i{f.x, f.y, f.z, f.w} : v4i{0, 0, 0, 0};
      }
      __syncthreads();
      loaded = operand;
      loaded_r = r;
    }
    const int R8 = (r + 7) >> 3;
    const float inv = tf->m_inv, bias = tf->m_bias;
    const int tb = im->tile_blocks, nblocks = im->nblocks;
    const int bs = (t - tile0) * tb;
    const int be = (seg_end - tile0) * tb < nblocks ? (seg_end - tile0) * tb : nblocks;
    SegImage si;
    si.ps = __builtin_amdgcn_readfirstlane(im->ps);
    si.pd = __builtin_amdgcn_readfirstlane(im->pd);
    si.bw = __builtin_amdgcn_readfirstlane(im->bw);
    si.bwp = __builtin_amdgcn_readfirstlane(im->bwp);
    {
      const int H = __builtin_amdgcn_readfirstlane(im->H), W = __builtin_amdgcn_readfirstlane(im->W);
      uint8_t* const dst = im->dst;
      si.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(im->src), 0, (H - 1) * si.ps + W,
                                                kRawBufferFlags);
      // no reconstruction wanted: an empty range drops every store
      si.rd = __builtin_amdgcn_make_buffer_rsrc(dst, 0, dst ? (H - 1) * si.pd + W : 0, kRawBufferFlags);
    }
    uint32_t sxx = 0, sxy = 0;
    const int base0 = bs + wave * 32;
#define RKLT_SEG(RR)                                                                                   \
  case RR:                                                                                             \
    if (path == 1) segment_any<RR, 1>(si, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy); \
    else if (path == 3) segment_any<RR, 3>(si, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy); \
    else segment_any<RR, 2>(si, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy);           \
    break;
    switch (R8) {
      RKLT_SEG(1) RKLT_SEG(2) RKLT_SEG(3) RKLT_SEG(4) RKLT_SEG(5) RKLT_SEG(6) RKLT_SEG(7)
      default:
        if (path == 1) segment_any<8, 1>(si, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy);
        else if (path == 3) segment_any<8, 3>(si, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy);
        else segment_any<8, 2>(si, base0, be, stride, sF, sV, lane, q, h, inv, bias, sxx, sxy);
        break;
    }
#undef RKLT_SEG
    reduce_and_finish(sxx - 2u * sxy, red, a.res + im->slot, seg_end - t, ntiles,
                      static_cast<long long>(im->H) * im->W);
    t = strided ? t + static_cast<int>(gridDim.x) : seg_end;
  }
}

rklt_status launched_mfma() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RKLT_E_HIP, "rklt_mfma8_kernel: launch failed: %s", hipGetErrorString(e));
  return RKLT_OK;
}

}  // namespace

int mfma8_resident_wgs_per_cu(int wg) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rklt_mfma8_kernel<true>, wg, 0) != hipSuccess) return 0;
  return n;
}

rklt_status launch_mfma8(const KArgs& a, int grid, int wg, void* stream) {
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.imgs) hipLaunchKernelGGL(rklt_mfma8_kernel<true>, dim3(grid), dim3(wg), 0, st, a);
  else hipLaunchKernelGGL(rklt_mfma8_kernel<false>, dim3(grid), dim3(wg), 0, st, a);
  return launched_mfma();
}

}  // namespace rklt
