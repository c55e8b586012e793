// Region matrix-core kernel of the codec (§4.1, Appendix A) for block
// lengths N in {4, 8, 16, 32} and any level shift ell, for T with |T_ij| <=
// 127 and 128 L1 + |128 - ell| max|sig| <= 32640 (L1 the largest row sum of
// |T|, sig_j the row sums of T), for quantised entries of such T, and for
// the float comparison transforms (MODE below).  A wave codes one 32 x 32
// pixel region per step: (32 / N)^2 blocks through the block-diagonal Tb (T
// on the diagonal; the off-diagonal products are zero, so the blocks stay
// independent).  Every stage is a 32 x 32 x 32 product:
//   row stage      Y  = (A - 128) Tb^T + (128 - ell) sig   v_mfma_i32_32x32x32_i8
//                  (the row sums of A - ell, from signed pixel bytes)
//   column stage   B^T = Y^T Tb^T             four v_mfma_f32_32x32x16_f16
//                  (Y as two exact fp16 parts: |Y| < 2^15, so hi keeps 11
//                  bits and lo < 16; Tb exact in fp16; every partial sum an
//                  integer below 2^24, so B is exact in FP32)
//   zonal + S      B_hat = (s_i s_j) B on the first r zig-zag positions, FP32
//                  (quantised entries: B_hat = Q c, c = round(B / Q~) as in
//                  Appendix A, on the same positions)
//   inverse        Z = B_hat Gb^T, A'^T = Z^T Gb^T  v_mfma_f32_32x32x16_f16
//                  (Gb = T_hat^-1 on the block diagonal; each FP32 operand
//                  as two fp16 parts x = hi + lo, 22 bits, and the products
//                  hi hi + hi lo + lo hi accumulated in FP32)
//   pixel          clip(floor(A' + ell + 1/2)), squared error: one add and
//                  the saturating round-to-nearest byte conversion of
//                  A' + ell + 2^-12 (the nudge sends exact ties up; it
//                  differs from floor(x + 1/2) only within 2^-12 below a
//                  tie, inside the FP32 inverse's own tie band)
// so B = T (A - ell) T^T is exact and the inverse is FP32 up to the
// dropped lo lo terms (relative 2^-22).
//
// Layouts.  With h = lane / 32 and c = lane % 32, accumulator register t of
// lane l holds row kap(t, h) = 8 (t / 4) + 4 h + t % 4, column c; an int8
// operand lane holds row (A) or column (B) c and 16 K elements, an fp16
// operand lane 8 K elements.  The K order of a product only has to agree
// between its two operands, so every stage reads the previous stage's
// accumulator registers as they are: K element e of lane l is index
// kap(e, h) (for fp16 operands, chunk k of a product takes registers
// 8k .. 8k + 7), and the tables m32T, m32Gs, m32Ms of the transform record
// hold Tb (int8), Gb and Mb (for an integer T: Tb in fp16) in that order.  Lane l holds row c of the region at the
// pixel columns kap(0..15, h) (the words at columns 8q + 4h), and the last
// product returns exactly those pixels of the reconstruction to it, so the
// squared error needs no exchange.  Memory is accessed 16 contiguous bytes
// per lane (columns 16h .. 16h + 15): lanes l and l ^ 32 swap two words
// after the load and before the store, one v_permlane32_swap per two words
// (narrow accesses scattered over 32 rows cost more than the exchange).
//
// Truncation: register t of the inverse operands carries columns (then rows)
// kap(t, 0) and kap(t, 1); when both are >= D modulo N (D anti-diagonals
// hold every kept coefficient) its coefficients are zero, and a K chunk whose
// eight registers are all zero is skipped.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "rklt_internal.h"

namespace rklt {
namespace {

typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v16i32 __attribute__((ext_vector_type(16)));
typedef float v16f32 __attribute__((ext_vector_type(16)));
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));
typedef _Float16 v8f16 __attribute__((ext_vector_type(8)));
typedef _Float16 v2f16 __attribute__((ext_vector_type(2)));

// Eight FP32 values as two fp16 parts: hi = x rounded toward zero, lo = the
// remainder x - hi (exact inside a mixed-precision FMA) rounded to fp16;
// hi + lo carries 22 bits.  The trailing s_nop keeps two wait states between
// these VALU writes and a matrix instruction that reads them.
__device__ __forceinline__ void split_parts(const float* x, v8f16& hi, v8f16& lo) {
  v4u32 wh, wl;
#pragma unroll
  for (int p = 0; p < 4; ++p) wh[p] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x[2 * p], x[2 * p + 1]));
  uint32_t l0, l1, l2, l3;
  asm("v_fma_mixlo_f16 %0, %4, -1.0, %8 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %0, %4, -1.0, %9 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixlo_f16 %1, %5, -1.0, %10 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %1, %5, -1.0, %11 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixlo_f16 %2, %6, -1.0, %12 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %2, %6, -1.0, %13 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixlo_f16 %3, %7, -1.0, %14 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %3, %7, -1.0, %15 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
      "s_nop 1"
      : "=&v"(l0), "=&v"(l1), "=&v"(l2), "=&v"(l3)
      : "v"(wh[0]), "v"(wh[1]), "v"(wh[2]), "v"(wh[3]), "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]),
        "v"(x[5]), "v"(x[6]), "v"(x[7]));
  wl[0] = l0;
  wl[1] = l1;
  wl[2] = l2;
  wl[3] = l3;
  hi = __builtin_bit_cast(v8f16, wh);
  lo = __builtin_bit_cast(v8f16, wl);
}

// Waves per workgroup; they take consecutive regions.
constexpr int kM32Waves = 4;

constexpr uint32_t kRegionOut = 0x80000000u;  // out-of-range buffer offset: zero load, dropped store
constexpr int kRegionFlags = 0x00020000;

__host__ __device__ constexpr int kap(int t, int h) { return 8 * (t >> 2) + 4 * h + (t & 3); }

// Row c of region (ry, rx): lane h = l / 32 loads and stores the 16 bytes at
// columns 16h .. 16h + 15, as one 16-byte access when they all lie in the
// image, else word by word; the accumulator layout has the words at columns
// 8q + 4h .. + 3 (q = 0..3), which lanes l and l ^ 32 swap into place.
struct RegionRows {
  int row, col16;     // image row of this lane, first column of its 16 bytes
  uint32_t so, dof;   // byte offsets of (row, col16) in the source and destination
  bool row_ok;        // the row lies in the image (and the region in the tile)
  __device__ bool wide(int W) const { return row_ok && col16 + 16 <= W; }
  // byte offset of column col16 + d, out of range outside the image
  __device__ uint32_t src(int d, int W) const { return row_ok && col16 + d < W ? so + d : kRegionOut; }
  __device__ uint32_t dst(int d, int W) const { return row_ok && col16 + d < W ? dof + d : kRegionOut; }
  // word q of the accumulator layout (columns col16 - 16h + 8q + 4h ..) lies in the image
  __device__ bool ok(int q, int h, int W) const { return row_ok && col16 - 12 * h + 8 * q < W; }
  // every word of the region row lies in the image
  __device__ bool full(int h, int W) const { return row_ok && col16 - 16 * h + 32 <= W; }
};

// bs, bd: byte offsets of the start of image row 32 ry + c in the source and
// destination (kept up to date as the region row advances: no multiply per
// region)
__device__ __forceinline__ RegionRows region_rows(int ry, int rx, int H, int c, int h, bool in_tile, uint32_t bs,
                                                  uint32_t bd) {
  RegionRows rr;
  rr.row = ry * 32 + c;
  rr.col16 = rx * 32 + 16 * h;
  rr.so = bs + rr.col16;
  rr.dof = bd + rr.col16;
  rr.row_ok = in_tile && rr.row < H;
  return rr;
}

// The 16 bytes of a lane's row segment (W is a multiple of 4: each word is
// all in or all out of the image).
__device__ __forceinline__ void load_segment(__amdgpu_buffer_rsrc_t rs, const RegionRows& rr, int W,
                                             uint32_t (&w)[4]) {
  if (rr.wide(W)) {
    const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(rs, rr.src(0, W), 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = v[q];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = __builtin_amdgcn_raw_buffer_load_b32(rs, rr.src(4 * q, W), 0, 0);
  }
}

// MODE 0: rounded transforms; 1: entries with the Appendix A quantiser,
// which takes the place of the scaling of the kept coefficients; 2: float
// transforms (the comparison arms): the row and column stages run on fp16
// products of (pixel - ell), exact in fp16, and two-part M, with FP32 sums.
template <bool PLAN, int MODE>
__global__ __launch_bounds__(64 * kM32Waves) __attribute__((amdgpu_waves_per_eu(4))) void rklt_mfma32_kernel(KArgs a) {
  __shared__ unsigned long long red[kM32Waves];
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  int loaded = -1, loaded_r = -1;
  v4i32 Tw = {0, 0, 0, 0};
  int S = 0;  // sig of this lane's region column
  float WM[16];  // scale of each kept coefficient, 0 otherwise
  v8f16 Gh[2] = {}, Gl[2] = {}, Mh[2] = {}, Ml[2] = {};
  constexpr bool QUANT = MODE == 1, FLT = MODE == 2;
  // quantiser: 1 / Q~ of each kept coefficient (0 otherwise) and Q, per lane
  // in LDS (float4 k of lane l at [wave][k][l]: registers 4k .. 4k + 3, 1 / Q~
  // for k < 4, Q for k >= 4) rather than in 32 more VGPRs
  __shared__ float4 qtab[QUANT ? kM32Waves : 1][8][64];
#pragma unroll
  for (int t = 0; t < 16; ++t) WM[t] = 0.0f;
  const v16i32 zi = {};
  const v16f32 zf = {};
  const ConstInt tile_img = (ConstInt)(a.tile_img);
  for (int tile = tile_begin(a.total_tiles); tile < tile_end_of(a.total_tiles); ++tile) {
    const int ii = PLAN ? __builtin_amdgcn_readfirstlane(tile_img[tile]) : 0;
    const ConstImage im = PLAN ? (ConstImage)(a.imgs + ii) : (ConstImage)(&a.one);
    const int tid = __builtin_amdgcn_readfirstlane(im->tid);
    const int r = __builtin_amdgcn_readfirstlane(im->r);
    const DevTransform* tf = a.tf + tid;
    if (tid != loaded || r != loaded_r) {
      // per-lane operands of the transform; weights of ranks >= r zeroed
      Tw = v4i32{tf->m32T[lane][0], tf->m32T[lane][1], tf->m32T[lane][2], tf->m32T[lane][3]};
      S = tf->m32S[lane];
      if (QUANT) {
        const int Nt = tf->N;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float wq[4], qs[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int t = 4 * k + v;
            const int idx = (c % Nt) * Nt + kap(t, h) % Nt;
            wq[v] = tf->m32R[t][lane] < r ? tf->qinv[idx] : 0.0f;
            qs[v] = tf->qstep[idx];
          }
          qtab[wave][k][lane] = make_float4(wq[0], wq[1], wq[2], wq[3]);
          qtab[wave][4 + k][lane] = make_float4(qs[0], qs[1], qs[2], qs[3]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) WM[t] = tf->m32R[t][lane] < r ? tf->m32W[t][lane] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        Gh[k] = *reinterpret_cast<const v8f16*>(&tf->m32Gs[k][0][lane][0]);
        Gl[k] = *reinterpret_cast<const v8f16*>(&tf->m32Gs[k][1][lane][0]);
        Mh[k] = *reinterpret_cast<const v8f16*>(&tf->m32Ms[k][0][lane][0]);
        if (FLT) {
          Ml[k] = *reinterpret_cast<const v8f16*>(&tf->m32Ms[k][1][lane][0]);
        }
      }
      loaded = tid;
      loaded_r = r;
    }
    const int N = __builtin_amdgcn_readfirstlane(as_constant(tf)->N);
    const int D = __builtin_amdgcn_readfirstlane(im->D);
    const int ell = __builtin_amdgcn_readfirstlane(im->ell);
    // row-sum correction of this lane's column (zero at ell = 128)
    const int lift = (128 - ell) * S;
    const float out_bias = static_cast<float>(ell) + 0x1p-12f;
    const _Float16 e1024 = static_cast<_Float16>(1024 + ell);  // exact
    const v2f16 ell1024 = {e1024, e1024};
    uint32_t keep = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (kap(t, 0) % N < D || kap(t, 1) % N < D) keep |= 1u << t;
    keep = __builtin_amdgcn_readfirstlane(keep);
    const int H = __builtin_amdgcn_readfirstlane(im->H), W = __builtin_amdgcn_readfirstlane(im->W);
    const int ps = __builtin_amdgcn_readfirstlane(im->ps), pd = __builtin_amdgcn_readfirstlane(im->pd);
    const int rw = __builtin_amdgcn_readfirstlane(im->bw);
    uint8_t* const dst = im->dst;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(im->src), 0, (H - 1) * ps + W, kRegionFlags);
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(dst, 0, dst ? (H - 1) * pd + W : 0, kRegionFlags);
    const int tb = im->tile_blocks, nreg = im->nblocks;
    const int g0 = (tile - im->tile0) * tb;
    const int g1 = g0 + tb < nreg ? g0 + tb : nreg;
    uint32_t sxx = 0, sxy = 0;
    // the next region's pixels are loaded while the current one is coded
    // region (ny, nxr) of index g0 + wave, then advanced by the wave stride
    // without a division per region
    int ny = (g0 + wave) / rw, nxr = (g0 + wave) - ((g0 + wave) / rw) * rw;
    uint32_t bs = static_cast<uint32_t>(ny * 32 + c) * static_cast<uint32_t>(ps);
    uint32_t bd = static_cast<uint32_t>(ny * 32 + c) * static_cast<uint32_t>(pd);
    auto advance = [&]() {
      nxr += kM32Waves;
      while (nxr >= rw) {
        nxr -= rw;
        ++ny;
        bs += 32u * static_cast<uint32_t>(ps);
        bd += 32u * static_cast<uint32_t>(pd);
      }
    };
    RegionRows nrr = region_rows(ny, nxr, H, c, h, g0 + wave < g1, bs, bd);
    uint32_t nx[4];
    load_segment(rs, nrr, W, nx);
    for (int g = g0 + wave; g < g1; g += kM32Waves) {
      const RegionRows cur = nrr;
      // this lane's words in the accumulator layout: h = 0 keeps columns
      // 0-3 and 8-11 and takes 16-19 and 24-27 from its partner; h = 1 takes
      // 4-7 and 12-15 and keeps 20-23 and 28-31 (v_permlane32_swap trades
      // lanes 32-63 of its first operand for lanes 0-31 of its second)
      uint32_t x[4];
      {
        const v2u32 s01 = __builtin_amdgcn_permlane32_swap(nx[0], nx[1], false, false);
        const v2u32 s23 = __builtin_amdgcn_permlane32_swap(nx[2], nx[3], false, false);
        x[0] = s01[0];
        x[1] = s23[0];
        x[2] = s01[1];
        x[3] = s23[1];
      }
      advance();
      nrr = region_rows(ny, nxr, H, c, h, g + kM32Waves < g1, bs, bd);
      load_segment(rs, nrr, W, nx);
      float Bs[16];
      if constexpr (FLT) {
        // row stage: K chunk k of lane l is pixel words x[2k], x[2k + 1]
        // (columns kap(8k .. 8k + 7, h)), as fp16 pixel - ell: a byte b
        // under the high byte 0x64 is the fp16 1024 + b, and one packed fp16
        // subtraction of 1024 + ell gives b - ell exactly, two pixels at once
        v16f32 Yf = zf;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          v4u32 w;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const uint32_t xw = x[2 * k + p / 2];
            // [byte 2(p % 2), 0x64, byte 2(p % 2) + 1, 0x64]
            const uint32_t b1024 = __builtin_amdgcn_perm(0x64646464u, xw, p % 2 ? 0x04030402u : 0x04010400u);
            w[p] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(v2f16, b1024) - ell1024);
          }
          const v8f16 A = __builtin_bit_cast(v8f16, w);
          Yf = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, Mh[k], Yf, 0, 0, 0);
          Yf = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, Ml[k], Yf, 0, 0, 0);
        }
        // column stage on two fp16 parts of Y
        float Yr[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) Yr[t] = Yf[t];
        v16f32 Bf = zf;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          v8f16 ah, al;
          split_parts(&Yr[8 * k], ah, al);
          Bf = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Mh[k], Bf, 0, 0, 0);
          Bf = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Ml[k], Bf, 0, 0, 0);
          Bf = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, Mh[k], Bf, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) Bs[t] = Bf[t] * WM[t];
      } else {
        // row stage on pixel - 128 (xor 0x80 makes the bytes signed)
        const v4i32 X = {static_cast<int>(x[0] ^ 0x80808080u), static_cast<int>(x[1] ^ 0x80808080u),
                         static_cast<int>(x[2] ^ 0x80808080u), static_cast<int>(x[3] ^ 0x80808080u)};
        v16i32 Y = __builtin_amdgcn_mfma_i32_32x32x32_i8(X, Tw, zi, 0, 0, 0);
        // column stage on the two fp16 parts of Y (|Y| < 2^15: hi keeps 11
        // bits, lo < 16 is exact) against Tb in fp16: every product and
        // partial sum is an integer below 2^24, so B comes out exact in FP32
        if (ell != 128) {
#pragma unroll
          for (int t = 0; t < 16; ++t) Y[t] += lift;
        }
        float Yr[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) Yr[t] = static_cast<float>(Y[t]);
        v16f32 Bf = zf;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          v8f16 ah, al;
          split_parts(&Yr[8 * k], ah, al);
          Bf = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Mh[k], Bf, 0, 0, 0);
          Bf = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, Mh[k], Bf, 0, 0, 0);
        }
        // register t: B[c][kap(t, h)], scaled and masked
        if constexpr (QUANT) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float4 wq = qtab[wave][k][lane], qs = qtab[wave][4 + k][lane];
            Bs[4 * k + 0] = quantise(Bf[4 * k + 0], wq.x, qs.x);
            Bs[4 * k + 1] = quantise(Bf[4 * k + 1], wq.y, qs.y);
            Bs[4 * k + 2] = quantise(Bf[4 * k + 2], wq.z, qs.z);
            Bs[4 * k + 3] = quantise(Bf[4 * k + 3], wq.w, qs.w);
          }
        } else {
#pragma unroll
          for (int t = 0; t < 16; ++t) Bs[t] = Bf[t] * WM[t];
        }
      }
      // inverse: Z = B_hat Gb^T, then A'^T = Z^T Gb^T
      v16f32 Z = zf, O = zf;
      // K chunk k holds registers 8k .. 8k + 7 (skipped when all of them are)
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if ((keep >> (8 * k)) & 0xffu) {
          v8f16 ah, al;
          split_parts(&Bs[8 * k], ah, al);
          Z = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Gh[k], Z, 0, 0, 0);
          Z = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Gl[k], Z, 0, 0, 0);
          Z = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, Gh[k], Z, 0, 0, 0);
        }
      float Zr[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) Zr[t] = Z[t];
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if ((keep >> (8 * k)) & 0xffu) {
          v8f16 ah, al;
          split_parts(&Zr[8 * k], ah, al);
          O = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Gh[k], O, 0, 0, 0);
          O = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, Gl[k], O, 0, 0, 0);
          O = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, Gh[k], O, 0, 0, 0);
        }
      // register t of O: A'[c][kap(t, h)] - ell
      uint32_t o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t word = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          word = __builtin_amdgcn_cvt_pk_u8_f32(O[4 * q + v] + out_bias, v, word);
        o[q] = word;
      }
      // squared error over the words that lie in the image (all of them
      // inside the image: no per-word test)
      if (cur.full(h, W)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          sxx = __builtin_amdgcn_udot4(x[q], x[q], sxx, false);
          sxx = __builtin_amdgcn_udot4(o[q], o[q], sxx, false);
          sxy = __builtin_amdgcn_udot4(x[q], o[q], sxy, false);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (cur.ok(q, h, W)) {
            sxx = __builtin_amdgcn_udot4(x[q], x[q], sxx, false);
            sxx = __builtin_amdgcn_udot4(o[q], o[q], sxx, false);
            sxy = __builtin_amdgcn_udot4(x[q], o[q], sxy, false);
          }
      }
      // columns 16h .. 16h + 15 of row c: lane h = 0 holds 0-3 and 8-11 and
      // needs 4-7 and 12-15 from its partner (which holds them in its
      // words 0 and 1), lane h = 1 the converse with 16-19 and 24-27
      const v2u32 s02 = __builtin_amdgcn_permlane32_swap(o[0], o[2], false, false);
      const v2u32 s13 = __builtin_amdgcn_permlane32_swap(o[1], o[3], false, false);
      v4u32 w;
      w[0] = s02[0];
      w[1] = s02[1];
      w[2] = s13[0];
      w[3] = s13[1];
      if (cur.wide(W)) {
        __builtin_amdgcn_raw_buffer_store_b128(w, rd, cur.dst(0, W), 0, 0);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) __builtin_amdgcn_raw_buffer_store_b32(w[q], rd, cur.dst(4 * q, W), 0, 0);
      }
    }
    reduce_and_finish(static_cast<unsigned long long>(sxx - 2u * sxy), red, a.res + im->slot, 1, im->ntiles,
                      static_cast<long long>(H) * W);
  }
}

}  // namespace

int mfma32_resident_wgs_per_cu(int mode) {
  int n = 0;
  const hipError_t e =
      mode == 1   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rklt_mfma32_kernel<true, 1>, 64 * kM32Waves, 0)
      : mode == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rklt_mfma32_kernel<true, 2>, 64 * kM32Waves, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rklt_mfma32_kernel<true, 0>, 64 * kM32Waves, 0);
  return e == hipSuccess ? n : 0;
}

rklt_status launch_mfma32(const KArgs& a, int grid, int mode, void* stream) {
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 g(grid), b(64 * kM32Waves);
  if (a.imgs) {
    if (mode == 1) hipLaunchKernelGGL((rklt_mfma32_kernel<true, 1>), g, b, 0, st, a);
    else if (mode == 2) hipLaunchKernelGGL((rklt_mfma32_kernel<true, 2>), g, b, 0, st, a);
    else hipLaunchKernelGGL((rklt_mfma32_kernel<true, 0>), g, b, 0, st, a);
  } else {
    if (mode == 1) hipLaunchKernelGGL((rklt_mfma32_kernel<false, 1>), g, b, 0, st, a);
    else if (mode == 2) hipLaunchKernelGGL((rklt_mfma32_kernel<false, 2>), g, b, 0, st, a);
    else hipLaunchKernelGGL((rklt_mfma32_kernel<false, 0>), g, b, 0, st, a);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RKLT_E_HIP, "rklt_mfma32_kernel: launch failed: %s", hipGetErrorString(e));
  return RKLT_OK;
}

}  // namespace rklt
