// Panel kernel of the codec for every block length N in {4, 8, 16, 32} and
// any level shift (§4.1, Appendix A): the path for the images the N = 8
// matrix-core and register kernels do not take.  The computation is the
// separable one, B = T (A - ell) T^T in exact integers, B_hat = (s s^T) (.) B
// on the first r zig-zag positions, A' = T_hat^-1 B_hat T_hat^-T + ell in
// FP32, pixel = clip(floor(A' + 1/2)).  The same kernel codes with the
// paper's float comparison transforms (exact KLT, DCT; §4.1 and Table 3):
// B = M (A - ell) M^T in FP32, no scaling, A' = M^-1 B M^-T + ell.  A
// quantised transform entry (Appendix A) replaces the scaling of each kept
// coefficient by the quantiser: code round(B / Q~), dequantised Q * code.
//
// A wave codes one panel at a time: the PB blocks of one block row that
// cover 128 pixel columns (64 for N = 32), i.e. 64 RPL (block, row) pairs,
// RPL per lane (2, or 1 for N = 32).  Lane (block b, row m) loads row m of block b
// (consecutive lanes read consecutive bytes of an image row), computes the
// row transform of that row, and at the end reconstructs, stores and scores
// the same row, so the squared error needs no exchange.  The column stages
// run on (block b, column j) pairs through a per-wave LDS buffer; no
// workgroup barrier is needed inside a tile.  Block rows are padded to whole
// panels; lanes in the padding get out-of-range buffer offsets (zero loads,
// dropped stores).
//
// Only the D anti-diagonals i + j < D that hold kept coefficients are
// computed (D from r), so truncation removes work: the row stage produces
// columns j < min(N, D), the column stage rows i < D - j, and both inverse
// stages run over the kept coefficients only.  With a coefficient dump every
// coefficient is computed.
//
// Arithmetic: pixel - ell is taken as (pixel xor 0x80) + (128 - ell), so the
// row stage is a signed int8 dot product (v_dot4) plus (128 - ell) sigma_j
// (sigma_j = sum_n T[j][n]); entries of T beyond int8 take int32 products.
// The host's check 255 L1^2 < 2^31 (L1 the largest row sum of |T|) keeps
// |T| < 2^15, the row sums Y within 24 bits (24-bit multiplies in the column
// stage) and B within int32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.h"
#include "rklt_internal.h"

namespace rklt {
namespace {

constexpr uint32_t kPanelOutOfRange = 0x80000000u;
constexpr int kPanelBufferFlags = 0x00020000;

template <int N>
struct Panel {
  static constexpr int NN = N * N;
  static constexpr int PW = N == 32 ? 64 : 128;  // panel width in pixels
  static constexpr int PB = PW / N;              // blocks per panel
  static constexpr int RPL = PW / 64;            // (block, row) pairs per lane
  static constexpr int W4 = N / 4;               // 32-bit words per block row
  static constexpr int SP = N + 1;               // padded row stride of the per-wave buffer (bank spread)
  static constexpr int BUF = PB * N * SP;        // words per wave
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Row m of block b: N bytes as W4 words, through a raw buffer (out-of-range
// offsets read zero).
template <int N>
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t (&w)[N / 4]) {
  if constexpr (N == 4) {
    w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
  } else if constexpr (N == 8) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    w[0] = v.x;
    w[1] = v.y;
  } else {
#pragma unroll
    for (int h = 0; h < N / 16; ++h) {
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * h, 0, 0);
      w[4 * h + 0] = v.x;
      w[4 * h + 1] = v.y;
      w[4 * h + 2] = v.z;
      w[4 * h + 3] = v.w;
    }
  }
}

template <int N>
__device__ __forceinline__ void store_row(__amdgpu_buffer_rsrc_t rd, uint32_t off, const uint32_t (&w)[N / 4]) {
  if constexpr (N == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(w[0], rd, off, 0, 0);
  } else if constexpr (N == 8) {
    u32x2 v;
    v.x = w[0];
    v.y = w[1];
    __builtin_amdgcn_raw_buffer_store_b64(v, rd, off, 0, 0);
  } else {
#pragma unroll
    for (int h = 0; h < N / 16; ++h) {
      u32x4 v;
      v.x = w[4 * h + 0];
      v.y = w[4 * h + 1];
      v.z = w[4 * h + 2];
      v.w = w[4 * h + 3];
      __builtin_amdgcn_raw_buffer_store_b128(v, rd, off + 16u * h, 0, 0);
    }
  }
}

// Keep the compiler from moving LDS accesses of one stage across another:
// lanes read what other lanes of the same wave wrote, which the compiler
// cannot see.  LDS operations of one wave complete in order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// MODE (PanelMode): integer T within int8 (v_dot4), integer T beyond int8
// (int32 row products), or a float transform (FP32 forward from Mf).
template <int N, bool PLAN, int MODE>
__global__ __launch_bounds__(256) void rklt_panel_kernel(KArgs a) {
  constexpr bool BIGT = MODE == kPanelBigT, FLT = MODE == kPanelFloat;
  using P = Panel<N>;
  constexpr int NN = P::NN, PB = P::PB, RPL = P::RPL, W4 = P::W4, SP = P::SP;
  // per-lane table reads go through LDS; wave-uniform ones (rows of T and
  // T_hat^-1) are scalar loads from the transform table
  __shared__ float sW[NN];           // s_i s_j
  __shared__ float sQi[NN], sQs[NN];  // quantiser: 1 / Q~ and Q (quantised entries only)
  __shared__ int16_t srank[NN];      // zig-zag rank of (i, j)
  // per wave: row sums Y[b][m][j], then W (in place), at ((m PB + b) SP + j)
  __shared__ float sbuf[4][P::BUF];
  __shared__ unsigned long long red[4];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  float* const buf = sbuf[wave];
  int loaded = -1;
  const ConstInt tile_img = (ConstInt)(a.tile_img);
  for (int tile = tile_begin(a.total_tiles); tile < tile_end_of(a.total_tiles); ++tile) {
    const int ii = PLAN ? __builtin_amdgcn_readfirstlane(tile_img[tile]) : 0;
    const ConstImage im = PLAN ? (ConstImage)(a.imgs + ii) : (ConstImage)(&a.one);
    const int tid = __builtin_amdgcn_readfirstlane(im->tid);
    const ConstTransform tf = as_constant(a.tf + tid);
    if (tid != loaded) {
      __syncthreads();
      for (int k = threadIdx.x; k < NN; k += blockDim.x) {
        sW[k] = tf->w[k];
        sQi[k] = tf->qinv[k];
        sQs[k] = tf->qstep[k];
        srank[k] = static_cast<int16_t>(tf->rank[k]);
      }
      __syncthreads();
      loaded = tid;
    }
    const int r = __builtin_amdgcn_readfirstlane(im->r);
    const int ell = __builtin_amdgcn_readfirstlane(im->ell);
    const bool quant = !FLT && tf->quant != 0;
    const int D = a.dump ? 2 * N - 1 : __builtin_amdgcn_readfirstlane(im->D);
    const int Dc = D < N ? D : N;  // columns j that hold a needed coefficient
    const int bw = __builtin_amdgcn_readfirstlane(im->bw), bwp = __builtin_amdgcn_readfirstlane(im->bwp);
    const int ps = __builtin_amdgcn_readfirstlane(im->ps), pd = __builtin_amdgcn_readfirstlane(im->pd);
    const int H = __builtin_amdgcn_readfirstlane(im->H), W = __builtin_amdgcn_readfirstlane(im->W);
    uint8_t* const dst = im->dst;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(im->src), 0, (H - 1) * ps + W, kPanelBufferFlags);
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(dst, 0, dst ? (H - 1) * pd + W : 0, kPanelBufferFlags);
    const int tile_blocks = im->tile_blocks;
    const int b0 = (tile - im->tile0) * tile_blocks;
    const int nblocks = im->nblocks;  // padded: (H / N) * bwp
    const int b1 = b0 + tile_blocks < nblocks ? b0 + tile_blocks : nblocks;
    const float shift = static_cast<float>(ell) + 0.5f;
    const int lift = 128 - ell;
    uint32_t sxx = 0, sxy = 0;
    // row offsets of this lane's rows in panel pb (out of range past the
    // tile or in the row padding)
    auto offsets = [&](int pb, uint32_t (&os)[RPL], uint32_t (&od)[RPL], bool (&ok)[RPL]) {
      const int by = pb / bwp, bx0 = pb - by * bwp;
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int p = lane + 64 * k, b = p % PB, m = p / PB;
        ok[k] = pb < b1 && bx0 + b < bw;
        const uint32_t row = static_cast<uint32_t>(by * N + m), col = static_cast<uint32_t>(bx0 + b) * N;
        os[k] = ok[k] ? row * ps + col : kPanelOutOfRange;
        od[k] = ok[k] ? row * pd + col : kPanelOutOfRange;
      }
    };
    // the next panel's rows are loaded while the current one is coded; the
    // loads are issued on every pass (out of range past the tile), so every
    // pass has the same memory operations and the waits stay exact
    uint32_t nx[RPL][W4], nos[RPL], nod[RPL];
    bool nok[RPL];
    offsets(b0 + wave * PB, nos, nod, nok);
#pragma unroll
    for (int k = 0; k < RPL; ++k) load_row<N>(rs, nos[k], nx[k]);
    for (int pb = b0 + wave * PB; pb < b1; pb += 4 * PB) {
      const int by = pb / bwp, bx0 = pb - by * bwp;
      uint32_t px[RPL][W4], offd[RPL];
      bool valid[RPL];
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        offd[k] = nod[k];
        valid[k] = nok[k];
#pragma unroll
        for (int w = 0; w < W4; ++w) px[k][w] = nx[k][w];
      }
      offsets(pb + 4 * PB, nos, nod, nok);
#pragma unroll
      for (int k = 0; k < RPL; ++k) load_row<N>(rs, nos[k], nx[k]);
      // ---- row stage: lane owns the rows p = lane + 64 k
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int p = lane + 64 * k;
        if constexpr (FLT) {
          // pixel - ell exactly in FP32, then y_j = sum_n M[j][n] x_n
          float xf[N];
#pragma unroll
          for (int n = 0; n < N; ++n)
            xf[n] = static_cast<float>((px[k][n / 4] >> (8 * (n % 4))) & 0xffu) - static_cast<float>(ell);
          for (int j = 0; j < Dc; ++j) {
            float y = 0.0f;
#pragma unroll
            for (int n = 0; n < N; ++n) y = fmaf(tf->Mf[j * N + n], xf[n], y);
            buf[p * SP + j] = y;
          }
        } else {
          uint32_t xs[W4];
#pragma unroll
          for (int w = 0; w < W4; ++w) xs[w] = px[k][w] ^ 0x80808080u;
          for (int j = 0; j < Dc; ++j) {
            int y = lift * tf->sig[j];
            if (!BIGT) {
#pragma unroll
              for (int w = 0; w < W4; ++w) y = __builtin_amdgcn_sdot4(static_cast<int>(xs[w]), tf->Tw[j * W4 + w], y, false);
            } else {
#pragma unroll
              for (int n = 0; n < N; ++n) {
                const int x = __builtin_amdgcn_sbfe(static_cast<int>(xs[n / 4]), 8 * (n % 4), 8);
                y = x * __builtin_amdgcn_sbfe(tf->T[j * N + n], 0, 24) + y;
              }
            }
            buf[p * SP + j] = __builtin_bit_cast(float, y);
          }
        }
      }
      wave_lds_sync();
      // ---- column stage and first inverse stage: lane owns the columns q = lane + 64 k
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int q = lane + 64 * k, b = q / N, j = q % N;
        if (j < Dc) {
          // column j of the row sums: int24 (integer T) or FP32 (float transform)
          int Yc[N];
          float Yf[N];
#pragma unroll
          for (int m = 0; m < N; ++m) {
            const float v = buf[(m * PB + b) * SP + j];
            Yf[m] = v;
            Yc[m] = __builtin_amdgcn_sbfe(__builtin_bit_cast(int, v), 0, 24);
          }
          float Wc[N];
#pragma unroll
          for (int m = 0; m < N; ++m) Wc[m] = 0.0f;
          const int iend = D - j < N ? D - j : N;
          const bool vb = bx0 + b < bw;
          const int gb = by * bw + bx0 + b;  // block index in the image (dump layout)
          for (int i = 0; i < iend; ++i) {
            float bs;
            if constexpr (FLT) {
              // B_ij = sum_m M[i][m] Y[m][j]; no scaling
              float B = 0.0f;
#pragma unroll
              for (int m = 0; m < N; ++m) B = fmaf(tf->Mf[i * N + m], Yf[m], B);
              bs = B;
              if (a.dump && vb && im->scaled) im->scaled[static_cast<size_t>(gb) * NN + i * N + j] = bs;
            } else {
              int B = 0;
#pragma unroll
              for (int m = 0; m < N; ++m) B = __builtin_amdgcn_sbfe(tf->T[i * N + m], 0, 24) * Yc[m] + B;
              if (quant) {
                bs = quantise(B, sQi[i * N + j], sQs[i * N + j]);
              } else {
                bs = static_cast<float>(B) * sW[i * N + j];
              }
              if (a.dump && vb) {
                if (im->coef) im->coef[static_cast<size_t>(gb) * NN + i * N + j] = B;
                if (im->scaled) im->scaled[static_cast<size_t>(gb) * NN + i * N + j] = bs;
              }
            }
            if (srank[i * N + j] < r) {
#pragma unroll
              for (int m = 0; m < N; ++m) Wc[m] = fmaf(tf->Gt[i * N + m], bs, Wc[m]);
            }
          }
#pragma unroll
          for (int m = 0; m < N; ++m) buf[(m * PB + b) * SP + j] = Wc[m];
        }
      }
      wave_lds_sync();
      // ---- second inverse stage, reconstruction, store and squared error
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int p = lane + 64 * k;
        float acc[N];
#pragma unroll
        for (int n = 0; n < N; ++n) acc[n] = shift;
        for (int j = 0; j < Dc; ++j) {
          const float wj = buf[p * SP + j];
#pragma unroll
          for (int n = 0; n < N; ++n) acc[n] = fmaf(wj, tf->Gt[j * N + n], acc[n]);
        }
        uint32_t out[W4];
#pragma unroll
        for (int w = 0; w < W4; ++w) {
          uint32_t word = 0;
#pragma unroll
          for (int e = 0; e < 4; ++e) word = __builtin_amdgcn_cvt_pk_u8_f32(floorf(acc[4 * w + e]), e, word);
          out[w] = word;
        }
        store_row<N>(rd, offd[k], out);
        if (valid[k]) {
#pragma unroll
          for (int w = 0; w < W4; ++w) {
            sxx = __builtin_amdgcn_udot4(px[k][w], px[k][w], sxx, false);
            sxx = __builtin_amdgcn_udot4(out[w], out[w], sxx, false);
            sxy = __builtin_amdgcn_udot4(px[k][w], out[w], sxy, false);
          }
        }
      }
      wave_lds_sync();
    }
    reduce_and_finish(static_cast<unsigned long long>(sxx - 2u * sxy), red, a.res + im->slot, 1, im->ntiles,
                      static_cast<long long>(H) * W);
  }
}

rklt_status launched_panel() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RKLT_E_HIP, "rklt_panel_kernel: launch failed: %s", hipGetErrorString(e));
  return RKLT_OK;
}

template <int N, int MODE>
void launch_panel_m(const KArgs& a, int grid, hipStream_t st) {
  if (a.imgs) hipLaunchKernelGGL((rklt_panel_kernel<N, true, MODE>), dim3(grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL((rklt_panel_kernel<N, false, MODE>), dim3(grid), dim3(256), 0, st, a);
}

template <int N>
void launch_panel_n(const KArgs& a, int grid, int mode, hipStream_t st) {
  if (mode == kPanelFloat) launch_panel_m<N, kPanelFloat>(a, grid, st);
  else if (mode == kPanelBigT) launch_panel_m<N, kPanelBigT>(a, grid, st);
  else launch_panel_m<N, kPanelInt8>(a, grid, st);
}

}  // namespace

int panel_blocks(int N) {
  switch (N) {
    case 4: return Panel<4>::PB;
    case 8: return Panel<8>::PB;
    case 16: return Panel<16>::PB;
    case 32: return Panel<32>::PB;
    default: return 0;
  }
}

rklt_status launch_panel(int N, const KArgs& a, int grid, int mode, void* stream) {
  const hipStream_t st = static_cast<hipStream_t>(stream);
  switch (N) {
    case 4: launch_panel_n<4>(a, grid, mode, st); break;
    case 8: launch_panel_n<8>(a, grid, mode, st); break;
    case 16: launch_panel_n<16>(a, grid, mode, st); break;
    case 32: launch_panel_n<32>(a, grid, mode, st); break;
    default: return fail(RKLT_E_INVAL, "panel kernel: N=%d not supported", N);
  }
  return launched_panel();
}

}  // namespace rklt
