// Internal declarations of librklt: error reporting, the device-side
// transform record and work-list entries shared by the host code and the
// kernels.  Not part of the public ABI.
#pragma once

#include <cstdint>

#include "rklt.h"

namespace rklt {

// Record `code` with a printf-style message in the thread-local error slot.
rklt_status fail(rklt_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

rklt_status build_transform(int N, double rho, double alpha, rklt_transform* out);
rklt_status zigzag(int N, int32_t* order);
rklt_status klt_matrix(int N, double rho, double* K);
rklt_status dct_matrix(int N, double* C);
rklt_status transform_measures(int N, const double* That, const double* ref, double rho, rklt_measures* out);
rklt_status algorithm1(int N, double alpha, double step, rklt_design_entry* out, int cap, int* count);
// FP64 Gauss-Jordan inverse with partial pivoting; false if singular.
bool invert_matrix(int n, const double* A, double* inv);
// Exact inverse of an integer matrix with entries in [-8, 8], N <= 8:
// T^-1 = adj / den in lowest terms, den > 0.  False if singular or out of range.
bool exact_inverse(int N, const int32_t* T, int64_t* adj, int64_t* den);

constexpr int kMaxTransforms = 256;

// Device copy of one transform (one entry of a context's table).  Everything
// the kernels read about T, in the layouts they read it in.
struct alignas(256) DevTransform {
  int32_t N, flags, max_abs, max_row_l1;
  int32_t sig[RKLT_MAX_N];       // sigma_i = sum_j T_ij (row sums)
  int32_t t8[8][2];              // N = 8: row j of T as int8x4 words, n = 0..3 | 4..7
  int32_t t16[8][4];             // N = 8: row i of T as int16x2 words, (m, m+1) pairs
  // N = 8 inverse constants.  The register kernel reconstructs
  //   pixel = RNE_sat(Out * inv_den2 + bias),  Out = fadj (mask (.) B) fadj^T.
  // exact = 1: T^-1 = adj / den with integer adj, fadj = adj, inv_den2 =
  //   1/den^2, bias = 128 + delta; every FMA is exact and the pixel equals
  //   floor(Out / den^2 + 1/2) + 128 exactly (bounds checked on the host).
  // exact = 0: fadj = T^-1 in FP32, inv_den2 = 1, bias = 128 + 2^-12 (an FP32
  //   reconstruction; exact ties go up as floor(x + 1/2) does).
  int32_t exact;
  int32_t den;
  float inv_den2, bias;
  int32_t adj[64];
  float fadj[64];                // m*8 + i
  // N = 8 matrix-core kernel (m_ok = 1 when its operands are built).  The
  // inverse of an image with r kept coefficients takes form
  //   1 when r <= m_r1: exact, one fp16 pass (mV);
  //   3 otherwise when m_path3: exact, fp16 with two accumulators (mV);
  //   2 otherwise: FP32 (mVf);
  // and the pixel is RNE_sat(Out * m_inv + m_bias) (exact forms: 1/den^2 and
  // 128 + delta; FP32 form without an exact inverse: 1 and 128 + 2^-12).
  // Operands, in the lane layout of the instructions:
  //   mF[mu][c][lane][w]   forward A operand of v_mfma_i32_32x32x32_i8, int8x4
  //                        words: row = zig-zag rank 32 mu + lane % 32, K =
  //                        pixel of K-chunk c; value T[i][m] T[j][n]
  //   mV[mu][kappa][lane]  inverse A operand of v_mfma_f32_32x32x16_f16, 8 halves:
  //                        row = pixel of chunk mu, K = (rank, hi/lo part) of
  //                        coefficient chunk kappa, halves ordered hi v0, hi v1,
  //                        lo v0, lo v1, hi v2, hi v3, lo v2, lo v3 for the
  //                        ranks 8 kappa + 4 (lane / 32) + v; value adj[m][i] adj[n][j]
  //   mVf[mu][kappa][v][lane] inverse A operand of v_mfma_f32_32x32x2_f32:
  //                        row = pixel, K = lane / 32 selects rank
  //                        8 kappa + 4 (lane / 32) + v; value adj (x) adj with
  //                        an exact inverse, else T^-1 (x) T^-1, in FP32
  int32_t m_ok, m_r1, m_path3, m_den;
  float m_inv, m_bias;
  // float transforms (rklt_ctx_add_float_transform): is_float = 1, the
  // forward matrix M in Mf, M^-1 transposed in Gt, w = 1; every integer
  // field is zero and the kernels for integer transforms never see them.
  // Quantised entries (rklt_ctx_add_quantizer): quant = 1, a copy of an
  // integer transform plus qinv and qstep below
  int32_t is_float, quant;
  int32_t mF[2][2][64][4];
  _Float16 mV[2][8][64][8];
  float mVf[2][8][4][64];
  float w[RKLT_MAX_N * RKLT_MAX_N];     // s_i s_j at i*N + j
  float G[RKLT_MAX_N * RKLT_MAX_N];     // T_hat^-1 at m*N + i
  float Mf[RKLT_MAX_N * RKLT_MAX_N];    // float transforms: M at i*N + n
  int32_t T[RKLT_MAX_N * RKLT_MAX_N];   // T at i*N + j
  int32_t rank[RKLT_MAX_N * RKLT_MAX_N];  // zig-zag position of (i, j)
  // panel kernel (read as wave-uniform scalars): rows of T as int8x4 words
  // (word j * N / 4 + w holds T[j][4w .. 4w + 3]; all zero when some
  // |T| > 127) and T_hat^-1 transposed (Gt[i * N + m] = G[m * N + i])
  int32_t Tw[RKLT_MAX_N * RKLT_MAX_N / 4];
  float Gt[RKLT_MAX_N * RKLT_MAX_N];
  // quantiser (quant = 1): qinv = fl32(s_i s_j / Q_ij), the reciprocal of
  // Q~ = Q / (s s^T); qstep = fl32(Q_ij); at i*N + j
  float qinv[RKLT_MAX_N * RKLT_MAX_N];
  float qstep[RKLT_MAX_N * RKLT_MAX_N];
  // region matrix-core kernel (m32_ok = 1 when it can take the transform):
  // a wave codes a 32 x 32 pixel region, (32 / N)^2 blocks of N in
  // {4, 8, 16, 32}, with Tb = T on the block diagonal (zero elsewhere) and
  // Gb likewise for T_hat^-1.  With h = lane / 32, c = lane % 32 and
  // kap(t, h) = 8 (t / 4) + 4 h + t % 4 (the row of accumulator register t):
  //   m32T[lane][w]  int8x4 words, byte e of word w = Tb[c][kap(4w + e, h)]:
  //                  B operand of the int8 row stage;
  //   m32W[t][lane]  s_i s_j of region coefficient (c, kap(t, h)), which is
  //                  coefficient (c % N, kap(t, h) % N) of one of the region's
  //                  blocks; m32R[t][lane] its zig-zag rank.
  //   m32Gs[k][p][lane][e]  Gb[c][kap(8k + e, h)] as two fp16 parts (p = 0:
  //                  Gb rounded to fp16, p = 1: the rest rounded to fp16): B
  //                  operands of both inverse stages.
  //   m32S[lane]     sig of region column c (row sum of T row c % N): the
  //                  level-shift correction (128 - ell) sig of the row stage.
  // m32_sig: the largest |sig_j| (bounds the corrected row sums).
  //   m32Ms[k][p][lane][e]  float transforms: Mb[c][kap(8k + e, h)] (M on
  //                  the block diagonal) as two fp16 parts: B operands of the
  //                  row and column stages; integer transforms: Tb in fp16
  //                  (exact, p = 1 zero), the B operand of the column stage.
  int32_t m32_ok, m32_sig, m32_pad[2];
  int32_t m32T[64][4];
  int32_t m32S[64];
  float m32W[16][64];
  int16_t m32R[16][64];
  _Float16 m32Gs[2][2][64][8];
  _Float16 m32Ms[2][2][64][8];
};

// One image of a launch (device memory for a plan, a kernel argument for the
// plain path).
struct DevImage {
  const uint8_t* src;
  uint8_t* dst;
  int32_t* coef;
  float* scaled;
  int32_t H, W, ps, pd;
  int32_t tid, r, ell, D;  // D: anti-diagonals i + j < D hold every kept coefficient
  int32_t bw, nblocks, tile0, ntiles;
  int32_t slot;            // index of this image's rklt_result
  int32_t tile_blocks;     // blocks per tile (the image has ntiles <= 65535 tiles)
  int32_t bwp;             // blocks per row of the block index space (see mfma8_pad_rows)
  int32_t pad;
};

struct KArgs {
  const DevImage* imgs;      // plan images, or nullptr for the plain path
  const int32_t* tile_img;   // image index of every tile (plan only)
  const int32_t* wg_tiles;   // matrix-core plans: tile range [wg_tiles[w], wg_tiles[w+1]) of workgroup w
  const DevTransform* tf;    // context transform table
  rklt_result* res;          // one per image
  int32_t total_tiles;
  int32_t dump;               // write coefficient dumps
  int32_t strided;            // matrix-core plans: workgroup w codes tiles w, w + grid, ...
  DevImage one;               // the image of the plain path
};

// The matrix-core kernel codes 32 consecutive blocks of one block row per
// wave step.  Images at least 32 blocks wide get a block index space whose
// rows are padded to a multiple of 32 blocks, so that no step straddles two
// block rows (a straddling step splits every load and store into short
// pieces, which costs about a third of the bandwidth); the padding blocks are
// never loaded or stored.  Narrower images keep their own width.
inline void mfma8_pad_rows(DevImage& d) {
  d.bwp = d.bw >= 32 ? (d.bw + 31) / 32 * 32 : d.bw;
  d.nblocks = (d.H / 8) * d.bwp;
}

// The panel kernel codes PB = panel_blocks(N) consecutive blocks of one
// block row per wave step: block rows are padded to a multiple of PB blocks
// in its block index space (the padding is never loaded or stored).
inline void panel_pad_rows(DevImage& d, int PB, int N) {
  d.bwp = (d.bw + PB - 1) / PB * PB;
  d.nblocks = (d.H / N) * d.bwp;
}

// Inverse form of the matrix-core kernel for r kept coefficients (see
// DevTransform): 1 and 3 exact, 2 FP32.
__host__ __device__ inline int mfma8_path(const DevTransform& t, int r) {
  return r <= t.m_r1 ? 1 : t.m_path3 ? 3 : 2;
}

// Number of anti-diagonals i + j < D that contain the first r zig-zag
// positions of an N x N block.
inline int diagonals_for(int N, int r) {
  int D = 0, covered = 0;
  while (covered < r) {
    covered += (D < N) ? D + 1 : 2 * N - 1 - D;
    ++D;
  }
  return D;
}

// Kernel launchers (codec.hip).
rklt_status launch_block8(const KArgs& a, int grid, int wg, void* stream);
rklt_status launch_mfma8(const KArgs& a, int grid, int wg, void* stream);
int mfma8_resident_wgs_per_cu(int wg);
// Panel kernel arithmetic: integer T within int8 (v_dot4), integer T beyond
// int8 (int32 products), or a float transform (FP32 throughout).
enum PanelMode { kPanelInt8 = 0, kPanelBigT = 1, kPanelFloat = 2 };
rklt_status launch_panel(int N, const KArgs& a, int grid, int mode, void* stream);

// MSSIM of a plan's images (codec_quality.hip): one record per image in
// slot order, tiles of 32 x 64 window positions numbered image by image.
struct MsImage {
  const uint8_t* x;  // source
  const uint8_t* y;  // reconstruction
  int32_t H, W, px, py;
  int32_t tile0, ntiles;  // this image's tiles (0 when it has no reconstruction or is smaller than 11)
  int32_t across;         // tiles per row of tiles
  int32_t slot;           // index of the result
};
struct MsArgs {
  const MsImage* imgs;  // n records, tile0 non-decreasing
  double* partials;     // one sum per tile
  double* out;          // one MSSIM per image slot
  int32_t n, total;
};
constexpr int kMsTileW = 64, kMsTileH = 32;
rklt_status launch_mssim(const MsArgs& a, int grid, void* stream);

// The region matrix-core kernel codes 32 x 32 pixel regions: its
// block index space is the grid of regions, ceil(H / 32) rows of
// ceil(W / 32) (regions past the image edge are partly out of range).
inline void mfma32_regions(DevImage& d) {
  d.bw = (d.W + 31) / 32;
  d.bwp = d.bw;
  d.nblocks = ((d.H + 31) / 32) * d.bw;
}
// mode: 0 rounded transforms, 1 quantised entries, 2 float transforms
rklt_status launch_mfma32(const KArgs& a, int grid, int mode, void* stream);
int mfma32_resident_wgs_per_cu(int mode);
rklt_status launch_copy(const void* src, void* dst, size_t nbytes, void* stream);
int panel_blocks(int N);  // blocks of one panel of the panel kernel
constexpr int kMaxTilesPerImage = 65535;  // tile count field of the packed accumulator

}  // namespace rklt
