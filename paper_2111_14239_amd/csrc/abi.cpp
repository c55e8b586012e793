// C ABI of librklt: error slot, contexts (device transform table), image
// validation, plans (device work lists) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rklt.h"
#include "rklt_internal.h"

struct rklt_ctx {
  int device = 0;
  int cus = 0;
  rklt::DevTransform* d_table = nullptr;
  std::vector<rklt::DevTransform> host;  // host mirror of the uploaded entries
  std::mutex mu;
};

// One launch of a plan: the images of one kernel class.  The offsets locate
// its work list (DevImage[n], tile -> image table, per-workgroup tile ranges)
// in the plan's device buffer.
struct PlanPart {
  int cls = 0;  // kernel class (see kernel_class)
  int n = 0;
  int64_t total_tiles = 0;
  int wg = 256;
  int grid = 0;
  size_t off_imgs = 0, off_tile_img = 0, off_wg_tiles = 0;
  bool has_wg_tiles = false;
  bool strided = false;  // matrix-core N = 8 kernel: tiles dealt round robin
  int mode = 0;  // panel kernel arithmetic (PanelMode)
};

// Kernel classes: 2 = matrix-core N = 8 kernel, 1 = register N = 8 kernel,
// 0 = panel kernel (integer T, any N, any level shift), 3 = panel kernel for
// float transforms, 4 = region matrix-core kernel, 5 = region kernel with
// the quantiser, 6 = region kernel for float transforms.
constexpr int kClasses = 7;

struct rklt_plan {
  rklt_ctx* ctx = nullptr;
  int N = 0;
  bool dump = false;
  int n = 0;
  int nparts = 0;
  PlanPart parts[kClasses];
  int64_t pixels = 0;
  rklt_tuning tuning{};
  bool has_tuning = false;
  // device work list and its host image (pinned when the plan is updated
  // asynchronously)
  void* d_buf = nullptr;
  size_t d_cap = 0;
  std::vector<unsigned char> h_image;
  void* h_pinned = nullptr;
  size_t h_cap = 0;
  // the caller's descriptors of the current images (for re-tiling)
  std::vector<rklt_image> images;
  // MSSIM work list (records in the device buffer, then the per-tile sums)
  size_t off_ms = 0, off_partials = 0, d_need = 0;
  int ms_total = 0;
};

namespace rklt {

namespace {
thread_local char g_error[512] = "";

constexpr int kDefaultWg = 256;
constexpr int kDefaultBpt = 1;

// Kernel class of an image (see kClasses).  Coefficient dumps are written by
// the register and panel kernels.
int kernel_class(const DevTransform& t, int ell, bool dump);
bool panel_class(int cls) { return cls == 0 || cls == 3; }

bool block8_fits(const DevTransform& t, int ell) {
  // level shift 128 (pixel xor 0x80), int8 entries for the row dots and
  // |Y| <= 128 * L1 within int16 for the column dots
  return ell == 128 && t.N == 8 && t.max_abs <= 127 && 128 * t.max_row_l1 <= 32767;
}

// The region kernel splits the corrected row sums Y = (A - 128) T^T +
// (128 - ell) sig into two signed bytes, hi = byte 1 of Y + 128: Y must lie
// in [-32640, 32639].  Pixels - 128 lie in [-128, 127], so -128 L1 - c <= Y
// <= 127 L1 + c with c = |128 - ell| max|sig|, and 128 L1 + c <= 32640
// keeps both ends inside (L1 >= 1).
bool region_fits(const DevTransform& t, int ell) {
  const int lift = 128 - ell;
  return t.m32_ok && 128 * t.max_row_l1 + (lift < 0 ? -lift : lift) * t.m32_sig <= 32640;
}

int kernel_class(const DevTransform& t, int ell, bool dump) {
  if (t.is_float) return (!dump && t.m32_ok) ? 6 : 3;
  if (t.quant) return (!dump && region_fits(t, ell)) ? 5 : 0;
  if (block8_fits(t, ell)) return (t.m_ok && !dump) ? 2 : 1;
  if (!dump && region_fits(t, ell)) return 4;
  return 0;
}

hipError_t use_device(int device) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  return cur == device ? hipSuccess : hipSetDevice(device);
}

rklt_status hip_fail(const char* what, hipError_t e) {
  return fail(RKLT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Check one image against the context and fill its device descriptor
// (tile fields excluded).
rklt_status check_image(rklt_ctx* ctx, const rklt_image& im, int index, DevImage* out, int* N_out) {
  if (im.transform_id < 0 || im.transform_id >= static_cast<int>(ctx->host.size()))
    return fail(RKLT_E_INVAL, "image %d: unknown transform_id %d", index, im.transform_id);
  const DevTransform& t = ctx->host[im.transform_id];
  const int N = t.N;
  if (!im.src) return fail(RKLT_E_INVAL, "image %d: src is NULL", index);
  if (im.H < N || im.W < N || im.H % N || im.W % N)
    return fail(RKLT_E_INVAL, "image %d: H=%d W=%d are not positive multiples of N=%d", index, im.H, im.W, N);
  if (static_cast<int64_t>(im.H) * im.W >= (int64_t{1} << 31))
    return fail(RKLT_E_INVAL, "image %d: H*W=%lld exceeds 2^31-1 pixels", index,
                static_cast<long long>(im.H) * im.W);
  if (im.pitch_src < im.W || im.pitch_src % 8)
    return fail(RKLT_E_INVAL, "image %d: pitch_src=%d must be >= W=%d and a multiple of 8", index,
                im.pitch_src, im.W);
  if (reinterpret_cast<uintptr_t>(im.src) % 8)
    return fail(RKLT_E_INVAL, "image %d: src is not 8-byte aligned", index);
  // the kernels address an image with 32-bit byte offsets and mark missing
  // blocks with offset 2^31, so an image must span less than 2^31 bytes
  if (static_cast<int64_t>(im.H - 1) * im.pitch_src + im.W >= (int64_t{1} << 31))
    return fail(RKLT_E_INVAL, "image %d: (H-1)*pitch_src+W spans 2^31 bytes or more", index);
  if (im.dst) {
    if (im.pitch_dst < im.W || im.pitch_dst % 8)
      return fail(RKLT_E_INVAL, "image %d: pitch_dst=%d must be >= W=%d and a multiple of 8", index,
                  im.pitch_dst, im.W);
    if (reinterpret_cast<uintptr_t>(im.dst) % 8)
      return fail(RKLT_E_INVAL, "image %d: dst is not 8-byte aligned", index);
    if (static_cast<int64_t>(im.H - 1) * im.pitch_dst + im.W >= (int64_t{1} << 31))
      return fail(RKLT_E_INVAL, "image %d: (H-1)*pitch_dst+W spans 2^31 bytes or more", index);
  }
  if (im.r < 1 || im.r > N * N)
    return fail(RKLT_E_INVAL, "image %d: r=%d outside 1..%d", index, im.r, N * N);
  if (im.level_shift < 0 || im.level_shift > 255)
    return fail(RKLT_E_INVAL, "image %d: level_shift=%d outside 0..255", index, im.level_shift);
  if (im.reserved != 0) return fail(RKLT_E_INVAL, "image %d: reserved field is not 0", index);
  if (t.is_float && im.coef_out)
    return fail(RKLT_E_INVAL, "image %d: coef_out (integer coefficients) with a float transform", index);
  DevImage& d = *out;
  std::memset(&d, 0, sizeof(d));
  d.src = im.src;
  d.dst = im.dst;
  d.coef = im.coef_out;
  d.scaled = im.scaled_out;
  d.H = im.H;
  d.W = im.W;
  d.ps = im.pitch_src;
  d.pd = im.dst ? im.pitch_dst : 0;
  d.tid = im.transform_id;
  d.r = im.r;
  d.ell = im.level_shift;
  d.D = diagonals_for(N, im.r);
  d.bw = im.W / N;
  d.bwp = d.bw;
  d.nblocks = (im.H / N) * (im.W / N);
  *N_out = N;
  return RKLT_OK;
}

// Forward operand of the matrix-core kernel (v_mfma_i32_32x32x32_i8 A
// operand): lane `lane` of row chunk mu and K-chunk c holds 16 int8 weights
// T[i][m] T[j][n] of the coefficient (i, j) with zig-zag rank 32 mu + lane % 32
// against the pixels (m, n) of rows 4c + 2 (lane / 32) + e / 8, column e % 8.
void fill_forward_operand(const int32_t* T, const int32_t* order, int32_t (&mF)[2][2][64][4]) {
  for (int mu = 0; mu < 2; ++mu)
    for (int c = 0; c < 2; ++c)
      for (int lane = 0; lane < 64; ++lane) {
        const int o = order[32 * mu + (lane & 31)];
        const int i = o / 8, j = o % 8;
        for (int w = 0; w < 4; ++w) {
          uint32_t word = 0;
          for (int b = 0; b < 4; ++b) {
            const int e = 4 * w + b;
            const int row = 4 * c + 2 * (lane >> 5) + e / 8, col = e % 8;
            const int v = T[i * 8 + row] * T[j * 8 + col];
            word |= (static_cast<uint32_t>(v) & 0xffu) << (8 * b);
          }
          mF[mu][c][lane][w] = static_cast<int32_t>(word);
        }
      }
}

// Blocks per tile for one image: the launch's tile size, grown (in steps of
// `unit` blocks) until the image has at most kMaxTilesPerImage tiles.
int image_tile_blocks(const DevImage& d, int base, int unit) {
  int tb = base;
  const int64_t need = (static_cast<int64_t>(d.nblocks) + kMaxTilesPerImage - 1) / kMaxTilesPerImage;
  if (tb < need) tb = static_cast<int>((need + unit - 1) / unit * unit);
  return tb;
}

rklt_status check_tuning(const rklt_tuning* tu, int* wg, int* bpt, int* grid, int* sched) {
  *wg = kDefaultWg;
  *bpt = kDefaultBpt;
  *grid = 0;
  *sched = 0;
  if (!tu) return RKLT_OK;
  if (tu->wg_threads) {
    if (tu->wg_threads != 64 && tu->wg_threads != 128 && tu->wg_threads != 256)
      return fail(RKLT_E_INVAL, "tuning: wg_threads=%d not in {64, 128, 256}", tu->wg_threads);
    *wg = tu->wg_threads;
  }
  if (tu->blocks_per_thread) {
    if (tu->blocks_per_thread < 1 || tu->blocks_per_thread > 16)
      return fail(RKLT_E_INVAL, "tuning: blocks_per_thread=%d outside 1..16", tu->blocks_per_thread);
    *bpt = tu->blocks_per_thread;
  }
  if (tu->grid_wgs < 0) return fail(RKLT_E_INVAL, "tuning: grid_wgs=%d is negative", tu->grid_wgs);
  *grid = tu->grid_wgs;
  if (tu->schedule != 0 && tu->schedule != 1)
    return fail(RKLT_E_INVAL, "tuning: schedule=%d not in {0, 1}", tu->schedule);
  *sched = tu->schedule;
  return RKLT_OK;
}

}  // namespace

rklt_status fail(rklt_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_error[0] = '\0'; }

}  // namespace rklt

using namespace rklt;

extern "C" {

const char* rklt_last_error(void) { return g_error; }

rklt_status rklt_build_transform(int32_t N, double rho, double alpha, rklt_transform* out) {
  clear_error();
  return build_transform(N, rho, alpha, out);
}

rklt_status rklt_zigzag(int32_t N, int32_t* order) {
  clear_error();
  return zigzag(N, order);
}

rklt_status rklt_ctx_create(int32_t device, rklt_ctx** out) {
  clear_error();
  if (!out) return fail(RKLT_E_INVAL, "rklt_ctx_create: out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail("hipGetDeviceCount", e);
  if (device < 0 || device >= count)
    return fail(RKLT_E_INVAL, "rklt_ctx_create: device %d not in 0..%d", device, count - 1);
  rklt_ctx* ctx = new (std::nothrow) rklt_ctx;
  if (!ctx) return fail(RKLT_E_NOMEM, "rklt_ctx_create: out of host memory");
  ctx->device = device;
  if ((e = use_device(device)) != hipSuccess) {
    delete ctx;
    return hip_fail("hipSetDevice", e);
  }
  e = hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) {
    delete ctx;
    return hip_fail("hipDeviceGetAttribute", e);
  }
  e = hipMalloc(&ctx->d_table, sizeof(DevTransform) * kMaxTransforms);
  if (e != hipSuccess) {
    delete ctx;
    return fail(RKLT_E_NOMEM, "rklt_ctx_create: hipMalloc of the transform table: %s", hipGetErrorString(e));
  }
  ctx->host.reserve(kMaxTransforms);
  *out = ctx;
  return RKLT_OK;
}

rklt_status rklt_ctx_destroy(rklt_ctx* ctx) {
  clear_error();
  if (!ctx) return fail(RKLT_E_INVAL, "rklt_ctx_destroy: ctx is NULL");
  if (ctx->d_table) {
    (void)use_device(ctx->device);
    (void)hipFree(ctx->d_table);
  }
  delete ctx;
  return RKLT_OK;
}

rklt_status rklt_ctx_add_transform(rklt_ctx* ctx, const rklt_transform* t, int32_t* id_out) {
  clear_error();
  if (!ctx || !t || !id_out) return fail(RKLT_E_INVAL, "rklt_ctx_add_transform: NULL argument");
  const int N = t->N;
  if (N != 4 && N != 8 && N != 16 && N != 32)
    return fail(RKLT_E_INVAL, "rklt_ctx_add_transform: N=%d; the codec supports N in {4, 8, 16, 32}", N);
  int max_abs = 0, max_l1 = 0;
  for (int i = 0; i < N; ++i) {
    int l1 = 0;
    for (int j = 0; j < N; ++j) {
      const int v = std::abs(t->T[i * N + j]);
      if (v > 1000000) return fail(RKLT_E_RANGE, "rklt_ctx_add_transform: |T| too large");
      l1 += v;
      max_abs = v > max_abs ? v : max_abs;
    }
    if (t->d[i] <= 0 || !(t->s[i] > 0.0))
      return fail(RKLT_E_SINGULAR, "rklt_ctx_add_transform: row %d has d_i <= 0", i);
    max_l1 = l1 > max_l1 ? l1 : max_l1;
  }
  // |B| <= 255 * L1^2 for pixels shifted by any ell in 0..255
  if (255.0 * max_l1 * max_l1 >= 2147483647.0)
    return fail(RKLT_E_RANGE, "rklt_ctx_add_transform: 255 * L1^2 = %.0f overflows int32 (L1=%d)",
                255.0 * max_l1 * max_l1, max_l1);

  DevTransform dt;
  std::memset(&dt, 0, sizeof(dt));
  dt.N = N;
  dt.flags = t->flags;
  dt.max_abs = max_abs;
  dt.max_row_l1 = max_l1;
  int32_t order[RKLT_MAX_N * RKLT_MAX_N];
  zigzag(N, order);
  for (int k = 0; k < N * N; ++k) dt.rank[order[k]] = k;
  for (int i = 0; i < N; ++i) {
    int sig = 0;
    for (int j = 0; j < N; ++j) {
      sig += t->T[i * N + j];
      dt.T[i * N + j] = t->T[i * N + j];
      dt.w[i * N + j] = static_cast<float>(t->s[i] * t->s[j]);
      dt.G[i * N + j] = static_cast<float>(t->G[i * N + j]);
    }
    dt.sig[i] = sig;
  }
  for (int i = 0; i < N; ++i)
    for (int m = 0; m < N; ++m) dt.Gt[i * N + m] = dt.G[m * N + i];
  if (max_abs <= 127)
    for (int j = 0; j < N; ++j)
      for (int w = 0; w < N / 4; ++w) {
        uint32_t word = 0;
        for (int e = 0; e < 4; ++e) word |= (static_cast<uint32_t>(t->T[j * N + 4 * w + e]) & 0xffu) << (8 * e);
        dt.Tw[j * (N / 4) + w] = static_cast<int32_t>(word);
      }
  if (N == 8) {
    // Exact inverse for the N = 8 register kernel, with the bounds that keep
    // every inverse stage exact in FP32: |B_ij| <= 128 L1_i L1_j (pixels - 128
    // lie in [-128, 127]); every product and partial sum of W = adj B and of
    // Out = W adj^T is bounded by wmax and omax, which must stay below 2^24
    // so that each FMA on these integers is exact; and half the spacing
    // 1/den^2 of the rationals Out/den^2 must exceed twice the FP32 rounding
    // error of Out/den^2 + 128 (<= 4e-5).
    int64_t adj[64], den = 0;
    if (exact_inverse(8, t->T, adj, &den)) {
      double L1[8];
      for (int i = 0; i < 8; ++i) {
        L1[i] = 0;
        for (int j = 0; j < 8; ++j) L1[i] += std::abs(t->T[i * 8 + j]);
      }
      double wmax = 0, omax = 0, amax = 0;
      for (int m = 0; m < 8; ++m) {
        for (int j = 0; j < 8; ++j) {
          double w = 0;
          for (int i = 0; i < 8; ++i) w += std::fabs(static_cast<double>(adj[m * 8 + i])) * 128.0 * L1[i] * L1[j];
          wmax = std::fmax(wmax, w);
        }
        for (int n = 0; n < 8; ++n) {
          double o = 0;
          for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j)
              o += std::fabs(static_cast<double>(adj[m * 8 + i])) * std::fabs(static_cast<double>(adj[n * 8 + j])) *
                   128.0 * L1[i] * L1[j];
          omax = std::fmax(omax, o);
        }
        for (int i = 0; i < 8; ++i) amax = std::fmax(amax, std::fabs(static_cast<double>(adj[m * 8 + i])));
      }
      const double d2 = static_cast<double>(den) * static_cast<double>(den);
      const double delta = (den % 2 == 0) ? 0.5 / d2 : 0.25 / d2;
      const bool ok = wmax < 16777216.0 && omax < 16777216.0 && amax < 16777216.0 && delta > 8e-5;
      if (ok) {
        dt.exact = 1;  // (exact = 0 and the FP32 constants are set below otherwise)
        dt.den = static_cast<int32_t>(den);
        dt.inv_den2 = static_cast<float>(1.0 / d2);
        dt.bias = static_cast<float>(128.0 + delta);
        for (int k = 0; k < 64; ++k) {
          dt.adj[k] = static_cast<int32_t>(adj[k]);
          dt.fadj[k] = static_cast<float>(adj[k]);
        }
      }
    }
  }
  if (N == 8 && !dt.exact) {
    dt.den = 0;
    dt.inv_den2 = 1.0f;
    dt.bias = 128.0f + 1.0f / 4096.0f;
    // T^-1 = T_hat^-1 S in FP32
    for (int m = 0; m < 8; ++m)
      for (int i = 0; i < 8; ++i) dt.fadj[m * 8 + i] = static_cast<float>(t->G[m * 8 + i] * t->s[i]);
  }
  if (N == 8 && max_abs * max_abs <= 127) {
    // Matrix-core operands.  The forward weights T_im T_jn fit int8.  The
    // inverse weights of output pixel (m, n) against coefficient k = (i, j)
    // are w = adj_mi adj_nj (exact inverse T^-1 = adj / den), and
    // |B_k| <= Bmax_k = 128 L1_i L1_j.  Per (transform, r) the kernel takes
    //   1  one fp16 pass, B = hi + lo with hi = B rounded toward zero to fp16
    //      and |lo| < 16 (needs |B| < 32768): exact when every partial sum,
    //      at most S_r = sum_{k<r} |w_k| (Bmax_k + 16), stays below 2^24;
    //      m_r1 is the largest such r;
    //   3  two accumulators, hi = B rounded to a multiple of 64 and lo = B - hi
    //      (|lo| <= 32): the hi sums are multiples of 64 below 2^30 and the lo
    //      sums below 2^24, so both are exact, and so is their sum Out when
    //      |Out| < 2^24.  Out = den^2 (A - 128) minus the dropped terms, so
    //      |Out| <= min(P_r, 128 den^2 + P_64 - P_r), P_r = sum_{k<r} |w_k| Bmax_k;
    //   2  FP32 (v_mfma_f32_32x32x2_f32) otherwise.
    // The weights must be exact fp16 integers (|w| <= 2048) for forms 1 and 3,
    // and the epilogue's rounding argument needs delta > 8e-5 (as for the
    // register kernel).
    int32_t order[64];
    zigzag(8, order);
    fill_forward_operand(t->T, order, dt.mF);
    double L1[8];
    for (int i = 0; i < 8; ++i) {
      L1[i] = 0;
      for (int j = 0; j < 8; ++j) L1[i] += std::abs(t->T[i * 8 + j]);
    }
    int64_t madj[64], mden = 0;
    bool mex = exact_inverse(8, t->T, madj, &mden);
    double d2 = 0, delta = 0;
    if (mex) {
      d2 = static_cast<double>(mden) * static_cast<double>(mden);
      delta = (mden % 2 == 0) ? 0.5 / d2 : 0.25 / d2;
      mex = delta > 8e-5;
    }
    bool wfit = mex;  // weights exact in fp16 and |B| < 32768
    for (int k = 0; k < 64 && wfit; ++k) {
      const int i = order[k] / 8, j = order[k] % 8;
      if (128.0 * L1[i] * L1[j] >= 32768.0) wfit = false;
      for (int m = 0; m < 8 && wfit; ++m)
        if (std::llabs(madj[m * 8 + i]) * std::llabs(madj[m * 8 + j]) > 2048) wfit = false;
    }
    // largest r for form 1, and form 3's bounds, over every output pixel
    int r1 = wfit ? 64 : 0;
    bool path3 = wfit;
    if (wfit) {
      for (int m = 0; m < 8; ++m)
        for (int n = 0; n < 8; ++n) {
          double S = 0, P[65], hi = 0, lo = 0;
          P[0] = 0;
          for (int k = 0; k < 64; ++k) {
            const int i = order[k] / 8, j = order[k] % 8;
            const double w = std::fabs(static_cast<double>(madj[m * 8 + i]) * static_cast<double>(madj[n * 8 + j]));
            const double bmax = 128.0 * L1[i] * L1[j];
            S += w * (bmax + 16.0);
            if (S >= 16777216.0 && k < r1) r1 = k;  // r = k + 1 coefficients break the bound
            P[k + 1] = P[k] + w * bmax;
            hi += w * (bmax + 32.0);
            lo += w * 32.0;
          }
          if (hi >= 1073741824.0 || lo >= 16777216.0) path3 = false;
          for (int r = 1; r <= 64 && path3; ++r)
            if (std::fmin(P[r], 128.0 * d2 + P[64] - P[r]) >= 16777216.0) path3 = false;
        }
    }
    dt.m_ok = 1;
    dt.m_r1 = r1;
    dt.m_path3 = path3 ? 1 : 0;
    dt.m_den = mex ? static_cast<int32_t>(mden) : 0;
    dt.m_inv = mex ? static_cast<float>(1.0 / d2) : 1.0f;
    dt.m_bias = mex ? static_cast<float>(128.0 + delta) : 128.0f + 1.0f / 4096.0f;
    for (int mu = 0; mu < 2; ++mu)
      for (int kappa = 0; kappa < 8; ++kappa)
        for (int lane = 0; lane < 64; ++lane) {
          // A-operand row: pixel M = lane % 32 of pixel chunk mu
          const int M = lane & 31;
          const int g = M >> 3, hm = (M >> 2) & 1, vm = M & 3;
          const int m = 4 * mu + 2 * hm + g / 2, n = 4 * (g % 2) + vm;
          if (wfit) {
            for (int e = 0; e < 8; ++e) {
              // halves e = [hi v0, hi v1, lo v0, lo v1, hi v2, hi v3, lo v2, lo v3]
              const int v = 2 * (e >> 2) + (e & 1);
              const int o = order[8 * kappa + 4 * (lane >> 5) + v];
              const int i = o / 8, j = o % 8;
              dt.mV[mu][kappa][lane][e] = static_cast<_Float16>(static_cast<float>(madj[m * 8 + i] * madj[n * 8 + j]));
            }
          }
          for (int v = 0; v < 4; ++v) {
            const int o = order[8 * kappa + 4 * (lane >> 5) + v];
            const int i = o / 8, j = o % 8;
            const double w = mex ? static_cast<double>(madj[m * 8 + i]) * static_cast<double>(madj[n * 8 + j])
                                 : static_cast<double>(t->G[m * 8 + i]) * t->s[i] * t->G[n * 8 + j] * t->s[j];
            dt.mVf[mu][kappa][v][lane] = static_cast<float>(w);
          }
        }
  }
  if (N == 8 && max_abs <= 127) {
    for (int j = 0; j < 8; ++j) {
      for (int h = 0; h < 2; ++h) {
        uint32_t word = 0;
        for (int b = 0; b < 4; ++b) word |= (static_cast<uint32_t>(t->T[j * 8 + 4 * h + b]) & 0xffu) << (8 * b);
        dt.t8[j][h] = static_cast<int32_t>(word);
      }
      for (int p = 0; p < 4; ++p) {
        const uint32_t lo = static_cast<uint32_t>(t->T[j * 8 + 2 * p]) & 0xffffu;
        const uint32_t hi = static_cast<uint32_t>(t->T[j * 8 + 2 * p + 1]) & 0xffffu;
        dt.t16[j][p] = static_cast<int32_t>(lo | (hi << 16));
      }
    }
  }

  if (max_abs <= 127 && 128 * max_l1 <= 32640) {
    // region matrix-core operands (layout in DevTransform): Tb and Gb on the
    // block diagonal of a 32 x 32 region, K order kap(e, h)
    auto kap = [](int t, int h) { return 8 * (t >> 2) + 4 * h + (t & 3); };
    dt.m32_ok = 1;
    for (int i = 0; i < N; ++i) dt.m32_sig = std::max(dt.m32_sig, std::abs(dt.sig[i]));
    for (int lane = 0; lane < 64; ++lane) {
      const int h = lane >> 5, c = lane & 31;
      dt.m32S[lane] = dt.sig[c % N];
      for (int w = 0; w < 4; ++w) {
        uint32_t word = 0;
        for (int b = 0; b < 4; ++b) {
          const int n = kap(4 * w + b, h);
          const int v = (c / N == n / N) ? t->T[(c % N) * N + n % N] : 0;
          word |= (static_cast<uint32_t>(v) & 0xffu) << (8 * b);
        }
        dt.m32T[lane][w] = static_cast<int32_t>(word);
      }
      for (int tt = 0; tt < 16; ++tt) {
        const int j = kap(tt, h);
        const bool diag = c / N == j / N;
        const double gv = diag ? t->G[(c % N) * N + j % N] : 0.0;
        const _Float16 ghi = static_cast<_Float16>(gv);
        dt.m32Gs[tt / 8][0][lane][tt % 8] = ghi;
        dt.m32Gs[tt / 8][1][lane][tt % 8] = static_cast<_Float16>(gv - static_cast<double>(ghi));
        // coefficient (c, j) of the region is coefficient (c % N, j % N) of
        // one of its blocks (all four quadrants hold coefficients)
        dt.m32W[tt][lane] = static_cast<float>(t->s[c % N] * t->s[j % N]);
        dt.m32R[tt][lane] = static_cast<int16_t>(dt.rank[(c % N) * N + j % N]);
        // Tb in fp16 (exact: |T_ij| <= 127) for the column stage; no lo part
        dt.m32Ms[tt / 8][0][lane][tt % 8] =
            static_cast<_Float16>(diag ? t->T[(c % N) * N + j % N] : 0);
        dt.m32Ms[tt / 8][1][lane][tt % 8] = static_cast<_Float16>(0);
      }
    }
  }

  std::lock_guard<std::mutex> lock(ctx->mu);
  for (size_t k = 0; k < ctx->host.size(); ++k) {
    const DevTransform& o = ctx->host[k];
    if (!o.is_float && !o.quant && o.N == N && std::memcmp(o.T, dt.T, sizeof(int32_t) * N * N) == 0) {
      *id_out = static_cast<int32_t>(k);
      return RKLT_OK;
    }
  }
  if (ctx->host.size() >= static_cast<size_t>(kMaxTransforms))
    return fail(RKLT_E_NOMEM, "rklt_ctx_add_transform: table full (%d transforms)", kMaxTransforms);
  const int id = static_cast<int>(ctx->host.size());
  hipError_t e = use_device(ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  e = hipMemcpy(ctx->d_table + id, &dt, sizeof(dt), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("rklt_ctx_add_transform: hipMemcpy", e);
  ctx->host.push_back(dt);
  *id_out = id;
  return RKLT_OK;
}

rklt_status rklt_transform_measures(int32_t N, const double* That, const double* ref, double rho,
                                    rklt_measures* out) {
  clear_error();
  return transform_measures(N, That, ref, rho, out);
}

rklt_status rklt_algorithm1(int32_t N, double alpha, double step, rklt_design_entry* out, int32_t cap,
                            int32_t* count) {
  clear_error();
  return algorithm1(N, alpha, step, out, cap, count);
}

rklt_status rklt_klt_matrix(int32_t N, double rho, double* K) {
  clear_error();
  return klt_matrix(N, rho, K);
}

rklt_status rklt_dct_matrix(int32_t N, double* C) {
  clear_error();
  return dct_matrix(N, C);
}

rklt_status rklt_ctx_add_float_transform(rklt_ctx* ctx, int32_t N, const double* M, int32_t* id_out) {
  clear_error();
  if (!ctx || !M || !id_out) return fail(RKLT_E_INVAL, "rklt_ctx_add_float_transform: NULL argument");
  if (N != 4 && N != 8 && N != 16 && N != 32)
    return fail(RKLT_E_INVAL, "rklt_ctx_add_float_transform: N=%d; the codec supports N in {4, 8, 16, 32}", N);
  for (int k = 0; k < N * N; ++k)
    if (!std::isfinite(M[k]) || std::fabs(M[k]) > 1e6)
      return fail(RKLT_E_INVAL, "rklt_ctx_add_float_transform: M[%d]=%g is not finite or beyond 1e6", k, M[k]);
  double G[RKLT_MAX_N * RKLT_MAX_N];
  if (!invert_matrix(N, M, G)) return fail(RKLT_E_SINGULAR, "rklt_ctx_add_float_transform: M is singular");
  DevTransform dt;
  std::memset(&dt, 0, sizeof(dt));
  dt.N = N;
  dt.is_float = 1;
  int32_t order[RKLT_MAX_N * RKLT_MAX_N];
  zigzag(N, order);
  for (int k = 0; k < N * N; ++k) dt.rank[order[k]] = k;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      dt.w[i * N + j] = 1.0f;
      dt.Mf[i * N + j] = static_cast<float>(M[i * N + j]);
      dt.G[i * N + j] = static_cast<float>(G[i * N + j]);
      dt.Gt[j * N + i] = dt.G[i * N + j];
    }
  {
    // region kernel operands (layout in DevTransform): M and M^-1 on the
    // block diagonal as two fp16 parts, unit weights, zig-zag ranks
    auto kap = [](int t, int h) { return 8 * (t >> 2) + 4 * h + (t & 3); };
    dt.m32_ok = 1;
    for (int lane = 0; lane < 64; ++lane) {
      const int h = lane >> 5, c = lane & 31;
      for (int tt = 0; tt < 16; ++tt) {
        const int j = kap(tt, h);
        const bool diag = c / N == j / N;
        const double mv = diag ? M[(c % N) * N + j % N] : 0.0;
        const double gv = diag ? G[(c % N) * N + j % N] : 0.0;
        const _Float16 mhi = static_cast<_Float16>(mv), ghi = static_cast<_Float16>(gv);
        dt.m32Ms[tt / 8][0][lane][tt % 8] = mhi;
        dt.m32Ms[tt / 8][1][lane][tt % 8] = static_cast<_Float16>(mv - static_cast<double>(mhi));
        dt.m32Gs[tt / 8][0][lane][tt % 8] = ghi;
        dt.m32Gs[tt / 8][1][lane][tt % 8] = static_cast<_Float16>(gv - static_cast<double>(ghi));
        dt.m32W[tt][lane] = 1.0f;
        dt.m32R[tt][lane] = static_cast<int16_t>(dt.rank[(c % N) * N + j % N]);
      }
    }
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  for (size_t k = 0; k < ctx->host.size(); ++k) {
    const DevTransform& o = ctx->host[k];
    if (o.is_float && o.N == N && std::memcmp(o.Mf, dt.Mf, sizeof(float) * N * N) == 0 &&
        std::memcmp(o.Gt, dt.Gt, sizeof(float) * N * N) == 0) {
      *id_out = static_cast<int32_t>(k);
      return RKLT_OK;
    }
  }
  if (ctx->host.size() >= static_cast<size_t>(kMaxTransforms))
    return fail(RKLT_E_NOMEM, "rklt_ctx_add_float_transform: table full (%d transforms)", kMaxTransforms);
  const int id = static_cast<int>(ctx->host.size());
  hipError_t e = use_device(ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  e = hipMemcpy(ctx->d_table + id, &dt, sizeof(dt), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("rklt_ctx_add_float_transform: hipMemcpy", e);
  ctx->host.push_back(dt);
  *id_out = id;
  return RKLT_OK;
}

rklt_status rklt_ctx_add_quantizer(rklt_ctx* ctx, int32_t transform_id, const double* Q, int32_t* id_out) {
  clear_error();
  if (!ctx || !Q || !id_out) return fail(RKLT_E_INVAL, "rklt_ctx_add_quantizer: NULL argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (transform_id < 0 || transform_id >= static_cast<int>(ctx->host.size()))
    return fail(RKLT_E_INVAL, "rklt_ctx_add_quantizer: unknown transform id %d", transform_id);
  DevTransform dt = ctx->host[transform_id];
  if (dt.is_float || dt.quant)
    return fail(RKLT_E_INVAL, "rklt_ctx_add_quantizer: transform %d is not a rounded (integer) transform",
                transform_id);
  const int N = dt.N;
  for (int k = 0; k < N * N; ++k)
    if (!(Q[k] > 0.0) || !(Q[k] <= 1e6))
      return fail(RKLT_E_INVAL, "rklt_ctx_add_quantizer: Q[%d]=%g outside (0, 1e6]", k, Q[k]);
  // s_i s_j = w_ij exactly as the host designed it: recompute s in FP64
  double s[RKLT_MAX_N];
  for (int i = 0; i < N; ++i) {
    int64_t d = 0;
    for (int j = 0; j < N; ++j) d += static_cast<int64_t>(dt.T[i * N + j]) * dt.T[i * N + j];
    s[i] = 1.0 / std::sqrt(static_cast<double>(d));
  }
  // quantised entries run on the region kernel (class 5) or the panel
  // kernel: neither N = 8 kernel (nor its exactness report) applies
  dt.quant = 1;
  dt.m_ok = 0;
  dt.exact = 0;
  dt.den = 0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      dt.qinv[i * N + j] = static_cast<float>((s[i] * s[j]) / Q[i * N + j]);
      dt.qstep[i * N + j] = static_cast<float>(Q[i * N + j]);
    }
  for (size_t k = 0; k < ctx->host.size(); ++k) {
    const DevTransform& o = ctx->host[k];
    if (o.quant && o.N == N && std::memcmp(o.T, dt.T, sizeof(int32_t) * N * N) == 0 &&
        std::memcmp(o.qinv, dt.qinv, sizeof(float) * N * N) == 0 &&
        std::memcmp(o.qstep, dt.qstep, sizeof(float) * N * N) == 0) {
      *id_out = static_cast<int32_t>(k);
      return RKLT_OK;
    }
  }
  if (ctx->host.size() >= static_cast<size_t>(kMaxTransforms))
    return fail(RKLT_E_NOMEM, "rklt_ctx_add_quantizer: table full (%d transforms)", kMaxTransforms);
  const int id = static_cast<int>(ctx->host.size());
  hipError_t e = use_device(ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  e = hipMemcpy(ctx->d_table + id, &dt, sizeof(dt), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("rklt_ctx_add_quantizer: hipMemcpy", e);
  ctx->host.push_back(dt);
  *id_out = id;
  return RKLT_OK;
}

rklt_status rklt_codec(rklt_ctx* ctx, const rklt_image* img, rklt_result* d_res, const rklt_tuning* tuning,
                       void* stream) {
  clear_error();
  if (!ctx || !img || !d_res) return fail(RKLT_E_INVAL, "rklt_codec: NULL argument");
  int wg, bpt, grid_req, sched;
  rklt_status st = check_tuning(tuning, &wg, &bpt, &grid_req, &sched);
  if (st) return st;
  if (!tuning) {
    // One image per launch: small tiles, so that even a 1-megapixel image
    // spreads over every CU.
    wg = 64;
    bpt = 1;
  }
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  int N = 0;
  {
    std::lock_guard<std::mutex> lock(ctx->mu);
    if ((st = check_image(ctx, *img, 0, &a.one, &N))) return st;
    a.dump = (img->coef_out || img->scaled_out) ? 1 : 0;
    const int cls = kernel_class(ctx->host[img->transform_id], img->level_shift, a.dump != 0);
    const int mode = cls == 3 ? kPanelFloat : ctx->host[img->transform_id].max_abs > 127 ? kPanelBigT : kPanelInt8;
    const int PB = panel_blocks(N);
    if (cls == 2) mfma8_pad_rows(a.one);
    if (panel_class(cls)) panel_pad_rows(a.one, PB, N);
    if (cls >= 4) mfma32_regions(a.one);
    a.one.tile0 = 0;
    a.one.slot = 0;
    a.one.tile_blocks = cls == 2   ? image_tile_blocks(a.one, (wg / 2) * bpt, wg / 2)
                        : cls == 1 ? image_tile_blocks(a.one, wg * bpt, wg)
                        : cls >= 4 ? image_tile_blocks(a.one, 16, 4)
                                   : image_tile_blocks(a.one, 4 * PB, 4 * PB);
    a.one.ntiles = (a.one.nblocks + a.one.tile_blocks - 1) / a.one.tile_blocks;
    a.total_tiles = a.one.ntiles;
    a.tf = ctx->d_table;
    a.res = d_res;
    hipError_t e = use_device(ctx->device);
    if (e != hipSuccess) return hip_fail("hipSetDevice", e);
    const int grid = a.total_tiles;
    return cls == 2 ? launch_mfma8(a, grid, wg, stream)
           : cls == 1 ? launch_block8(a, grid, wg, stream)
           : cls >= 4 ? launch_mfma32(a, grid, cls - 4, stream)
                      : launch_panel(N, a, grid, mode, stream);
  }
}

namespace {

// Cost of one 8x8 block in the matrix-core kernel for each inverse form and
// number R8 = ceil(r / 8) of 8-coefficient chunks: picoseconds per block of
// a full-chip launch, measured on MI355X with batches of one form and one R8.
// Form 1 is bound by memory up to 32 coefficients; forms 3 and 2 (two
// accumulators; eight 32x32x2 products per chunk) by the matrix cores.
constexpr double kMfma8ImageCost = 150 * 22.2;

double mfma8_block_cost(int path, int r) {
  static const double form1[8] = {22.3, 21.9, 22.1, 22.2, 22.9, 24.4, 26.2, 26.9};
  const int R8 = (r + 7) / 8;
  if (path == 1) return form1[R8 - 1];
  if (path == 3) return 21.0 + 3.3 * R8;
  return 17.6 + 5.1 * R8;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Tile the images of one kernel class and append its work list to `img`
// (the plan's host image of the device buffer).
rklt_status build_part(rklt_ctx* ctx, std::vector<DevImage>& imgs, int cls, int wg, int bpt, int grid_req, int sched,
                       int N, PlanPart* q, std::vector<unsigned char>& img) {
  const bool b8 = cls == 1 || cls == 2;
  // panel kernel: tiles of 64 panels (16 per wave), grown in whole rounds;
  // region kernel: tiles of 64 regions (16 per wave); smaller tiles spend
  // more on per-tile set-up and result atomics (16 regions: 5-10% slower),
  // larger ones leave the resident grid's equal shares uneven on batches of
  // ~2800 tiles (128: 15% slower there)
  const int PB = panel_blocks(N);
  const int base = cls == 2 ? (wg / 2) * bpt : cls == 1 ? wg * bpt : cls >= 4 ? 64 : 64 * PB;
  const int unit = cls == 2 ? wg / 2 : cls == 1 ? wg : cls >= 4 ? 4 : 4 * PB;
  q->mode = cls == 3 ? kPanelFloat : kPanelInt8;
  int64_t total = 0;
  for (auto& d : imgs) {
    if (cls >= 4) mfma32_regions(d);
    if (panel_class(cls)) {
      panel_pad_rows(d, PB, N);
      if (cls == 0 && ctx->host[d.tid].max_abs > 127) q->mode = kPanelBigT;
    }
    d.tile0 = static_cast<int32_t>(total);
    d.tile_blocks = image_tile_blocks(d, base, unit);
    d.ntiles = (d.nblocks + d.tile_blocks - 1) / d.tile_blocks;
    total += d.ntiles;
  }
  if (total >= (int64_t{1} << 31)) return fail(RKLT_E_INVAL, "rklt_plan: too many tiles");
  q->cls = cls;
  q->n = static_cast<int>(imgs.size());
  q->total_tiles = total;
  q->wg = b8 ? wg : 256;
  // The matrix-core kernel schedules statically over a resident grid (one
  // workgroup per resident slot); the others take enough workgroups to fill
  // every CU several times over.
  int auto_grid = ctx->cus * (b8 ? 2048 / q->wg : 8);
  if (cls == 2) {
    const int per_cu = mfma8_resident_wgs_per_cu(q->wg);
    if (per_cu > 0) auto_grid = ctx->cus * per_cu;
  }
  if (cls >= 4) {
    // one workgroup per resident slot, each with an equal run of tiles
    const int per_cu = mfma32_resident_wgs_per_cu(cls - 4);
    if (per_cu > 0) auto_grid = ctx->cus * per_cu;
  }
  q->grid = grid_req > 0 ? grid_req : auto_grid;
  if (q->grid > total) q->grid = static_cast<int>(total);

  std::vector<int32_t> tile_img(static_cast<size_t>(total));
  for (size_t k = 0; k < imgs.size(); ++k)
    for (int t = 0; t < imgs[k].ntiles; ++t) tile_img[imgs[k].tile0 + t] = static_cast<int32_t>(k);
  std::vector<int32_t> wg_tiles;
  // round-robin tiles need no ranges; contiguous ones are cost-balanced
  q->strided = cls == 2 && sched == 1;
  q->has_wg_tiles = cls == 2 && q->grid > 0 && !q->strided;
  if (q->has_wg_tiles) {
    // Split the tiles into grid contiguous ranges of (nearly) equal estimated
    // cost: range w ends at the first tile where the running cost reaches
    // (w + 1) / grid of the total.
    std::vector<double> cost(static_cast<size_t>(total));
    double sum = 0;
    for (size_t k = 0; k < imgs.size(); ++k) {
      const double c = mfma8_block_cost(mfma8_path(ctx->host[imgs[k].tid], imgs[k].r), imgs[k].r);
      for (int t = 0; t < imgs[k].ntiles; ++t) {
        const int64_t b0 = static_cast<int64_t>(t) * imgs[k].tile_blocks;
        const int64_t nb = std::min<int64_t>(imgs[k].tile_blocks, imgs[k].nblocks - b0);
        // each image also costs a fixed set-up (operands, ring fill, final
        // reduction): about as much as 150 blocks, measured with batches of
        // thousands of 64 x 64 and 128 x 128 images
        const double c_t = c * static_cast<double>(nb) + (t == 0 ? kMfma8ImageCost : 0.0);
        cost[imgs[k].tile0 + t] = c_t;
        sum += c_t;
      }
    }
    wg_tiles.assign(static_cast<size_t>(q->grid) + 1, static_cast<int32_t>(total));
    wg_tiles[0] = 0;
    double run = 0;
    int w = 1;
    for (int64_t t = 0; t < total && w < q->grid; ++t) {
      run += cost[t];
      while (w < q->grid && run >= sum * w / q->grid) wg_tiles[w++] = static_cast<int32_t>(t + 1);
    }
  }
  auto append = [&img](const void* src, size_t bytes) {
    const size_t off = align256(img.size());
    img.resize(off + bytes);
    if (bytes) std::memcpy(img.data() + off, src, bytes);
    return off;
  };
  q->off_imgs = append(imgs.data(), sizeof(DevImage) * imgs.size());
  q->off_tile_img = append(tile_img.data(), sizeof(int32_t) * tile_img.size());
  q->off_wg_tiles = q->has_wg_tiles ? append(wg_tiles.data(), sizeof(int32_t) * wg_tiles.size()) : 0;
  return RKLT_OK;
}

// Validate `imgs`, group them by kernel class and build the plan's parts and
// the host image of its work list.
rklt_status build_plan(rklt_plan* p, const rklt_image* imgs, int32_t n) {
  rklt_ctx* ctx = p->ctx;
  int wg, bpt, grid_req, sched;
  rklt_status st = check_tuning(p->has_tuning ? &p->tuning : nullptr, &wg, &bpt, &grid_req, &sched);
  if (st) return st;
  std::vector<DevImage> by_class[kClasses];  // indexed by kernel class
  std::vector<DevImage> all;
  int N = 0;
  bool dump = false;
  int64_t pixels = 0;
  {
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (int k = 0; k < n; ++k) {
      DevImage d;
      int Nk = 0;
      if ((st = check_image(ctx, imgs[k], k, &d, &Nk))) return st;
      if (k == 0) N = Nk;
      else if (Nk != N)
        return fail(RKLT_E_INVAL, "image %d: N=%d differs from N=%d of image 0 (one N per plan)", k, Nk, N);
      d.slot = k;
      dump = dump || imgs[k].coef_out || imgs[k].scaled_out;
      pixels += static_cast<int64_t>(imgs[k].H) * imgs[k].W;
      all.push_back(d);
    }
    // a plan that dumps coefficients keeps every image on a dumping kernel
    for (int k = 0; k < n; ++k) {
      const int cls = kernel_class(ctx->host[imgs[k].transform_id], imgs[k].level_shift, dump);
      if (cls == 2) mfma8_pad_rows(all[k]);
      by_class[cls].push_back(all[k]);
    }
  }
  p->images.assign(imgs, imgs + n);
  p->N = N;
  p->dump = dump;
  p->n = n;
  p->pixels = pixels;
  p->nparts = 0;
  p->h_image.clear();
  for (int c : {2, 4, 5, 6, 1, 3, 0}) {
    if (by_class[c].empty()) continue;
    st = build_part(ctx, by_class[c], c, wg, bpt, grid_req, sched, N, &p->parts[p->nparts], p->h_image);
    if (st) return st;
    ++p->nparts;
  }
  // MSSIM tiles of every image with a reconstruction, in slot order
  std::vector<MsImage> ms(static_cast<size_t>(n));
  int64_t ms_total = 0;
  for (int k = 0; k < n; ++k) {
    MsImage& m = ms[k];
    std::memset(&m, 0, sizeof(m));
    m.x = imgs[k].src;
    m.y = imgs[k].dst;
    m.H = imgs[k].H;
    m.W = imgs[k].W;
    m.px = imgs[k].pitch_src;
    m.py = imgs[k].dst ? imgs[k].pitch_dst : 0;
    m.slot = k;
    m.tile0 = static_cast<int32_t>(ms_total);
    if (imgs[k].dst && m.H >= 11 && m.W >= 11) {
      m.across = (m.W - 10 + kMsTileW - 1) / kMsTileW;
      m.ntiles = m.across * ((m.H - 10 + kMsTileH - 1) / kMsTileH);
    }
    ms_total += m.ntiles;
  }
  if (ms_total >= (int64_t{1} << 31)) return fail(RKLT_E_INVAL, "rklt_plan: too many MSSIM tiles");
  p->ms_total = static_cast<int>(ms_total);
  p->off_ms = align256(p->h_image.size());
  p->h_image.resize(p->off_ms + sizeof(MsImage) * ms.size());
  std::memcpy(p->h_image.data() + p->off_ms, ms.data(), sizeof(MsImage) * ms.size());
  p->off_partials = align256(p->h_image.size());
  p->d_need = p->off_partials + sizeof(double) * static_cast<size_t>(ms_total);
  return RKLT_OK;
}

rklt_status ensure_device_capacity(rklt_plan* p) {
  const size_t need = std::max(p->h_image.size(), p->d_need);
  if (need <= p->d_cap) return RKLT_OK;
  (void)hipFree(p->d_buf);
  p->d_buf = nullptr;
  p->d_cap = 0;
  const size_t cap = need + need / 2 + 4096;
  const hipError_t e = hipMalloc(&p->d_buf, cap);
  if (e != hipSuccess) return fail(RKLT_E_NOMEM, "rklt_plan: hipMalloc of %zu bytes: %s", cap, hipGetErrorString(e));
  p->d_cap = cap;
  return RKLT_OK;
}

void destroy_plan(rklt_plan* p) {
  (void)hipFree(p->d_buf);
  if (p->h_pinned) (void)hipHostFree(p->h_pinned);
  delete p;
}

}  // namespace

rklt_status rklt_plan_create(rklt_ctx* ctx, const rklt_image* imgs, int32_t n, const rklt_tuning* tuning,
                             rklt_plan** out) {
  clear_error();
  if (!ctx || !imgs || !out || n < 1) return fail(RKLT_E_INVAL, "rklt_plan_create: NULL argument or n < 1");
  *out = nullptr;
  rklt_plan* p = new (std::nothrow) rklt_plan;
  if (!p) return fail(RKLT_E_NOMEM, "rklt_plan_create: out of host memory");
  p->ctx = ctx;
  if (tuning) {
    p->tuning = *tuning;
    p->has_tuning = true;
  }
  rklt_status st = build_plan(p, imgs, n);
  if (st) {
    destroy_plan(p);
    return st;
  }
  hipError_t e = use_device(ctx->device);
  if (e != hipSuccess) {
    destroy_plan(p);
    return hip_fail("hipSetDevice", e);
  }
  if ((st = ensure_device_capacity(p))) {
    destroy_plan(p);
    return st;
  }
  e = hipMemcpy(p->d_buf, p->h_image.data(), p->h_image.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    destroy_plan(p);
    return hip_fail("rklt_plan_create: hipMemcpy", e);
  }
  *out = p;
  return RKLT_OK;
}

rklt_status rklt_plan_update(rklt_plan* p, const rklt_image* imgs, int32_t n, void* stream) {
  clear_error();
  if (!p) return fail(RKLT_E_INVAL, "rklt_plan_update: plan is NULL");
  if (!imgs || n < 1) {
    p->nparts = 0;
    return fail(RKLT_E_INVAL, "rklt_plan_update: imgs is NULL or n < 1");
  }
  rklt_status st = build_plan(p, imgs, n);
  if (st) {
    p->nparts = 0;  // a failed update leaves an empty plan
    return st;
  }
  hipError_t e = use_device(p->ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  if ((st = ensure_device_capacity(p))) {
    p->nparts = 0;
    return st;
  }
  const size_t need = p->h_image.size();
  if (need > p->h_cap) {
    if (p->h_pinned) (void)hipHostFree(p->h_pinned);
    p->h_pinned = nullptr;
    p->h_cap = 0;
    const size_t cap = need + need / 2 + 4096;
    e = hipHostMalloc(&p->h_pinned, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      p->nparts = 0;
      return fail(RKLT_E_NOMEM, "rklt_plan_update: hipHostMalloc of %zu bytes: %s", cap, hipGetErrorString(e));
    }
    p->h_cap = cap;
  }
  std::memcpy(p->h_pinned, p->h_image.data(), need);
  e = hipMemcpyAsync(p->d_buf, p->h_pinned, need, hipMemcpyHostToDevice, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    p->nparts = 0;
    return hip_fail("rklt_plan_update: hipMemcpyAsync", e);
  }
  return RKLT_OK;
}

rklt_status rklt_plan_autotune(rklt_plan* p, rklt_result* d_res, int32_t reps, void* stream, rklt_tuning* chosen) {
  clear_error();
  if (!p || !d_res) return fail(RKLT_E_INVAL, "rklt_plan_autotune: NULL argument");
  if (reps < 1 || reps > 1000) return fail(RKLT_E_INVAL, "rklt_plan_autotune: reps=%d outside 1..1000", reps);
  if (p->nparts == 0) return fail(RKLT_E_STATE, "rklt_plan_autotune: the plan holds no images");
  hipError_t e = use_device(p->ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const rklt_tuning orig = p->tuning;
  const bool orig_has = p->has_tuning;
  const std::vector<rklt_image> imgs = p->images;
  // re-tile the plan with tuning `t` and upload its work list
  auto apply = [&](const rklt_tuning& t, bool has) -> rklt_status {
    p->tuning = t;
    p->has_tuning = has;
    rklt_status s = build_plan(p, imgs.data(), static_cast<int32_t>(imgs.size()));
    if (!s) s = ensure_device_capacity(p);
    if (!s) {
      const hipError_t he = hipMemcpyAsync(p->d_buf, p->h_image.data(), p->h_image.size(), hipMemcpyHostToDevice, st);
      if (he == hipSuccess) {
        const hipError_t hs = hipStreamSynchronize(st);
        if (hs != hipSuccess) s = hip_fail("rklt_plan_autotune: hipStreamSynchronize", hs);
      } else {
        s = hip_fail("rklt_plan_autotune: hipMemcpyAsync", he);
      }
    }
    if (s) p->nparts = 0;
    return s;
  };
  hipEvent_t ev[2] = {nullptr, nullptr};
  if ((e = hipEventCreate(&ev[0])) != hipSuccess || (e = hipEventCreate(&ev[1])) != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return hip_fail("rklt_plan_autotune: hipEventCreate", e);
  }
  // candidates: workgroup size, blocks per thread (tile size) and the tile
  // schedule of the matrix-core kernel; the grid stays at the resident
  // capacity
  static const int kWg[] = {128, 256};
  static const int kBpt[] = {1, 2, 4, 8};
  rklt_tuning best{};
  float best_ms = -1.0f;
  rklt_status st_out = RKLT_OK;
  for (int cand = 0; cand < 2 * 2 * 4 && !st_out; ++cand) {
    const int sched = cand / 8, wg = kWg[(cand / 4) % 2], bpt = kBpt[cand % 4];
    const rklt_tuning t{wg, bpt, 0, sched};
    if ((st_out = apply(t, true))) break;
    if ((st_out = rklt_plan_run(p, d_res, stream))) break;  // warm-up
    (void)hipEventRecord(ev[0], st);
    for (int k = 0; k < reps && !st_out; ++k) st_out = rklt_plan_run(p, d_res, stream);
    (void)hipEventRecord(ev[1], st);
    if (st_out) break;
    if ((e = hipEventSynchronize(ev[1])) != hipSuccess) {
      st_out = hip_fail("rklt_plan_autotune: hipEventSynchronize", e);
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (st_out) {
    // keep the error message of the failure; restore the original tiling
    char msg[sizeof(g_error)];
    std::memcpy(msg, g_error, sizeof(msg));
    (void)apply(orig, orig_has);
    std::memcpy(g_error, msg, sizeof(msg));
    return st_out;
  }
  rklt_status s = apply(best, true);
  if (s) return s;
  if (chosen) *chosen = best;
  return RKLT_OK;
}

rklt_status rklt_plan_run(rklt_plan* p, rklt_result* d_res, void* stream) {
  clear_error();
  if (!p || !d_res) return fail(RKLT_E_INVAL, "rklt_plan_run: NULL argument");
  if (p->nparts == 0) return fail(RKLT_E_STATE, "rklt_plan_run: the plan holds no images (a failed update)");
  hipError_t e = use_device(p->ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  unsigned char* base = static_cast<unsigned char*>(p->d_buf);
  for (int k = 0; k < p->nparts; ++k) {
    const PlanPart& q = p->parts[k];
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.imgs = reinterpret_cast<const DevImage*>(base + q.off_imgs);
    a.tile_img = reinterpret_cast<const int32_t*>(base + q.off_tile_img);
    a.wg_tiles = q.has_wg_tiles ? reinterpret_cast<const int32_t*>(base + q.off_wg_tiles) : nullptr;
    a.tf = p->ctx->d_table;
    a.res = d_res;
    a.total_tiles = static_cast<int32_t>(q.total_tiles);
    a.dump = p->dump ? 1 : 0;
    a.strided = q.strided ? 1 : 0;
    const rklt_status st = q.cls == 2   ? launch_mfma8(a, q.grid, q.wg, stream)
                           : q.cls == 1 ? launch_block8(a, q.grid, q.wg, stream)
                           : q.cls >= 4 ? launch_mfma32(a, q.grid, q.cls - 4, stream)
                                        : launch_panel(p->N, a, q.grid, q.mode, stream);
    if (st) return st;
  }
  return RKLT_OK;
}

rklt_status rklt_plan_mssim(rklt_plan* p, double* d_mssim, void* stream) {
  clear_error();
  if (!p || !d_mssim) return fail(RKLT_E_INVAL, "rklt_plan_mssim: NULL argument");
  if (p->nparts == 0) return fail(RKLT_E_STATE, "rklt_plan_mssim: the plan holds no images");
  hipError_t e = use_device(p->ctx->device);
  if (e != hipSuccess) return hip_fail("hipSetDevice", e);
  unsigned char* base = static_cast<unsigned char*>(p->d_buf);
  MsArgs a;
  a.imgs = reinterpret_cast<const MsImage*>(base + p->off_ms);
  a.partials = reinterpret_cast<double*>(base + p->off_partials);
  a.out = d_mssim;
  a.n = p->n;
  a.total = p->ms_total;
  const int grid = std::max(1, std::min(p->ms_total, p->ctx->cus * 8));
  return launch_mssim(a, grid, stream);
}

rklt_status rklt_plan_destroy(rklt_plan* p) {
  clear_error();
  if (!p) return fail(RKLT_E_INVAL, "rklt_plan_destroy: plan is NULL");
  (void)use_device(p->ctx->device);
  destroy_plan(p);
  return RKLT_OK;
}

rklt_status rklt_plan_info(const rklt_plan* p, int64_t* tiles, int32_t* grid_wgs, int64_t* pixels) {
  clear_error();
  if (!p) return fail(RKLT_E_INVAL, "rklt_plan_info: plan is NULL");
  int64_t t = 0;
  int32_t g = 0;
  for (int k = 0; k < p->nparts; ++k) {
    t += p->parts[k].total_tiles;
    g += p->parts[k].grid;
  }
  if (tiles) *tiles = t;
  if (grid_wgs) *grid_wgs = g;
  if (pixels) *pixels = p->pixels;
  return RKLT_OK;
}

rklt_status rklt_plan_launches(const rklt_plan* p, int32_t* launches, int32_t* images_per_class) {
  clear_error();
  if (!p) return fail(RKLT_E_INVAL, "rklt_plan_launches: plan is NULL");
  if (launches) *launches = p->nparts;
  if (images_per_class) {
    for (int c = 0; c < kClasses; ++c) images_per_class[c] = 0;
    for (int k = 0; k < p->nparts; ++k) images_per_class[p->parts[k].cls] += p->parts[k].n;
  }
  return RKLT_OK;
}

rklt_status rklt_ctx_transform_exact(rklt_ctx* ctx, int32_t id, int32_t* exact, int64_t* den) {
  clear_error();
  if (!ctx) return fail(RKLT_E_INVAL, "rklt_ctx_transform_exact: ctx is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (id < 0 || id >= static_cast<int>(ctx->host.size()))
    return fail(RKLT_E_INVAL, "rklt_ctx_transform_exact: unknown transform id %d", id);
  if (exact) *exact = ctx->host[id].exact;
  if (den) *den = ctx->host[id].den;
  return RKLT_OK;
}

rklt_status rklt_ctx_mfma_form(rklt_ctx* ctx, int32_t id, int32_t r, int32_t* form) {
  clear_error();
  if (!ctx || !form) return fail(RKLT_E_INVAL, "rklt_ctx_mfma_form: NULL argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (id < 0 || id >= static_cast<int>(ctx->host.size()))
    return fail(RKLT_E_INVAL, "rklt_ctx_mfma_form: unknown transform id %d", id);
  const DevTransform& t = ctx->host[id];
  if (r < 1 || r > t.N * t.N) return fail(RKLT_E_INVAL, "rklt_ctx_mfma_form: r=%d outside 1..%d", r, t.N * t.N);
  *form = t.m_ok ? mfma8_path(t, r) : 0;
  return RKLT_OK;
}

rklt_status rklt_copy_bytes(const void* src, void* dst, size_t nbytes, void* stream) {
  clear_error();
  if (!src || !dst) return fail(RKLT_E_INVAL, "rklt_copy_bytes: NULL pointer");
  if (nbytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
    return fail(RKLT_E_INVAL, "rklt_copy_bytes: pointers and size must be 16-byte aligned");
  return launch_copy(src, dst, nbytes, stream);
}

}  // extern "C"
