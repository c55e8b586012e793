/*
 * rklt.h -- C ABI of the MI355X (gfx950) rounded-KLT block codec.
 *
 * The operation is the JPEG-like compression experiment of Radünz, Bayer and
 * Cintra, "Low-complexity Rounded KLT Approximation for Image Compression"
 * (arXiv 2111.14239):
 *
 *   transform design  (§2.1, §2.2 Eq. 1, §2.3 Eq. 2)
 *     K   the exact KLT of a first-order Markov signal with correlation rho
 *     T   = round(alpha K), round(x) = floor(x + 1/2), element-wise
 *     S   = diag(s), s_i = (T T^T)_ii^(-1/2);  T_hat = S T
 *   codec             (§4.1, Appendix A)
 *     every disjoint N x N sub-block A of an 8-bit image, shifted by ell:
 *       B      = T (A - ell) T^T                  exact integer forward transform
 *       B_hat  = (s s^T) (.) B                    scaling S folded into the zonal stage
 *       keep the first r coefficients of the zig-zag scan, zero the rest
 *       A'     = T_hat^-1 (masked B_hat) T_hat^-T + ell
 *       recon  = clip(floor(A' + 1/2), 0, 255)
 *     per image: SSE = sum (img - recon)^2, MSE = SSE / (H W),
 *                PSNR = 10 log10(255^2 / MSE)  (+inf when MSE = 0)
 *
 * Conventions.  All matrices are row-major.  Row k of K and T is the k-th
 * basis vector.  i (row of B) is the vertical frequency; the zig-zag scan is
 * (0,0), (0,1), (1,0), (2,0), (1,1), (0,2), ...  Integer stages are exact
 * (int32 on the device); scaling, inverse and PSNR run in FP32 on the device;
 * the transform design runs in FP64 on the host.
 *
 * Errors.  Every call returns an rklt_status and never throws.  Argument
 * errors are detected on the host before anything is launched;
 * rklt_last_error() returns a thread-local message describing the most recent
 * failure on the calling thread.
 *
 * Streams.  `stream` arguments are hipStream_t handles passed as void*;
 * NULL is the default stream.  Device calls are asynchronous on that stream;
 * their outputs are valid once the stream has been synchronised.
 */
#ifndef RKLT_H
#define RKLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RKLT_OK = 0,
  RKLT_E_INVAL = 1,    /* an argument is out of range or a pointer is NULL        */
  RKLT_E_SINGULAR = 2, /* the rounded transform has a zero row or det T = 0       */
  RKLT_E_RANGE = 3,    /* the exact integer stages would overflow int32           */
  RKLT_E_NOMEM = 4,    /* a host or device allocation failed                      */
  RKLT_E_HIP = 5,      /* a HIP runtime call or kernel launch failed              */
  RKLT_E_STATE = 6     /* the call does not fit the object's state                */
} rklt_status;

#define RKLT_MAX_N 32

/* flags of rklt_transform */
#define RKLT_ORTHOGONAL 1u /* T T^T is diagonal, so T_hat^-1 = T_hat^T     */
#define RKLT_ADDS_ONLY 2u  /* every entry of T lies in {0, +1, -1}        */

/* One rounded KLT and everything the codec derives from it (host memory). */
typedef struct {
  int32_t N;                           /* block length, 2 <= N <= 32            */
  int32_t flags;                       /* RKLT_ORTHOGONAL | RKLT_ADDS_ONLY      */
  double rho;                          /* correlation coefficient, 0 < rho < 1  */
  double alpha;                        /* expansion factor, alpha > 0           */
  double K[RKLT_MAX_N * RKLT_MAX_N];   /* exact KLT (§2.1), first N*N used      */
  int32_t T[RKLT_MAX_N * RKLT_MAX_N];  /* round(alpha K) (Eq. 2)                */
  int64_t d[RKLT_MAX_N];               /* d_i = (T T^T)_ii                      */
  double s[RKLT_MAX_N];                /* s_i = d_i^(-1/2), S = diag(s) (Eq. 1) */
  double G[RKLT_MAX_N * RKLT_MAX_N];   /* T_hat^-1 = (S T)^-1                   */
  int32_t max_abs;                     /* max |T_ij|                            */
  int32_t max_row_l1;                  /* max_i sum_j |T_ij|                    */
} rklt_transform;

/* One image handed to the codec.  Pointers are device pointers. */
typedef struct {
  const uint8_t* src;   /* H rows of W pixels, row stride pitch_src bytes        */
  uint8_t* dst;         /* reconstruction (same geometry), or NULL: PSNR only    */
  int32_t* coef_out;    /* optional, verification: int32 B, H*W values (NULL     */
                        /* for a float transform)                                */
  float* scaled_out;    /* optional, verification: float B_hat, H*W values      */
  int32_t H, W;         /* multiples of N, 1 <= H, W; (H-1)*pitch + W < 2^31     */
  int32_t pitch_src;    /* >= W, multiple of 8 bytes                             */
  int32_t pitch_dst;    /* >= W, multiple of 8 bytes (ignored when dst is NULL)  */
  int32_t transform_id; /* from rklt_ctx_add_transform                           */
  int32_t r;            /* zig-zag coefficients kept per block, 1 <= r <= N*N    */
  int32_t level_shift;  /* ell, 0 <= ell <= 255 (128 shifts to signed range)     */
  int32_t reserved;     /* must be 0                                             */
} rklt_image;
/* coef_out / scaled_out layout: block-major; block (by, bx) of the image
 * occupies N*N consecutive values starting at (by * (W/N) + bx) * N*N, in
 * row-major (i, j) order.  Both hold every coefficient (not only the kept
 * ones); scaled_out is (s s^T) (.) B before zonal masking.  Writing them adds
 * 4 bytes per pixel each, so they are meant for verification only. */

/* Per-image result (device memory, written by the codec).  `acc` is the
 * codec's own accumulator (tile count above bit 48, running SSE below): the
 * array must be zero-filled once before its first use, and every completed
 * call leaves `acc` at zero again, so the same array can be reused without
 * clearing it.  Calls that share a results array must not overlap. */
typedef struct {
  uint64_t sse;      /* sum of squared pixel errors (exact)                     */
  float mse;         /* sse / (H W) in FP32                                     */
  float psnr_db;     /* 10 log10(255^2 / mse) in FP32, +inf when sse == 0       */
  uint64_t acc;      /* internal: running tile count and SSE of a call          */
  uint32_t tiles;    /* number of tiles the image was coded in (set when final) */
  uint32_t reserved;
} rklt_result;

/* Launch shape of the block kernels.  Zero fields take the defaults. */
typedef struct {
  int32_t wg_threads;        /* threads per workgroup: 64, 128 or 256            */
  int32_t blocks_per_thread; /* N = 8 path: N x N blocks per thread per tile     */
  int32_t grid_wgs;          /* persistent grid size in workgroups (0: auto)     */
  int32_t schedule;          /* batched matrix-core N = 8 kernel: 0 (default) one
                                contiguous, cost-balanced run of tiles per
                                workgroup; 1 tiles dealt round robin (workgroup
                                w codes tiles w, w + grid, ...), so the grid
                                sweeps the batch together; other values E_INVAL */
} rklt_tuning;

typedef struct rklt_ctx rklt_ctx;
typedef struct rklt_plan rklt_plan;

/* Thread-local message of the last failure on this thread ("" if none). */
const char* rklt_last_error(void);

/* ---- host-side transform design (no GPU needed) ------------------------- */

/* Build T = round(alpha K_rho) for block length N and everything derived
 * from it: the omega roots of §2.1 (one in each (k pi/N, (k+1) pi/N)), the
 * eigenvalues lambda_k, K, T (Eq. 2), d, s and S (Eq. 1), and G = T_hat^-1.
 * `out` is caller-owned.  Errors: E_INVAL (N outside 2..32, rho outside
 * (0,1), alpha not positive and finite, out NULL); E_SINGULAR (a zero row of
 * T or a singular T, e.g. alpha = 1 at N = 8, where every |K_ij| < 1/2). */
rklt_status rklt_build_transform(int32_t N, double rho, double alpha, rklt_transform* out);

/* The zig-zag scan of §4.1 for an N x N block: order[k] = i*N + j of the
 * k-th scanned coefficient, k = 0 .. N*N-1.  `order` holds N*N int32 values
 * (caller-owned).  Errors: E_INVAL (N outside 1..32, order NULL). */
rklt_status rklt_zigzag(int32_t N, int32_t* order);

/* The paper's float comparison transforms (§4.1, Table 3), FP64, N x N
 * row-major, row k the k-th basis vector; caller-owned output.
 * rklt_klt_matrix: the exact KLT K_rho of §2.1 (the same K that
 *   rklt_build_transform returns, for any rho in (0, 1)).
 * rklt_dct_matrix: the orthonormal DCT-II, C[k][n] = c_k cos(pi (2n+1) k / (2N)),
 *   c_0 = sqrt(1/N), c_k = sqrt(2/N) for k > 0.
 * Errors: E_INVAL (N outside 2..32, rho outside (0, 1), NULL output). */
rklt_status rklt_klt_matrix(int32_t N, double rho, double* K);
rklt_status rklt_dct_matrix(int32_t N, double* C);

/* ---- host-side design tools (§3, §3.1; no GPU needed) ------------------- */

/* Figures of merit of an N x N transform T_hat (FP64, row-major, rows the
 * basis vectors), for the unit-variance first-order Markov model of
 * correlation rho, R_ij = rho^|i-j|:
 *   coding_gain_db     unified coding gain (§3.1.1), -(10/N) sum_k
 *                      log10(A_k B_k), A_k = h_k R h_k^T (h_k row k of
 *                      T_hat), B_k = squared norm of row k of T_hat^-1;
 *   coding_gain_tt_db  the same with T_hat^T in place of T_hat^-1 (equal for
 *                      an orthonormal T_hat; the reading under which the
 *                      paper's Table 2 values of its non-orthogonal matrices
 *                      are reproduced);
 *   efficiency_pct     transform efficiency (§3.1.2), 100 sum_i |r_ii| /
 *                      sum_ij |r_ij|, r = T_hat R T_hat^T;
 *   mse                (1/N) tr(D R D^T), D = ref - T_hat (§3.1.3);
 *   error_energy       pi ||D||_F^2 (§3.1.4).
 * `ref` is the matrix T_hat is compared with (K_rho in Table 2, the DCT for
 * the RDCT).  Errors: E_INVAL (NULL, N outside 2..32, rho outside (0, 1), a
 * non-finite entry), E_SINGULAR (T_hat singular). */
typedef struct {
  double coding_gain_db;
  double coding_gain_tt_db;
  double efficiency_pct;
  double mse;
  double error_energy;
} rklt_measures;
rklt_status rklt_transform_measures(int32_t N, const double* That, const double* ref, double rho,
                                    rklt_measures* out);

/* Algorithm 1 (§3): sweep rho over step, 2 step, ... (the grid points below
 * 1) and record every T' = round(alpha K_rho) (round(x) = floor(x + 1/2))
 * that differs from the previous one, starting from the zero matrix.  Entry
 * k holds the first and last grid rho that gave it and T' (N x N in the first
 * N*N entries of T).  At most `cap` entries are written to `out`
 * (caller-owned); *count receives the total, so a call with cap = 0 sizes
 * the array.  Errors: E_INVAL (count NULL, out NULL with cap > 0, N outside
 * 2..32, alpha not positive and finite, step outside (0, 1/2) or finer than
 * 1e-6), E_RANGE (entries beyond 1e6). */
typedef struct {
  double rho_first;
  double rho_last;
  int32_t T[RKLT_MAX_N * RKLT_MAX_N];
} rklt_design_entry;
rklt_status rklt_algorithm1(int32_t N, double alpha, double step, rklt_design_entry* out, int32_t cap,
                            int32_t* count);

/* ---- device context ----------------------------------------------------- */

/* Create a context on HIP device `device`.  The context owns a device-side
 * table of up to 256 transforms; it allocates nothing else. */
rklt_status rklt_ctx_create(int32_t device, rklt_ctx** out);
rklt_status rklt_ctx_destroy(rklt_ctx* ctx);

/* Upload a transform built by rklt_build_transform (N must be 4, 8, 16 or
 * 32) into the context's table and return its id.  A transform whose T
 * equals one already uploaded returns the existing id.  The copy is
 * synchronous; it never touches entries that launched kernels may read.
 * Errors: E_INVAL, E_RANGE (255 * max_row_l1^2 >= 2^31), E_NOMEM (table
 * full), E_HIP. */
rklt_status rklt_ctx_add_transform(rklt_ctx* ctx, const rklt_transform* t, int32_t* id_out);

/* Upload a float transform M (N x N, FP64, row-major, row k the k-th basis
 * vector; N in {4, 8, 16, 32}) for the comparison arms of §4.1 / Table 3:
 * images coded with it take B = M (A - ell) M^T, keep the first r zig-zag
 * coefficients (no scaling stage), and reconstruct A' = M^-1 B M^-T + ell,
 * pixel = clip(floor(A' + 1/2), 0, 255).  M^-1 is computed on the host in
 * FP64 (for an orthonormal M it is M^T up to rounding); the device stores M
 * and M^-1 in FP32 (panel kernel, for images with a dump) and as two fp16
 * parts (region matrix-core kernel: fp16 products, FP32 sums, 22-bit
 * operands), so a pixel may differ by one level from the FP64 result where
 * that result lies within about 1e-3 (N = 8) of a rounding tie.  An identical M returns the existing
 * id.  Images of a float transform take no coef_out; scaled_out receives the
 * FP32 coefficients B.  Errors: E_INVAL (NULL argument, N, an entry not
 * finite or beyond 1e6), E_SINGULAR (M singular), E_NOMEM (table full),
 * E_HIP. */
rklt_status rklt_ctx_add_float_transform(rklt_ctx* ctx, int32_t N, const double* M, int32_t* id_out);

/* JPEG-style quantisation with the scaling matrix folded into the
 * quantiser (Appendix A): returns a new id naming rounded transform
 * `transform_id` together with the quantisation matrix Q (N x N, FP64,
 * row-major, entries in (0, 1e6]).  Images coded with that id keep the first
 * r zig-zag coefficients as usual (r = N*N keeps all) and replace their
 * scaling by the quantiser:
 *   code    c_ij = floor(t + 1/2),  t = fl32(B_ij * q_ij),
 *           q_ij = fl32(s_i s_j / Q_ij) (computed in FP64 on the host): the
 *           reciprocal of Q~ = Q / (s s^T), so B / Q~ = (T_hat A T_hat^T) / Q;
 *   dequantised scaled coefficient Q_ij c_ij (FP32), then the usual inverse
 *   A' = T_hat^-1 (Q (.) c) T_hat^-T + ell in FP32 and pixel rounding.
 * The codes are exact functions of the integer B (the same FP32 steps on any
 * IEEE machine).
 * scaled_out receives Q_ij c_ij for every coefficient (the quantiser's
 * output before the zonal mask), coef_out the integer B.  An identical (T, Q) returns the existing id.  Errors: E_INVAL
 * (NULL argument, unknown id, a float or already quantised transform, an
 * entry of Q outside (0, 1e6] or NaN), E_NOMEM (table full), E_HIP. */
rklt_status rklt_ctx_add_quantizer(rklt_ctx* ctx, int32_t transform_id, const double* Q, int32_t* id_out);

/* Whether the N = 8 register kernel reconstructs transform `id` exactly:
 * T^-1 = adj / den with integer adj small enough that every step of the
 * inverse is exact, so reconstructed pixels equal floor(x + 1/2) of the exact
 * rational x (ties included).  Otherwise (*exact = 0, *den = 0) the inverse
 * runs in FP32 and a pixel may differ by one level where x is within about
 * 1e-3 of a rounding tie.  Errors: E_INVAL (NULL ctx, unknown id). */
rklt_status rklt_ctx_transform_exact(rklt_ctx* ctx, int32_t id, int32_t* exact, int64_t* den);

/* Inverse form the N = 8 matrix-core kernel (level shift 128, the batched
 * path's usual kernel) uses for transform `id` with r kept coefficients:
 *   *form = 1  exact, one fp16 pass (every partial sum below 2^24);
 *           3  exact, fp16 with separate accumulators for the high and low
 *              parts of each coefficient;
 *           2  FP32 (no exact inverse, or its bounds do not hold): a pixel may
 *              differ by one level where x is within about 1e-3 of a tie;
 *           0  the transform does not run on the matrix-core kernel.
 * Exact forms give floor(x + 1/2) of the exact rational x, ties included.
 * Errors: E_INVAL (NULL ctx or form, unknown id, r outside 1..N*N). */
rklt_status rklt_ctx_mfma_form(rklt_ctx* ctx, int32_t id, int32_t r, int32_t* form);

/* ---- codec -------------------------------------------------------------- */

/* Plain path: code one image with one kernel launch on `stream` (§4.1).
 * `d_res` is one device rklt_result (see its zero-fill rule).  Errors:
 * E_INVAL (geometry, r, ell, pointers, unknown transform id), E_HIP. */
rklt_status rklt_codec(rklt_ctx* ctx, const rklt_image* img, rklt_result* d_res,
                       const rklt_tuning* tuning, void* stream);

/* Batched path: a plan holds the work list of `n` images (host array of
 * descriptors with device pointers) on the device: per image its tile range
 * and parameters, and a tile -> image table, so that rklt_plan_run codes the
 * whole batch in one persistent launch.  All images of a plan share N.
 * Creating a plan validates every image (the first bad one is named in
 * rklt_last_error), allocates and uploads the work list synchronously.
 * `tuning` NULL takes the defaults.  A plan must not run concurrently with
 * itself; different plans may run on different streams. */
rklt_status rklt_plan_create(rklt_ctx* ctx, const rklt_image* imgs, int32_t n,
                             const rklt_tuning* tuning, rklt_plan** out);
/* d_res: n device rklt_result, in the order of the plan's images. */
rklt_status rklt_plan_run(rklt_plan* plan, rklt_result* d_res, void* stream);
/* Tile-shape autotuning of the batched launch (a persistent grid over
 * uneven images; the tile shape and blocks per workgroup decide balance and
 * per-tile overhead): re-tiles the plan for each candidate tuning
 * (wg_threads in {128, 256} x blocks_per_thread in {1, 2, 4, 8} x schedule
 * in {0, 1}, grid at the resident capacity), times `reps` runs of each on `stream` with HIP events
 * after one warm-up run, and keeps the fastest.  The runs code the plan's
 * images for real: dst and d_res hold a complete, valid result afterwards.
 * Synchronous (waits for the timing runs).  `chosen` (may be NULL) receives
 * the tuning kept.  Errors: E_INVAL (NULL plan or d_res, reps outside
 * 1..1000), E_STATE (empty plan), E_HIP; after an error the plan keeps its
 * previous tuning (or holds no images if re-tiling failed). */
rklt_status rklt_plan_autotune(rklt_plan* plan, rklt_result* d_res, int32_t reps, void* stream,
                               rklt_tuning* chosen);
/* Mean structural similarity of every image's reconstruction against its
 * source, the paper's third quality measure (§4.1, the SSIM of Wang et al.
 * 2004): an 11 x 11 Gaussian window with standard deviation 1.5, C1 =
 * (0.01 * 255)^2, C2 = (0.03 * 255)^2, evaluated at every window position
 * inside the image and averaged.  Reads src and dst of the plan's images, so
 * it belongs after rklt_plan_run on the same stream.  d_mssim: n device
 * doubles in the order of the plan's images; NaN for an image without a
 * reconstruction or with a side below 11.  FP32 window sums, double
 * accumulation in a fixed order (deterministic).  Two launches; no
 * allocation (the per-tile sums live in the plan's device buffer).
 * Errors: E_INVAL (NULL plan or d_mssim), E_STATE (empty plan), E_HIP. */
rklt_status rklt_plan_mssim(rklt_plan* plan, double* d_mssim, void* stream);
/* Replace the plan's images with `n` new ones (same rules as
 * rklt_plan_create; the tuning given at creation is kept) without a
 * synchronous copy: the work list is rebuilt on the host and uploaded with an
 * asynchronous copy on `stream`, from pinned host memory the plan owns, into
 * the plan's device buffer (grown only when it is too small).  The plan must
 * not be in flight: its previous run (and update) must have completed, e.g.
 * observed through an event recorded after the run.  A run on `stream` after
 * the update sees the new images.  On error the plan holds no images and
 * rklt_plan_run fails with E_STATE until a successful update. */
rklt_status rklt_plan_update(rklt_plan* plan, const rklt_image* imgs, int32_t n, void* stream);
rklt_status rklt_plan_destroy(rklt_plan* plan);
/* Number of tiles and of workgroups the plan launches (for reporting). */
rklt_status rklt_plan_info(const rklt_plan* plan, int64_t* tiles, int32_t* grid_wgs,
                           int64_t* pixels);
/* A plan launches one kernel per kernel class among its images:
 *   class 2  the N = 8 matrix-core kernel: level shift 128 and a transform
 *            whose exact inverse fits its operands (every {0, +-1} T of
 *            alpha in {2, 3} but one);
 *   class 1  the N = 8 register kernel: level shift 128, |T_ij| <= 127,
 *            128 * max row L1 <= 32767 (also every plan that dumps coefficients);
 *   class 0  the panel kernel (any N, any level shift): every other rounded
 *            or quantised transform;
 *   class 3  the panel kernel in FP32: float transforms with a dump;
 *   class 4  the region matrix-core kernel (32 x 32 pixel regions, any N):
 *            the rounded transforms the classes above do not take, with
 *            |T_ij| <= 127 and 128 L1 + |128 - ell| max_j |sum_n T_jn| <=
 *            32640, no coefficient dump;
 *   class 5  the region kernel for quantised entries (same bounds);
 *   class 6  the region kernel for float transforms (no coefficient dump).
 * Reports the number of launches per run and, in images_per_class[7] (may be
 * NULL), how many images each class codes. */
rklt_status rklt_plan_launches(const rklt_plan* plan, int32_t* launches, int32_t* images_per_class);

/* ---- measurement -------------------------------------------------------- */

/* Copy nbytes from src to dst (device pointers, 16-byte aligned, nbytes a
 * multiple of 16) with a plain streaming kernel: the bandwidth reference the
 * codec's HBM traffic is compared with.  Errors: E_INVAL, E_HIP. */
rklt_status rklt_copy_bytes(const void* src, void* dst, size_t nbytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RKLT_H */
