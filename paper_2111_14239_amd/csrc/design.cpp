// Host-side design tools (FP64, no HIP): the figures of merit of §3.1 and
// the sweep of Algorithm 1 (§3) that derives the set of distinct rounded KLT
// matrices over a grid of correlation coefficients.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "rklt.h"
#include "rklt_internal.h"

namespace rklt {

namespace {

// R_ij = rho^|i - j|: covariance of the unit-variance first-order Markov
// signal (§2.1).
void markov_covariance(int N, double rho, double* R) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) R[i * N + j] = std::pow(rho, std::abs(i - j));
}

}  // namespace

rklt_status transform_measures(int N, const double* That, const double* ref, double rho, rklt_measures* out) {
  if (!That || !ref || !out) return fail(RKLT_E_INVAL, "rklt_transform_measures: NULL argument");
  if (N < 2 || N > RKLT_MAX_N)
    return fail(RKLT_E_INVAL, "rklt_transform_measures: N=%d outside 2..%d", N, RKLT_MAX_N);
  if (!(rho > 0.0 && rho < 1.0))
    return fail(RKLT_E_INVAL, "rklt_transform_measures: rho=%g outside (0, 1)", rho);
  for (int k = 0; k < N * N; ++k)
    if (!std::isfinite(That[k]) || !std::isfinite(ref[k]))
      return fail(RKLT_E_INVAL, "rklt_transform_measures: entry %d is not finite", k);
  double R[RKLT_MAX_N * RKLT_MAX_N], G[RKLT_MAX_N * RKLT_MAX_N], C[RKLT_MAX_N * RKLT_MAX_N];
  markov_covariance(N, rho, R);
  if (!invert_matrix(N, That, G)) return fail(RKLT_E_SINGULAR, "rklt_transform_measures: T_hat is singular");

  // §3.1.1 unified coding gain: Cg = -(10/N) sum_k log10(A_k B_k) with
  // A_k = h_k R h_k^T (h_k row k of T_hat) and B_k the squared norm of row k
  // of the inverse (of T_hat^-1, or of T_hat^T for the second figure).
  double cg = 0.0, cg_t = 0.0;
  for (int k = 0; k < N; ++k) {
    double A = 0.0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) A += That[k * N + i] * R[i * N + j] * That[k * N + j];
    double Bi = 0.0, Bt = 0.0;
    for (int i = 0; i < N; ++i) {
      Bi += G[k * N + i] * G[k * N + i];
      Bt += That[i * N + k] * That[i * N + k];
    }
    cg += std::log10(A * Bi);
    cg_t += std::log10(A * Bt);
  }
  out->coding_gain_db = -10.0 * cg / N;
  out->coding_gain_tt_db = -10.0 * cg_t / N;

  // §3.1.2 transform efficiency of r = T_hat R T_hat^T
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double v = 0.0;
      for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) v += That[i * N + a] * R[a * N + b] * That[j * N + b];
      C[i * N + j] = v;
    }
  double diag = 0.0, all = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      all += std::fabs(C[i * N + j]);
      if (i == j) diag += std::fabs(C[i * N + j]);
    }
  out->efficiency_pct = 100.0 * diag / all;

  // §3.1.3 MSE = (1/N) tr(D R D^T) and §3.1.4 epsilon = pi ||D||_F^2, D = ref - T_hat
  double tr = 0.0, fro = 0.0;
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < N; ++i) {
      const double di = ref[k * N + i] - That[k * N + i];
      fro += di * di;
      for (int j = 0; j < N; ++j) tr += di * R[i * N + j] * (ref[k * N + j] - That[k * N + j]);
    }
  out->mse = tr / N;
  out->error_energy = M_PI * fro;
  return RKLT_OK;
}

rklt_status algorithm1(int N, double alpha, double step, rklt_design_entry* out, int cap, int* count) {
  if (!count || cap < 0 || (cap > 0 && !out)) return fail(RKLT_E_INVAL, "rklt_algorithm1: bad output arguments");
  if (N < 2 || N > RKLT_MAX_N) return fail(RKLT_E_INVAL, "rklt_algorithm1: N=%d outside 2..%d", N, RKLT_MAX_N);
  if (!(alpha > 0.0) || !std::isfinite(alpha))
    return fail(RKLT_E_INVAL, "rklt_algorithm1: alpha=%g is not positive and finite", alpha);
  if (!(step > 0.0 && step < 0.5)) return fail(RKLT_E_INVAL, "rklt_algorithm1: step=%g outside (0, 1/2)", step);
  const long long steps = std::llround(1.0 / step) - 1;  // rho = step, 2 step, ..., below 1
  if (steps > 1000000) return fail(RKLT_E_INVAL, "rklt_algorithm1: step=%g gives too many grid points", step);
  int32_t prev[RKLT_MAX_N * RKLT_MAX_N], cur[RKLT_MAX_N * RKLT_MAX_N];
  std::memset(prev, 0, sizeof(prev));  // the sweep starts from the zero matrix
  double K[RKLT_MAX_N * RKLT_MAX_N];
  int n = 0;
  for (long long g = 1; g <= steps; ++g) {
    const double rho = static_cast<double>(g) * step;
    rklt_status st = klt_matrix(N, rho, K);
    if (st) return st;
    for (int k = 0; k < N * N; ++k) {
      const double v = std::floor(alpha * K[k] + 0.5);
      if (std::fabs(v) > 1e6) return fail(RKLT_E_RANGE, "rklt_algorithm1: alpha=%g gives entries beyond 1e6", alpha);
      cur[k] = static_cast<int32_t>(v);
    }
    if (std::memcmp(cur, prev, sizeof(int32_t) * N * N) != 0) {
      if (n < cap) {
        std::memset(&out[n], 0, sizeof(out[n]));
        out[n].rho_first = rho;
        out[n].rho_last = rho;
        std::memcpy(out[n].T, cur, sizeof(int32_t) * N * N);
      }
      ++n;
      std::memcpy(prev, cur, sizeof(int32_t) * N * N);
    } else if (n > 0 && n <= cap) {
      out[n - 1].rho_last = rho;
    }
  }
  *count = n;
  return RKLT_OK;
}

}  // namespace rklt
