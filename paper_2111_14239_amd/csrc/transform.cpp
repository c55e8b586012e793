// Host-side design of the rounded KLT (FP64): §2.1 (KLT of a first-order
// Markov signal), §2.2 Eq. (1) (scaling S), §2.3 Eq. (2) (T = round(alpha K))
// and the zig-zag scan of §4.1.  Pure C++; no HIP.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "rklt.h"
#include "rklt_internal.h"

namespace rklt {

namespace {

// Root function of the §2.1 frequency equation
//   tan(N w) = -(1 - rho^2) sin w / ((1 + rho^2) cos w - 2 rho)
// with both denominators multiplied out, and its derivative in w.
struct FreqEq {
  int N;
  double a, b;  // a = 1 + rho^2, b = 1 - rho^2
  double rho;
  double f(double w) const {
    return std::sin(N * w) * (a * std::cos(w) - 2.0 * rho) + b * std::sin(w) * std::cos(N * w);
  }
  double df(double w) const {
    const double sN = std::sin(N * w), cN = std::cos(N * w);
    const double s1 = std::sin(w), c1 = std::cos(w);
    return N * cN * (a * c1 - 2.0 * rho) - sN * a * s1 + b * (c1 * cN - N * s1 * sN);
  }
};

// Safeguarded Newton iteration on [lo, hi], where f changes sign: a Newton
// step is taken when it stays inside the current bracket, a bisection step
// otherwise; the bracket shrinks every iteration.
double solve_bracketed(const FreqEq& eq, double lo, double hi) {
  double flo = eq.f(lo);
  double fhi = eq.f(hi);
  if (flo == 0.0) return lo;
  if (fhi == 0.0) return hi;
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double fx = eq.f(x);
    if (fx == 0.0) return x;
    if ((fx < 0.0) == (flo < 0.0)) {
      lo = x;
      flo = fx;
    } else {
      hi = x;
    }
    if (hi - lo <= 4e-16 * std::fabs(hi)) break;
    const double dfx = eq.df(x);
    double nx = (dfx != 0.0) ? x - fx / dfx : lo - 1.0;
    if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
    if (nx == x) break;
    x = nx;
  }
  return x;
}

}  // namespace

// Gauss-Jordan inverse with partial pivoting, FP64.  Returns false when a
// pivot is negligible against the row scale (singular matrix).
bool invert_matrix(int n, const double* A, double* inv) {
  double M[RKLT_MAX_N][2 * RKLT_MAX_N];
  double scale = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      M[i][j] = A[i * n + j];
      M[i][n + j] = (i == j) ? 1.0 : 0.0;
      scale = std::fmax(scale, std::fabs(A[i * n + j]));
    }
  }
  if (scale == 0.0) return false;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(M[i][c]) > std::fabs(M[p][c])) p = i;
    if (std::fabs(M[p][c]) <= 1e-10 * scale) return false;
    if (p != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(M[p][j], M[c][j]);
    const double piv = M[c][c];
    for (int j = 0; j < 2 * n; ++j) M[c][j] /= piv;
    for (int i = 0; i < n; ++i) {
      if (i == c || M[i][c] == 0.0) continue;
      const double f = M[i][c];
      for (int j = 0; j < 2 * n; ++j) M[i][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = M[i][n + j];
  return true;
}

rklt_status klt_matrix(int N, double rho, double* K) {
  if (!K) return fail(RKLT_E_INVAL, "rklt_klt_matrix: K is NULL");
  if (N < 2 || N > RKLT_MAX_N) return fail(RKLT_E_INVAL, "rklt_klt_matrix: N=%d outside 2..%d", N, RKLT_MAX_N);
  if (!(rho > 0.0 && rho < 1.0)) return fail(RKLT_E_INVAL, "rklt_klt_matrix: rho=%g outside (0, 1)", rho);
  // §2.1: one frequency in each open interval (k pi / N, (k+1) pi / N).
  // w = 0 and w = pi are trivial zeros of the cleared equation, so the two
  // outer brackets start a little way inside.
  const FreqEq eq{N, 1.0 + rho * rho, 1.0 - rho * rho, rho};
  double omega[RKLT_MAX_N], lambda[RKLT_MAX_N];
  const double step = M_PI / N;
  for (int k = 0; k < N; ++k) {
    double lo = k * step, hi = (k + 1) * step;
    if (k == 0) lo += 1e-7 * step;
    if (k == N - 1) hi -= 1e-7 * step;
    omega[k] = solve_bracketed(eq, lo, hi);
    lambda[k] = (1.0 - rho * rho) / (1.0 + rho * rho - 2.0 * rho * std::cos(omega[k]));
  }
  // §2.1: basis vector k sampled at n (row k of K), with the frequency and the
  // phase indexed by the basis index k.
  for (int k = 0; k < N; ++k) {
    const double amp = std::sqrt(2.0 / (N + lambda[k]));
    for (int n = 0; n < N; ++n) K[k * N + n] = amp * std::sin(omega[k] * (n - 0.5 * (N - 1)) + 0.5 * (k + 1) * M_PI);
  }
  return RKLT_OK;
}

rklt_status dct_matrix(int N, double* C) {
  if (!C) return fail(RKLT_E_INVAL, "rklt_dct_matrix: C is NULL");
  if (N < 2 || N > RKLT_MAX_N) return fail(RKLT_E_INVAL, "rklt_dct_matrix: N=%d outside 2..%d", N, RKLT_MAX_N);
  // orthonormal DCT-II: row k is c_k cos(pi (2n + 1) k / (2N)), c_0 = sqrt(1/N),
  // c_k = sqrt(2/N) otherwise
  for (int k = 0; k < N; ++k) {
    const double c = std::sqrt((k == 0 ? 1.0 : 2.0) / N);
    for (int n = 0; n < N; ++n) C[k * N + n] = c * std::cos(M_PI * (2 * n + 1) * k / (2.0 * N));
  }
  return RKLT_OK;
}

rklt_status build_transform(int N, double rho, double alpha, rklt_transform* out) {
  if (!out) return fail(RKLT_E_INVAL, "rklt_build_transform: out is NULL");
  if (N < 2 || N > RKLT_MAX_N)
    return fail(RKLT_E_INVAL, "rklt_build_transform: N=%d outside 2..%d", N, RKLT_MAX_N);
  if (!(rho > 0.0 && rho < 1.0))
    return fail(RKLT_E_INVAL, "rklt_build_transform: rho=%g outside (0, 1)", rho);
  if (!(alpha > 0.0) || !std::isfinite(alpha))
    return fail(RKLT_E_INVAL, "rklt_build_transform: alpha=%g is not positive and finite", alpha);

  std::memset(out, 0, sizeof(*out));
  out->N = N;
  out->rho = rho;
  out->alpha = alpha;

  rklt_status st = klt_matrix(N, rho, out->K);
  if (st) return st;

  // Eq. (2): T = round(alpha K), round(x) = floor(x + 1/2).
  int max_abs = 0, max_l1 = 0;
  bool adds_only = true;
  for (int i = 0; i < N; ++i) {
    int l1 = 0;
    for (int j = 0; j < N; ++j) {
      const double v = std::floor(alpha * out->K[i * N + j] + 0.5);
      if (std::fabs(v) > 1e6)
        return fail(RKLT_E_RANGE, "rklt_build_transform: alpha=%g gives entries beyond 1e6", alpha);
      const int t = static_cast<int>(v);
      out->T[i * N + j] = t;
      const int a = t < 0 ? -t : t;
      max_abs = a > max_abs ? a : max_abs;
      l1 += a;
      if (a > 1) adds_only = false;
    }
    max_l1 = l1 > max_l1 ? l1 : max_l1;
  }
  out->max_abs = max_abs;
  out->max_row_l1 = max_l1;

  // Eq. (1): d = diag(T T^T), s = d^(-1/2).  T T^T diagonal <=> orthogonal rows.
  bool orthogonal = true;
  for (int i = 0; i < N; ++i) {
    for (int k = 0; k < N; ++k) {
      int64_t dot = 0;
      for (int j = 0; j < N; ++j)
        dot += static_cast<int64_t>(out->T[i * N + j]) * out->T[k * N + j];
      if (i == k) out->d[i] = dot;
      else if (dot != 0) orthogonal = false;
    }
    if (out->d[i] == 0)
      return fail(RKLT_E_SINGULAR,
                  "rklt_build_transform: row %d of round(alpha K) is zero (N=%d rho=%g alpha=%g)", i,
                  N, rho, alpha);
    out->s[i] = 1.0 / std::sqrt(static_cast<double>(out->d[i]));
  }
  out->flags = (orthogonal ? RKLT_ORTHOGONAL : 0u) | (adds_only ? RKLT_ADDS_ONLY : 0u);

  // G = T_hat^-1 with T_hat = S T.
  double That[RKLT_MAX_N * RKLT_MAX_N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) That[i * N + j] = out->s[i] * out->T[i * N + j];
  if (!invert_matrix(N, That, out->G))
    return fail(RKLT_E_SINGULAR, "rklt_build_transform: round(alpha K) is singular (N=%d rho=%g alpha=%g)",
                N, rho, alpha);
  return RKLT_OK;
}

bool exact_inverse(int N, const int32_t* T, int64_t* adj, int64_t* den) {
  // Fraction-free Gauss-Jordan elimination of [T | I] over the integers: each
  // update (p_k M_ij - M_ik M_kj) / p_{k-1} divides exactly, the left block
  // ends as D I with D = +-det T and the right block as the matching
  // adjugate, so T^-1 = right / D.  The result is reduced to lowest terms
  // and checked (T adj = den I) before it is returned.
  typedef __int128 i128;
  if (N < 1 || N > 8) return false;
  i128 M[8][16];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      if (T[i * N + j] > 8 || T[i * N + j] < -8) return false;  // keeps every product in range
      M[i][j] = T[i * N + j];
      M[i][N + j] = (i == j) ? 1 : 0;
    }
  i128 prev = 1;
  for (int k = 0; k < N; ++k) {
    int p = k;
    while (p < N && M[p][k] == 0) ++p;
    if (p == N) return false;
    if (p != k)
      for (int j = 0; j < 2 * N; ++j) std::swap(M[p][j], M[k][j]);
    for (int i = 0; i < N; ++i) {
      if (i == k) continue;
      const i128 f = M[i][k];
      for (int j = 0; j < 2 * N; ++j) {
        const i128 num = M[k][k] * M[i][j] - f * M[k][j];
        if (num % prev != 0) return false;
        M[i][j] = num / prev;
      }
    }
    prev = M[k][k];
  }
  i128 D = M[N - 1][N - 1];
  for (int i = 0; i < N; ++i)
    if (M[i][i] != D) return false;
  i128 g = D < 0 ? -D : D;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      i128 a = M[i][N + j] < 0 ? -M[i][N + j] : M[i][N + j];
      while (a != 0) {
        const i128 t = g % a;
        g = a;
        a = t;
      }
    }
  if (g == 0) return false;
  const int sign = D < 0 ? -1 : 1;
  *den = static_cast<int64_t>(sign * D / g);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) adj[i * N + j] = static_cast<int64_t>(sign * M[i][N + j] / g);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      i128 acc = 0;
      for (int k = 0; k < N; ++k) acc += static_cast<i128>(T[i * N + k]) * adj[k * N + j];
      if (acc != ((i == j) ? static_cast<i128>(*den) : 0)) return false;
    }
  return true;
}

rklt_status zigzag(int N, int32_t* order) {
  if (!order) return fail(RKLT_E_INVAL, "rklt_zigzag: order is NULL");
  if (N < 1 || N > RKLT_MAX_N) return fail(RKLT_E_INVAL, "rklt_zigzag: N=%d outside 1..%d", N, RKLT_MAX_N);
  // Walk the anti-diagonals i + j = t in turn.  On odd t the scan moves
  // down-left (row i rising), on even t up-right (row i falling); this starts
  // (0,0) -> (0,1) -> (1,0) -> (2,0) as in JPEG.
  int k = 0;
  for (int t = 0; t <= 2 * (N - 1); ++t) {
    const int ilo = t < N ? 0 : t - (N - 1);
    const int ihi = t < N ? t : N - 1;
    if (t & 1) {
      for (int i = ilo; i <= ihi; ++i) order[k++] = i * N + (t - i);
    } else {
      for (int i = ihi; i >= ilo; --i) order[k++] = i * N + (t - i);
    }
  }
  return RKLT_OK;
}

}  // namespace rklt
