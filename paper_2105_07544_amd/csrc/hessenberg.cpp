// Host-side dense helpers of the polynomial setup: eigenvalues of a small
// upper Hessenberg matrix by the Francis double-shift QR iteration
// (Golub & Van Loan, Matrix Computations, Alg. 7.5.1/7.5.2: implicit
// double-shift step with 3x3 Householder reflectors, deflation on negligible
// subdiagonal entries, an ad hoc shift every tenth step of a stalled block),
// and the modified Leja ordering of the resulting roots.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/gmres_ir.h"
#include "host_common.hpp"

namespace {

// Apply the reflector I - 2 v v^T / (v^T v) (v of length `len`) from the left to
// rows r0.. r0+len-1, columns c0..c1, and from the right to columns r0.., rows
// q0..q1 of the row-major matrix A (n x n).
struct Reflector {
  double v[3];
  double beta;  // 2 / (v^T v), 0 for the identity
  int len;
};

Reflector make_reflector(const double* x, int len) {
  Reflector R;
  R.len = len;
  double nrm2 = 0.0;
  for (int i = 0; i < len; ++i) nrm2 += x[i] * x[i];
  const double nrm = sqrt(nrm2);
  if (nrm == 0.0) {
    R.beta = 0.0;
    for (int i = 0; i < 3; ++i) R.v[i] = 0.0;
    return R;
  }
  const double alpha = (x[0] >= 0.0) ? -nrm : nrm;  // x -> alpha e1 without cancellation
  for (int i = 0; i < len; ++i) R.v[i] = x[i];
  R.v[0] -= alpha;
  double vv = 0.0;
  for (int i = 0; i < len; ++i) vv += R.v[i] * R.v[i];
  R.beta = (vv == 0.0) ? 0.0 : 2.0 / vv;
  return R;
}

void apply_left(double* A, int n, const Reflector& R, int r0, int c0, int c1) {
  if (R.beta == 0.0) return;
  for (int c = c0; c <= c1; ++c) {
    double s = 0.0;
    for (int i = 0; i < R.len; ++i) s += R.v[i] * A[(r0 + i) * n + c];
    s *= R.beta;
    for (int i = 0; i < R.len; ++i) A[(r0 + i) * n + c] -= s * R.v[i];
  }
}

void apply_right(double* A, int n, const Reflector& R, int c0, int q0, int q1) {
  if (R.beta == 0.0) return;
  for (int q = q0; q <= q1; ++q) {
    double s = 0.0;
    for (int i = 0; i < R.len; ++i) s += A[q * n + c0 + i] * R.v[i];
    s *= R.beta;
    for (int i = 0; i < R.len; ++i) A[q * n + c0 + i] -= s * R.v[i];
  }
}

// One implicit double-shift step on the active block lo..hi (hi - lo >= 2),
// with shifts given by their sum `ssum` and product `sprod`.
void francis_step(double* A, int n, int lo, int hi, double ssum, double sprod) {
  auto a = [&](int i, int j) -> double& { return A[i * n + j]; };
  // first column of (H - s1 I)(H - s2 I), which has three nonzeros
  double x[3];
  x[0] = a(lo, lo) * a(lo, lo) + a(lo, lo + 1) * a(lo + 1, lo) - ssum * a(lo, lo) + sprod;
  x[1] = a(lo + 1, lo) * (a(lo, lo) + a(lo + 1, lo + 1) - ssum);
  x[2] = a(lo + 1, lo) * a(lo + 2, lo + 1);
  for (int k = lo - 1; k <= hi - 3; ++k) {
    Reflector R = make_reflector(x, 3);
    const int cfirst = std::max(k, lo);
    apply_left(A, n, R, k + 1, cfirst, hi);
    const int rlast = std::min(k + 4, hi);
    apply_right(A, n, R, k + 1, lo, rlast);
    x[0] = a(k + 2, k + 1);
    x[1] = a(k + 3, k + 1);
    if (k < hi - 3) x[2] = a(k + 4, k + 1);
  }
  Reflector R = make_reflector(x, 2);
  apply_left(A, n, R, hi - 1, hi - 2, hi);
  apply_right(A, n, R, hi - 1, lo, hi);
  // clean the bulge remnants below the subdiagonal
  for (int i = lo + 2; i <= hi; ++i)
    for (int j = lo; j < i - 1; ++j) a(i, j) = 0.0;
}

void eig2x2(double p, double q, double r, double s, double* re, double* im) {
  // eigenvalues of [[p, q], [r, s]]
  const double mid = 0.5 * (p + s);
  const double half = 0.5 * (p - s);
  const double disc = half * half + q * r;
  if (disc >= 0.0) {
    const double root = sqrt(disc);
    const double l1 = mid + (mid >= 0.0 ? root : -root);
    const double det = p * s - q * r;
    const double l2 = (l1 != 0.0) ? det / l1 : mid - (mid >= 0.0 ? root : -root);
    re[0] = l1;
    re[1] = l2;
    im[0] = im[1] = 0.0;
  } else {
    const double root = sqrt(-disc);
    re[0] = re[1] = mid;
    im[0] = root;
    im[1] = -root;
  }
}

}  // namespace

extern "C" gmr_status gmr_hessenberg_eigvals(int32_t k, const double* H, double* re, double* im) {
  if (k <= 0 || !H || !re || !im) return gmr::fail(GMR_ERR_INVALID, "gmr_hessenberg_eigvals: bad arguments");
  const int n = k;
  std::vector<double> A((size_t)n * n);
  // column-major input -> row-major work copy; entries below the subdiagonal ignored
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = (i > j + 1) ? 0.0 : H[(size_t)j * n + i];
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0;
  int total = 0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  while (hi >= 0) {
    int lo = hi;
    while (lo > 0) {
      double s = fabs(a(lo - 1, lo - 1)) + fabs(a(lo, lo));
      if (s == 0.0) s = 1.0;
      if (fabs(a(lo, lo - 1)) <= eps * s) {
        a(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      re[hi] = a(hi, hi);
      im[hi] = 0.0;
      hi -= 1;
      iter = 0;
    } else if (lo == hi - 1) {
      double r2[2], i2[2];
      eig2x2(a(hi - 1, hi - 1), a(hi - 1, hi), a(hi, hi - 1), a(hi, hi), r2, i2);
      re[hi - 1] = r2[0];
      im[hi - 1] = i2[0];
      re[hi] = r2[1];
      im[hi] = i2[1];
      hi -= 2;
      iter = 0;
    } else {
      ++iter;
      if (++total > 60 * n) return gmr::fail(GMR_ERR_NONFINITE, "Hessenberg QR did not converge");
      double ssum, sprod;
      if (iter % 10 == 0) {
        const double s = fabs(a(hi, hi - 1)) + fabs(a(hi - 1, hi - 2));
        ssum = 1.5 * s;
        sprod = s * s;
      } else {
        ssum = a(hi - 1, hi - 1) + a(hi, hi);
        sprod = a(hi - 1, hi - 1) * a(hi, hi) - a(hi - 1, hi) * a(hi, hi - 1);
      }
      francis_step(A.data(), n, lo, hi, ssum, sprod);
    }
  }
  for (int i = 0; i < n; ++i)
    if (!isfinite(re[i]) || !isfinite(im[i])) return gmr::fail(GMR_ERR_NONFINITE, "non-finite eigenvalue");
  return GMR_OK;
}

extern "C" gmr_status gmr_harmonic_ritz(int32_t k, const double* H, int32_t ldh, double* re,
                                        double* im) {
  if (k <= 0 || ldh < k + 1 || !H || !re || !im)
    return gmr::fail(GMR_ERR_INVALID, "gmr_harmonic_ritz: bad arguments");
  // M = H_k + h_{k+1,k}^2 f e_k^T, where H_k^T f = e_k, column-major k x k
  std::vector<double> M((size_t)k * k);
  // entries below the subdiagonal are zero by definition and are not read
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) M[(size_t)j * k + i] = (i > j + 1) ? 0.0 : H[(size_t)j * ldh + i];
  const double hk1 = H[(size_t)(k - 1) * ldh + k];
  // Gaussian elimination with partial pivoting on T = H_k^T (row-major T[i][j] = H(j, i))
  std::vector<double> T((size_t)k * k), f(k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) T[(size_t)i * k + j] = M[(size_t)i * k + j];
  f[k - 1] = 1.0;
  for (int c = 0; c < k; ++c) {
    int p = c;
    for (int i = c + 1; i < k; ++i)
      if (fabs(T[(size_t)i * k + c]) > fabs(T[(size_t)p * k + c])) p = i;
    if (T[(size_t)p * k + c] == 0.0) return gmr::fail(GMR_ERR_NONFINITE, "gmr_harmonic_ritz: singular H_k");
    if (p != c) {
      for (int j = 0; j < k; ++j) std::swap(T[(size_t)p * k + j], T[(size_t)c * k + j]);
      std::swap(f[p], f[c]);
    }
    for (int i = c + 1; i < k; ++i) {
      const double l = T[(size_t)i * k + c] / T[(size_t)c * k + c];
      if (l == 0.0) continue;
      for (int j = c; j < k; ++j) T[(size_t)i * k + j] -= l * T[(size_t)c * k + j];
      f[i] -= l * f[c];
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = f[i];
    for (int j = i + 1; j < k; ++j) s -= T[(size_t)i * k + j] * f[j];
    f[i] = s / T[(size_t)i * k + i];
  }
  for (int i = 0; i < k; ++i) M[(size_t)(k - 1) * k + i] += hk1 * hk1 * f[i];
  return gmr_hessenberg_eigvals(k, M.data(), re, im);
}

extern "C" gmr_status gmr_leja_order(int32_t k, double* re, double* im) {
  if (k <= 0 || !re || !im) return gmr::fail(GMR_ERR_INVALID, "gmr_leja_order: bad arguments");
  struct C { double re, im; };
  std::vector<C> rest(k), out;
  for (int i = 0; i < k; ++i) rest[i] = {re[i], im[i]};
  auto take = [&](int i) {
    C t = rest[i];
    rest.erase(rest.begin() + i);
    if (t.im != 0.0) {
      // drop the remaining value closest to the conjugate of the one taken
      int best = -1;
      double bd = INFINITY;
      for (int q = 0; q < (int)rest.size(); ++q) {
        const double d = hypot(rest[q].re - t.re, rest[q].im + t.im);
        if (d < bd) { bd = d; best = q; }
      }
      if (best >= 0) rest.erase(rest.begin() + best);
      t.im = fabs(t.im);
      out.push_back(t);
      out.push_back({t.re, -t.im});
    } else {
      out.push_back(t);
    }
  };
  // largest modulus first (ties: larger imaginary part)
  int i0 = 0;
  for (int q = 1; q < (int)rest.size(); ++q) {
    const double m0 = hypot(rest[i0].re, rest[i0].im), mq = hypot(rest[q].re, rest[q].im);
    if (mq > m0 || (mq == m0 && rest[q].im > rest[i0].im)) i0 = q;
  }
  take(i0);
  while (!rest.empty()) {
    int best = 0;
    double bs = -INFINITY;
    for (int q = 0; q < (int)rest.size(); ++q) {
      double s = 0.0;
      for (const C& c : out) s += log(hypot(rest[q].re - c.re, rest[q].im - c.im));
      if (s > bs || (s == bs && rest[q].im > rest[best].im)) { bs = s; best = q; }
    }
    take(best);
  }
  if ((int)out.size() != k) return gmr::fail(GMR_ERR_INVALID, "gmr_leja_order: unpaired complex value");
  for (int i = 0; i < k; ++i) { re[i] = out[i].re; im[i] = out[i].im; }
  return GMR_OK;
}
