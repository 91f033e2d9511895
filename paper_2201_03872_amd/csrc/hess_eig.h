// Eigenvalues and right eigenvectors of a small complex matrix (host code):
// the harmonic Ritz problem of GMRES with deflated restarting (H_m plus a
// rank-one update of its last column; after a deflated restart H_m has a
// full leading block, so it is first reduced to Hessenberg form).
//
// Method: Householder reduction to upper Hessenberg form, then the shifted
// QR algorithm on the Hessenberg form (Francis' single
// shift, complex arithmetic, Wilkinson shift from the trailing 2x2 block,
// an exceptional shift every 10 iterations without deflation), with
// deflation at negligible subdiagonal entries, accumulating the unitary
// transformations so that H = Z S Z^H with S upper triangular; the
// eigenvectors of S follow by back substitution and are mapped back by Z.
// Matrices are row-major, a[i * n + j].
#pragma once

#include <cmath>
#include <complex>
#include <limits>
#include <vector>

namespace ddamg {

using hcd = std::complex<double>;

// Givens rotation G = [c s; -conj(s) c] (c real) with G [a; b] = [r; 0].
inline void hess_givens(hcd a, hcd b, double& c, hcd& s) {
  const double na = std::abs(a), nb = std::abs(b);
  if (nb == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (na == 0.0) {
    c = 0.0;
    s = std::conj(b) / nb;
    return;
  }
  const double nr = std::hypot(na, nb);
  c = na / nr;
  s = (a / na) * std::conj(b) / nr;
}

// Householder reduction a -> Q^H a Q (upper Hessenberg), z <- z Q.
inline void hess_reduce(int n, std::vector<hcd>& a, std::vector<hcd>& z) {
  auto A = [&](int i, int j) -> hcd& { return a[(size_t)i * n + j]; };
  std::vector<hcd> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(A(i, k));
    xn = std::sqrt(xn);
    double tail = 0;
    for (int i = k + 2; i < n; ++i) tail += std::norm(A(i, k));
    if (tail == 0.0) continue;
    // v = x + e^{i arg x0} |x| e_0, P = I - 2 v v^H / (v^H v)
    const hcd x0 = A(k + 1, k);
    const hcd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : hcd(1.0);
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = A(i, k);
    v[k + 1] += ph * xn;
    double vn = 0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // a <- P a (rows k+1..n-1)
    for (int j = 0; j < n; ++j) {
      hcd d = 0.0;
      for (int i = k + 1; i < n; ++i) d += std::conj(v[i]) * A(i, j);
      d *= 2.0 / vn;
      for (int i = k + 1; i < n; ++i) A(i, j) -= d * v[i];
    }
    // a <- a P, z <- z P (columns k+1..n-1)
    for (int i = 0; i < n; ++i) {
      hcd d = 0.0, dz = 0.0;
      for (int j = k + 1; j < n; ++j) {
        d += A(i, j) * v[j];
        dz += z[(size_t)i * n + j] * v[j];
      }
      d *= 2.0 / vn;
      dz *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) {
        A(i, j) -= d * std::conj(v[j]);
        z[(size_t)i * n + j] -= dz * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < n; ++i) A(i, k) = 0.0;
  }
}

// Returns false if the QR iteration did not converge.  w: n eigenvalues,
// vec: n x n, column i the unit eigenvector of w[i].  Any square input.
inline bool hess_eig(int n, std::vector<hcd> a, std::vector<hcd>& w, std::vector<hcd>& vec) {
  const double eps = std::numeric_limits<double>::epsilon();
  std::vector<hcd> z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
  hess_reduce(n, a, z);
  auto A = [&](int i, int j) -> hcd& { return a[(size_t)i * n + j]; };
  double anorm = 0;
  for (auto& v : a) anorm = std::max(anorm, std::abs(v));
  if (anorm == 0) anorm = 1;
  int hi = n - 1, its = 0, total = 0;
  while (hi >= 0) {
    // find the start l of the unreduced block ending at hi
    int l = hi;
    while (l > 0) {
      const double s = std::abs(A(l - 1, l - 1)) + std::abs(A(l, l));
      if (std::abs(A(l, l - 1)) <= eps * (s > 0 ? s : anorm)) {
        A(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {   // 1x1 block converged
      --hi;
      its = 0;
      continue;
    }
    if (++total > 60 * n) return false;
    ++its;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 closest to A(hi, hi)
    hcd sigma;
    if (its % 10 == 0) {
      sigma = A(hi, hi) + std::abs(A(hi, hi - 1)) * 1.5;
    } else {
      const hcd p = A(hi - 1, hi - 1), q = A(hi - 1, hi), r = A(hi, hi - 1), t = A(hi, hi);
      const hcd tr = p + t, det = p * t - q * r;
      const hcd disc = std::sqrt(tr * tr * 0.25 - det);
      const hcd e1 = tr * 0.5 + disc, e2 = tr * 0.5 - disc;
      sigma = std::abs(e1 - t) < std::abs(e2 - t) ? e1 : e2;
    }
    // one QR step on rows/columns l..hi of (A - sigma I), applied to the
    // whole matrix so that the Schur form and Z stay consistent
    std::vector<double> cs(hi - l);
    std::vector<hcd> sn(hi - l);
    for (int k = l; k <= hi; ++k) A(k, k) -= sigma;
    for (int k = l; k < hi; ++k) {
      double c;
      hcd s;
      hess_givens(A(k, k), A(k + 1, k), c, s);
      cs[k - l] = c;
      sn[k - l] = s;
      for (int j = k; j < n; ++j) {   // rows k, k+1 from the left
        const hcd x = A(k, j), y = A(k + 1, j);
        A(k, j) = c * x + s * y;
        A(k + 1, j) = -std::conj(s) * x + c * y;
      }
    }
    for (int k = l; k < hi; ++k) {   // columns k, k+1 from the right (G^H)
      const double c = cs[k - l];
      const hcd s = sn[k - l];
      const int imax = std::min(hi, k + 2);
      for (int i = 0; i <= imax; ++i) {
        const hcd x = A(i, k), y = A(i, k + 1);
        A(i, k) = c * x + std::conj(s) * y;
        A(i, k + 1) = -s * x + c * y;
      }
      for (int i = 0; i < n; ++i) {
        const hcd x = z[(size_t)i * n + k], y = z[(size_t)i * n + k + 1];
        z[(size_t)i * n + k] = c * x + std::conj(s) * y;
        z[(size_t)i * n + k + 1] = -s * x + c * y;
      }
    }
    for (int k = l; k <= hi; ++k) A(k, k) += sigma;
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A(i, i);
  // eigenvectors of the triangular S, then back to the original basis
  vec.assign((size_t)n * n, 0.0);
  std::vector<hcd> y(n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) y[j] = 0.0;
    y[i] = 1.0;
    for (int j = i - 1; j >= 0; --j) {
      hcd s = 0.0;
      for (int l2 = j + 1; l2 <= i; ++l2) s += A(j, l2) * y[l2];
      hcd d = A(j, j) - w[i];
      if (std::abs(d) < eps * anorm) d = eps * anorm;
      y[j] = -s / d;
    }
    double nv = 0;
    for (int r = 0; r < n; ++r) {
      hcd v = 0.0;
      for (int j = 0; j <= i; ++j) v += z[(size_t)r * n + j] * y[j];
      vec[(size_t)r * n + i] = v;
      nv += std::norm(v);
    }
    nv = std::sqrt(nv);
    if (nv > 0)
      for (int r = 0; r < n; ++r) vec[(size_t)r * n + i] /= nv;
  }
  return true;
}

}  // namespace ddamg
