// Host dense linear algebra for the window and deflation problems (see hostla.h).
#include "hostla.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace ebicg {

namespace {

inline double cabs1(cd z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

// Householder reduction A = Q Hs Q^+ with Hs upper Hessenberg (A overwritten by Hs).
void hessenberg(CMat &A, CMat &Q) {
  const int n = A.rows;
  Q = CMat(n, n);
  for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
  std::vector<cd> v(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(A(i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    cd x0 = A(k + 1, k);
    cd ph = (std::abs(x0) == 0.0) ? cd(1.0) : x0 / std::abs(x0);
    cd alpha = -ph * xn;  // reflect x onto alpha e_1
    double vn = 0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = A(i, k);
      if (i == k + 1) v[i] -= alpha;
      vn += std::norm(v[i]);
    }
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // A <- (I - 2 v v^+) A
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * A(i, j);
      s *= 2.0;
      for (int i = k + 1; i < n; ++i) A(i, j) -= v[i] * s;
    }
    // A <- A (I - 2 v v^+),  Q <- Q (I - 2 v v^+)
    for (int i = 0; i < n; ++i) {
      cd s = 0, t = 0;
      for (int j = k + 1; j < n; ++j) {
        s += A(i, j) * v[j];
        t += Q(i, j) * v[j];
      }
      s *= 2.0;
      t *= 2.0;
      for (int j = k + 1; j < n; ++j) {
        A(i, j) -= s * std::conj(v[j]);
        Q(i, j) -= t * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < n; ++i) A(i, k) = 0.0;
  }
}

// Rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0].
inline void givens(cd x, cd y, double &c, cd &s) {
  double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = std::conj(y) / ay;
    return;
  }
  double r = std::hypot(ax, ay);
  c = ax / r;
  s = (x / ax) * std::conj(y) / r;
}

// Complex Schur form of the Hessenberg T (in place, T becomes upper triangular),
// accumulating the unitary similarity into Z (A = Z T Z^+ on return).
bool schur(CMat &T, CMat &Z) {
  const int n = T.rows;
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0;
  for (auto &e : T.a) anorm = std::max(anorm, cabs1(e));
  if (anorm == 0.0) anorm = 1.0;
  int ihi = n - 1;
  int its = 0, total = 0;
  const int max_total = 100 * std::max(n, 1);
  while (ihi > 0) {
    int l = 0;
    for (int k = ihi; k >= 1; --k) {
      double tst = cabs1(T(k - 1, k - 1)) + cabs1(T(k, k));
      if (tst == 0.0) tst = anorm;
      if (cabs1(T(k, k - 1)) <= eps * tst) {
        T(k, k - 1) = 0.0;
        l = k;
        break;
      }
    }
    if (l == ihi) {  // a 1x1 block has converged
      --ihi;
      its = 0;
      continue;
    }
    if (++total > max_total) return false;
    ++its;
    cd mu;
    if (its % 10 == 0) {  // exceptional shift
      mu = T(ihi, ihi) + cd(std::fabs(T(ihi, ihi - 1).real()) +
                                (ihi >= 2 ? std::fabs(T(ihi - 1, ihi - 2).real()) : 0.0),
                            0.0);
    } else {  // Wilkinson shift: eigenvalue of the trailing 2x2 closer to T(ihi, ihi)
      cd a = T(ihi - 1, ihi - 1), b = T(ihi - 1, ihi), c = T(ihi, ihi - 1), d = T(ihi, ihi);
      cd hm = 0.5 * (a - d);
      cd disc = std::sqrt(hm * hm + b * c);
      cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    }
    // implicit single-shift QR sweep over the active block l..ihi
    for (int k = l; k < ihi; ++k) {
      cd x, y;
      if (k == l) {
        x = T(k, k) - mu;
        y = T(k + 1, k);
      } else {
        x = T(k, k - 1);
        y = T(k + 1, k - 1);
      }
      double c;
      cd s;
      givens(x, y, c, s);
      int j0 = (k == l) ? k : k - 1;
      for (int j = j0; j < n; ++j) {
        cd a = T(k, j), b = T(k + 1, j);
        T(k, j) = c * a + s * b;
        T(k + 1, j) = -std::conj(s) * a + c * b;
      }
      if (k > l) T(k + 1, k - 1) = 0.0;
      int i1 = std::min(k + 2, ihi);
      for (int i = 0; i <= i1; ++i) {
        cd a = T(i, k), b = T(i, k + 1);
        T(i, k) = a * c + b * std::conj(s);
        T(i, k + 1) = -a * s + b * c;
      }
      for (int i = 0; i < n; ++i) {
        cd a = Z(i, k), b = Z(i, k + 1);
        Z(i, k) = a * c + b * std::conj(s);
        Z(i, k + 1) = -a * s + b * c;
      }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) T(i, j) = 0.0;
  return true;
}

}  // namespace

CMat matmul(const CMat &A, const CMat &B) {
  CMat C(A.rows, B.cols);
  for (int j = 0; j < B.cols; ++j)
    for (int k = 0; k < A.cols; ++k) {
      cd b = B(k, j);
      if (b == cd(0)) continue;
      for (int i = 0; i < A.rows; ++i) C(i, j) += A(i, k) * b;
    }
  return C;
}

CMat adjoint(const CMat &A) {
  CMat B(A.cols, A.rows);
  for (int j = 0; j < A.cols; ++j)
    for (int i = 0; i < A.rows; ++i) B(j, i) = std::conj(A(i, j));
  return B;
}

std::vector<int> eig_sort_order(const std::vector<cd> &lam, int which) {
  std::vector<int> idx(lam.size());
  std::iota(idx.begin(), idx.end(), 0);
  auto key = [&](int i) {
    return which == 1 ? lam[i].real() : (which == 2 ? -std::abs(lam[i]) : std::abs(lam[i]));
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) {
    const double ki = key(i), kj = key(j);
    const double scale = std::max({std::abs(lam[i]), std::abs(lam[j]), 1e-300});
    if (std::fabs(ki - kj) > 1e-12 * scale) return ki < kj;
    if (lam[i].imag() != lam[j].imag()) return lam[i].imag() > lam[j].imag();
    return i < j;
  });
  return idx;
}

bool eig_small(const CMat &C, std::vector<cd> &lam, CMat &y, CMat &z, int which) {
  const int n = C.rows;
  lam.assign(n, 0.0);
  y = CMat(n, n);
  z = CMat(n, n);
  if (n == 0) return true;
  CMat T = C, Q;
  hessenberg(T, Q);
  if (!schur(T, Q)) return false;
  const double eps = std::numeric_limits<double>::epsilon();
  double tnorm = 0;
  for (auto &e : T.a) tnorm = std::max(tnorm, std::abs(e));
  const double smin = std::max(eps * tnorm, std::numeric_limits<double>::min());
  std::vector<cd> x(n), w(n), ty(n), tz(n);
  CMat Y(n, n), Zl(n, n);
  for (int k = 0; k < n; ++k) {
    const cd lk = T(k, k);
    lam[k] = lk;
    // right: (T - lk) x = 0, x_k = 1, x_j = 0 for j > k
    std::fill(x.begin(), x.end(), cd(0));
    x[k] = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      cd s = 0;
      for (int j = i + 1; j <= k; ++j) s += T(i, j) * x[j];
      cd d = T(i, i) - lk;
      if (std::abs(d) < smin) d = smin;
      x[i] = -s / d;
    }
    // left: (T^+ - conj(lk)) w = 0, w_k = 1, w_j = 0 for j < k
    std::fill(w.begin(), w.end(), cd(0));
    w[k] = 1.0;
    for (int i = k + 1; i < n; ++i) {
      cd s = 0;
      for (int j = k; j < i; ++j) s += std::conj(T(j, i)) * w[j];
      cd d = std::conj(T(i, i) - lk);
      if (std::abs(d) < smin) d = smin;
      w[i] = -s / d;
    }
    // back to the original basis
    for (int i = 0; i < n; ++i) {
      cd sy = 0, sz = 0;
      for (int j = 0; j <= k; ++j) sy += Q(i, j) * x[j];
      for (int j = k; j < n; ++j) sz += Q(i, j) * w[j];
      ty[i] = sy;
      tz[i] = sz;
    }
    double yn = 0;
    for (int i = 0; i < n; ++i) yn += std::norm(ty[i]);
    yn = std::sqrt(yn);
    cd d = 0;
    for (int i = 0; i < n; ++i) {
      ty[i] /= yn;
      d += std::conj(tz[i]) * ty[i];
    }
    for (int i = 0; i < n; ++i) {
      Y(i, k) = ty[i];
      Zl(i, k) = tz[i] / std::conj(d);
    }
  }
  std::vector<int> ord = eig_sort_order(lam, which);
  std::vector<cd> ls(n);
  for (int c = 0; c < n; ++c) {
    ls[c] = lam[ord[c]];
    for (int i = 0; i < n; ++i) {
      y(i, c) = Y(i, ord[c]);
      z(i, c) = Zl(i, ord[c]);
    }
  }
  lam = ls;
  return true;
}

bool lu_solve(const CMat &Ain, std::vector<cd> &b) {
  CMat A = Ain;
  const int n = A.rows;
  double amax = 0;
  for (auto &e : A.a) amax = std::max(amax, std::abs(e));
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A(i, k)) > std::abs(A(p, k))) p = i;
    // relative pivot test: a pivot at rounding level of the largest entry
    // means H is singular to working precision
    if (!(std::abs(A(p, k)) > n * std::numeric_limits<double>::epsilon() * amax)) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(p, j));
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      cd f = A(i, k) / A(k, k);
      if (f == cd(0)) continue;
      for (int j = k + 1; j < n; ++j) A(i, j) -= f * A(k, j);
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    cd s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A(i, j) * b[j];
    b[i] = s / A(i, i);
  }
  return true;
}

}  // namespace ebicg
