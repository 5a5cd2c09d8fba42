// Host-side dense linear algebra for the small problems of eigBiCG:
// the m x m window eigenproblem eig(C) (Sec. 1, end; Alg. BiCG-eigen),
// biorthogonalisation in coefficient space, and the K x K deflation solve
// H d = U_l^+ r (Alg. Incremental eigBiCG).  No LAPACK is linked: ROCm ships
// no non-symmetric eigensolver, so the library carries its own.
#pragma once

#include <complex>
#include <vector>

namespace ebicg {

using cd = std::complex<double>;

// Column-major dense matrix.
struct CMat {
  int rows = 0, cols = 0;
  std::vector<cd> a;
  CMat() = default;
  CMat(int r, int c) : rows(r), cols(c), a(size_t(r) * c, cd(0)) {}
  cd &operator()(int i, int j) { return a[size_t(i) + size_t(j) * rows]; }
  const cd &operator()(int i, int j) const { return a[size_t(i) + size_t(j) * rows]; }
  cd *col(int j) { return a.data() + size_t(j) * rows; }
  const cd *col(int j) const { return a.data() + size_t(j) * rows; }
};

CMat matmul(const CMat &A, const CMat &B);
CMat adjoint(const CMat &A);

// Sort order of eigenvalues by a criterion (Sec. 1, end: a user-chosen one):
// which = 0 |lambda| ascending, 1 real part ascending, 2 |lambda| descending.
// Keys equal to 1e-12 relative (to the larger modulus) are ordered by
// imaginary part descending.
std::vector<int> eig_sort_order(const std::vector<cd> &lam, int which = 0);

// [y, z, lam] = eig(C): right vectors y, left vectors z (z_i^+ C = lam_i z_i^+),
// ||y_i|| = 1, z_i^+ y_i = 1, sorted by eig_sort_order.  Householder
// Hessenberg reduction, complex single-shift QR (Wilkinson shifts), and
// triangular back/forward substitution for the eigenvectors of the Schur form.
// Returns false if the QR iteration fails to converge.
bool eig_small(const CMat &C, std::vector<cd> &lam, CMat &y, CMat &z, int which = 0);

// Solve A x = b (A square) by Gaussian elimination with partial pivoting.
// Returns false if A is numerically singular.
bool lu_solve(const CMat &A, std::vector<cd> &b);

}  // namespace ebicg
