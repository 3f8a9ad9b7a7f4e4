// Host-side setup math: knots, Gauss rule, B-spline tables, banded 1D
// matrices and their banded LU (Section 2: the 1D matrices M_x, K_x;
// Section 5: the mixed matrices; Appendix: banded structure |i-j| <= p and
// O(n) factorization).
#pragma once

#include <cstddef>
#include <vector>

namespace ads {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1], by Newton
// iteration on the Legendre polynomial P_q.
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);

// Open uniform knot vector on [0, 1]: p+1 zeros, k/E (k=1..E-1), p+1 ones.
std::vector<double> open_knots(int E, int p);

// Values and first derivatives of the p+1 B-splines that are non-zero on
// knot span s (t_s <= x < t_{s+1}), i.e. functions s-p .. s.
void basis_on_span(const std::vector<double>& t, int p, int s, double x, double* N, double* D);

// Element tables of one direction: for element e and Gauss point g,
// N[(e*q+g)*P + a] = B_{e+a}(x_{e,g}), D[...] = B'_{e+a}(x_{e,g}),
// W[e*q+g] = Gauss weight times element length.  Also the physical points.
struct Tables1D {
  int E, p, q, n;
  std::vector<double> N, D, W, X;
};
Tables1D make_tables(int E, int p, int q);
// The missing direction of a two-dimensional problem: one element [0, 1]
// carrying one constant function (N = 1 in slot 0, D = 0), so that its 1D
// mass matrix is [1] and its stiffness [0].
Tables1D make_tables_flat(int p, int q);

// Banded n x n matrix, band[i*(2p+1) + (j-i+p)] for |i-j| <= p.
struct Band {
  int n, p;
  std::vector<double> a;
  double& at(int i, int j) { return a[(size_t)i * (2 * p + 1) + (j - i + p)]; }
  double at(int i, int j) const { return a[(size_t)i * (2 * p + 1) + (j - i + p)]; }
};
enum MatKind { MAT_MASS = 0, MAT_STIFF = 1, MAT_MIXED = 2 };
// M = (B_i, B_j), K = (B_i', B_j'), G = (B_i, B_j') on the full index set.
Band assemble(const Tables1D& t, MatKind kind);
// Free block [off, off+m) of a banded matrix.
Band restrict_band(const Band& A, int off, int m);
// alpha*A + beta*B (same n, p).
Band axpby(double alpha, const Band& A, double beta, const Band& B);

// Banded LU without pivoting; fails (returns false) on a non-positive pivot.
struct BandLU {
  int m, p;
  std::vector<double> L, U, rd;   // L[i*p+k-1], U[i*p+k-1], rd[i]
};
bool band_lu(const Band& A, BandLU& out);

}  // namespace ads
