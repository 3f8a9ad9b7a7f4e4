#include "host_math.hpp"

#include <algorithm>
#include <cmath>

namespace ads {

void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  std::vector<int> ord(q);
  for (int i = 0; i < q; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(q), ws(q);
  for (int i = 0; i < q; ++i) {
    xs[i] = x[ord[i]];
    ws[i] = w[ord[i]];
  }
  x = xs;
  w = ws;
}

std::vector<double> open_knots(int E, int p) {
  std::vector<double> t;
  for (int i = 0; i <= p; ++i) t.push_back(0.0);
  for (int k = 1; k < E; ++k) t.push_back((double)k / E);
  for (int i = 0; i <= p; ++i) t.push_back(1.0);
  return t;
}

// Triangular evaluation of the non-zero degree-k functions on span s.
static void span_values(const std::vector<double>& t, int k, int s, double x, double* N) {
  double left[8], right[8];
  N[0] = 1.0;
  for (int j = 1; j <= k; ++j) {
    left[j] = x - t[s + 1 - j];
    right[j] = t[s + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      double den = right[r + 1] + left[j - r];
      double tmp = den != 0.0 ? N[r] / den : 0.0;
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
}

void basis_on_span(const std::vector<double>& t, int p, int s, double x, double* N, double* D) {
  span_values(t, p, s, x, N);
  double Nm[8];  // degree p-1 functions s-p+1 .. s
  if (p == 0) {
    D[0] = 0.0;
    return;
  }
  span_values(t, p - 1, s, x, Nm);
  for (int a = 0; a <= p; ++a) {
    int i = s - p + a;  // function index
    // B'_{i,p} = p/(t_{i+p}-t_i) B_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1}
    double b_i = (a >= 1) ? Nm[a - 1] : 0.0;       // B_{i,p-1}, index i-(s-p+1) = a-1
    double b_i1 = (a <= p - 1) ? Nm[a] : 0.0;      // B_{i+1,p-1}
    double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
    double v = 0.0;
    if (d1 > 0) v += p / d1 * b_i;
    if (d2 > 0) v -= p / d2 * b_i1;
    D[a] = v;
  }
}

Tables1D make_tables(int E, int p, int q) {
  Tables1D T;
  T.E = E;
  T.p = p;
  T.q = q;
  T.n = E + p;
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  std::vector<double> t = open_knots(E, p);
  const int P = p + 1;
  T.N.assign((size_t)E * q * P, 0.0);
  T.D.assign((size_t)E * q * P, 0.0);
  T.W.assign((size_t)E * q, 0.0);
  T.X.assign((size_t)E * q, 0.0);
  for (int e = 0; e < E; ++e) {
    double a = (double)e / E, b = (double)(e + 1) / E;
    for (int g = 0; g < q; ++g) {
      double x = 0.5 * (a + b) + 0.5 * (b - a) * gx[g];
      T.X[e * q + g] = x;
      T.W[e * q + g] = 0.5 * (b - a) * gw[g];
      basis_on_span(t, p, e + p, x, &T.N[((size_t)e * q + g) * P], &T.D[((size_t)e * q + g) * P]);
    }
  }
  return T;
}

Tables1D make_tables_flat(int p, int q) {
  Tables1D T;
  T.E = 1;
  T.p = p;
  T.q = q;
  T.n = 1 + p;
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  const int P = p + 1;
  T.N.assign((size_t)q * P, 0.0);
  T.D.assign((size_t)q * P, 0.0);
  T.W.assign(q, 0.0);
  T.X.assign(q, 0.0);
  for (int g = 0; g < q; ++g) {
    T.X[g] = 0.5 + 0.5 * gx[g];
    T.W[g] = 0.5 * gw[g];
    T.N[(size_t)g * P] = 1.0;
  }
  return T;
}

Band assemble(const Tables1D& t, MatKind kind) {
  Band A;
  A.n = t.n;
  A.p = t.p;
  A.a.assign((size_t)t.n * (2 * t.p + 1), 0.0);
  const int P = t.p + 1;
  for (int e = 0; e < t.E; ++e)
    for (int g = 0; g < t.q; ++g) {
      const double* N = &t.N[((size_t)e * t.q + g) * P];
      const double* D = &t.D[((size_t)e * t.q + g) * P];
      double w = t.W[e * t.q + g];
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
          double v = kind == MAT_MASS ? N[i] * N[j] : kind == MAT_STIFF ? D[i] * D[j] : N[i] * D[j];
          A.at(e + i, e + j) += w * v;
        }
    }
  return A;
}

Band restrict_band(const Band& A, int off, int m) {
  Band B;
  B.n = m;
  B.p = A.p;
  B.a.assign((size_t)m * (2 * A.p + 1), 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = std::max(0, i - A.p); j <= std::min(m - 1, i + A.p); ++j) B.at(i, j) = A.at(i + off, j + off);
  return B;
}

Band axpby(double alpha, const Band& A, double beta, const Band& B) {
  Band C = A;
  for (size_t k = 0; k < C.a.size(); ++k) C.a[k] = alpha * A.a[k] + beta * B.a[k];
  return C;
}

bool band_lu(const Band& A0, BandLU& out) {
  Band A = A0;
  const int m = A.n, p = A.p;
  for (int k = 0; k < m; ++k) {
    double piv = A.at(k, k);
    if (!(piv > 0.0)) return false;
    for (int i = k + 1; i <= std::min(m - 1, k + p); ++i) {
      double l = A.at(i, k) / piv;
      A.at(i, k) = l;
      for (int j = k + 1; j <= std::min(m - 1, k + p); ++j) A.at(i, j) -= l * A.at(k, j);
    }
  }
  out.m = m;
  out.p = p;
  out.L.assign((size_t)m * p, 0.0);
  out.U.assign((size_t)m * p, 0.0);
  out.rd.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    for (int k = 1; k <= p; ++k) {
      if (i - k >= 0) out.L[(size_t)i * p + k - 1] = A.at(i, i - k);
      if (i + k < m) out.U[(size_t)i * p + k - 1] = A.at(i, i + k);
    }
    out.rd[i] = 1.0 / A.at(i, i);
  }
  return true;
}

}  // namespace ads
