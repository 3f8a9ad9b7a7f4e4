// Host-side checks of the library's setup math, built with the address and
// undefined-behaviour sanitizers by tests/test_host_sanitizers.py: every
// degree 1..5, Gauss rules p+1..p+3, element counts from 1 up, both boundary
// conditions.  Checks, besides memory safety: Gauss weights sum to 2 and
// integrate x^(2q-2) exactly, the basis is a partition of unity with
// derivatives summing to zero, the mass matrix sums to 1, the stiffness
// annihilates constants, and the banded LU of M + eta K reproduces the
// matrix.  Exit status 0 on success.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1911_08158_amd/csrc/host_math.hpp"

using namespace ads;

static int fails = 0;
static void check(bool ok, const char* what, int p, int E, int q) {
  if (!ok) {
    std::printf("FAIL %s p=%d E=%d q=%d\n", what, p, E, q);
    ++fails;
  }
}

int main() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> uni(0.0, 1.0);
  for (int q = 1; q <= 8; ++q) {
    std::vector<double> x, w;
    gauss_legendre(q, x, w);
    double sw = 0.0, mom = 0.0;
    for (int i = 0; i < q; ++i) {
      sw += w[i];
      mom += w[i] * std::pow(x[i], 2 * q - 2);
    }
    check(std::fabs(sw - 2.0) < 1e-13, "weights", 0, 0, q);
    check(std::fabs(mom - 2.0 / (2 * q - 1)) < 1e-13, "moment", 0, 0, q);
  }
  for (int p = 1; p <= 5; ++p)
    for (int E : {1, 2, 3, 7, 17}) {
      const std::vector<double> t = open_knots(E, p);
      for (int k = 0; k < 20; ++k) {
        const double xv = uni(rng);
        int s = p;
        while (s < E + p - 1 && xv >= t[s + 1]) ++s;
        std::vector<double> N(p + 1), D(p + 1);
        basis_on_span(t, p, s, xv, N.data(), D.data());
        double sn = 0.0, sd = 0.0;
        for (int a = 0; a <= p; ++a) {
          sn += N[a];
          sd += D[a];
        }
        check(std::fabs(sn - 1.0) < 1e-13, "partition of unity", p, E, 0);
        check(std::fabs(sd) < 1e-9 * E, "derivatives sum", p, E, 0);
      }
      for (int q = p + 1; q <= p + 3; ++q) {
        const Tables1D tb = make_tables(E, p, q);
        const Band M = assemble(tb, MAT_MASS), K = assemble(tb, MAT_STIFF), G = assemble(tb, MAT_MIXED);
        double sm = 0.0, kmax = 0.0;
        for (int i = 0; i < M.n; ++i) {
          double rk = 0.0;
          for (int j = std::max(0, i - p); j <= std::min(M.n - 1, i + p); ++j) {
            sm += M.at(i, j);
            rk += K.at(i, j);
            (void)G.at(i, j);
          }
          kmax = std::max(kmax, std::fabs(rk));
        }
        check(std::fabs(sm - 1.0) < 1e-13, "mass sums to 1", p, E, q);
        check(kmax < 1e-9 * E, "stiffness annihilates constants", p, E, q);
        for (int off : {0, 1}) {
          const int m = M.n - 2 * off;
          if (m < 1) continue;
          const double eta = 0.25 * 1e-4;
          const Band A = axpby(1.0, restrict_band(M, off, m), eta, restrict_band(K, off, m));
          BandLU lu;
          const bool ok = band_lu(A, lu);
          check(ok, "band LU", p, E, q);
          if (!ok) continue;
          // L U = A on the band (L unit lower, U upper with 1/rd on the diagonal)
          double err = 0.0, amax = 0.0;
          for (int i = 0; i < m; ++i)
            for (int j = std::max(0, i - p); j <= std::min(m - 1, i + p); ++j) {
              double s = 0.0;
              for (int k = std::max(0, std::max(i, j) - p); k <= std::min(i, j); ++k) {
                const double l = (k == i) ? 1.0 : lu.L[(size_t)i * p + (i - k) - 1];
                const double u = (k == j) ? 1.0 / lu.rd[k] : lu.U[(size_t)k * p + (j - k) - 1];
                s += l * u;
              }
              err = std::max(err, std::fabs(s - A.at(i, j)));
              amax = std::max(amax, std::fabs(A.at(i, j)));
            }
          check(err <= 1e-13 * amax, "L U = A", p, E, q);
        }
      }
    }
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
