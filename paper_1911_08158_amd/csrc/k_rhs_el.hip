// Right-hand side of the elasticity step by sum-factorized Gauss quadrature
// (Section 5: the weak form (w_(i,j), sigma_ij) with
// sigma = 2 mu eps(u) + lambda tr(eps(u)) I, i.e. the operator Upsilon):
//
//   R_{i,node} = rscale * ( amp * b_{i,node}
//                - sum_e sum_g W_g sum_j d_j B_node(x_g) sigma_ij(U^n)(x_g) ),
//
// with rscale = tau^2 for the three-level scheme.  Same tiling as the
// P-wave kernel (z-marching, LDS ring of coefficient layers, z / y
// contractions on the column grid, x-forward + stress + x-backward with one
// lane per x-element and a cross-lane assembly), carried for the three
// displacement components: 9 gradient entries forward, 9 stress-weighted
// channels backward.
#include "common.hpp"

namespace ads {

__device__ __forceinline__ int find_job_rhs_el(const RhsJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int P, int Q>
struct RhsElGeom {
  static constexpr int p = P - 1;
  static constexpr int G = 16;
  static constexpr int TX = G - p;
  static constexpr int TY = (P == 3) ? 6 : 3;   // LDS-bound: 9 channels per Gauss row
  static constexpr int TXH = TX + 2 * p;
  static constexpr int TYH = TY + 2 * p;
  static constexpr int EY = TY + p;
  static constexpr int R = EY * Q;
  static constexpr int NT = 256;
};

template <int P, int Q>
__global__ __launch_bounds__(256) void rhs_elastic_kernel(const LaunchHdr* __restrict__ hdr) {
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const RhsJob* __restrict__ jobs = hdr_jobs<RhsJob>(hdr);
  using Gm = RhsElGeom<P, Q>;
  constexpr int p = Gm::p, TX = Gm::TX, TY = Gm::TY, TXH = Gm::TXH, TYH = Gm::TYH, EY = Gm::EY,
                R = Gm::R, NT = Gm::NT;
  __shared__ double ring[3][P][TYH][TXH];
  __shared__ double Ab[3][TYH][TXH];
  __shared__ double Bb[3][TYH][TXH];
  __shared__ double S[9][R][TXH];
  __shared__ double tyN[EY][Q][P];
  __shared__ double tyD[EY][Q][P];
  __shared__ double tyW[EY][Q];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int j = lane & 15;
  const int rg = (tid >> 6) * 4 + (lane >> 4);
  const bool own = tid < TX * TY;
  const int cxo = tid % TX, cyo = tid / TX;

  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const RhsJob& J = jobs[find_job_rhs_el(jobs, njobs, tile)];
    const int t = tile - J.tile0;
    const int tx = t % J.tiles[0];
    const int t2 = t / J.tiles[0];
    const int ty = t2 % J.tiles[1];
    const int tz = t2 / J.tiles[1];
    const int Ex = J.E[0], Ey = J.E[1], Ez = J.E[2];
    const int nfx = J.nf[0], nfy = J.nf[1], nfz = J.nf[2];
    const int ox = J.off[0], oy = J.off[1], oz = J.off[2];
    const int X0 = ox + tx * TX, Y0 = oy + ty * TY, Z0 = oz + tz * J.TZ;
    const int Zend = min(Z0 + J.TZ, oz + nfz);
    const long long sxy = (long long)nfx * nfy;
    const long long nfree = sxy * nfz;
    const double mu = J.mu, lam = J.lam;
    const gmem<double>* __restrict__ Ug = gview(J.u);
    const gmem<double>* __restrict__ LD = gview(J.load);
    gmem<double>* __restrict__ Rg = gview(J.R);
    const double rscale = J.rscale;

    const gmem<double>* tyg = gview(J.tab[1]);
    for (int k = tid; k < EY * Q * P; k += NT) {
      int eyl = k / (Q * P), rest = k - eyl * (Q * P);
      int ey = Y0 - p + eyl;
      bool v = ey >= 0 && ey < Ey;
      (&tyN[0][0][0])[k] = v ? tyg[(long long)ey * Q * P + rest] : 0.0;
      (&tyD[0][0][0])[k] = v ? tyg[(long long)Ey * Q * P + (long long)ey * Q * P + rest] : 0.0;
    }
    for (int k = tid; k < EY * Q; k += NT) {
      int eyl = k / Q, g = k - eyl * Q;
      int ey = Y0 - p + eyl;
      (&tyW[0][0])[k] = (ey >= 0 && ey < Ey) ? tyg[2ll * Ey * Q * P + (long long)ey * Q + g] : 0.0;
    }
    const int ex = X0 - p + j;
    const bool exv = ex >= 0 && ex < Ex;
    double xN[Q][P], xD[Q][P], xW[Q];
    {
      const gmem<double>* txg = gview(J.tab[0]);
#pragma unroll
      for (int g = 0; g < Q; ++g) {
#pragma unroll
        for (int a = 0; a < P; ++a) {
          xN[g][a] = exv ? txg[((long long)ex * Q + g) * P + a] : 0.0;
          xD[g][a] = exv ? txg[(long long)Ex * Q * P + ((long long)ex * Q + g) * P + a] : 0.0;
        }
        xW[g] = exv ? txg[2ll * Ex * Q * P + (long long)ex * Q + g] : 0.0;
      }
    }
    double ampv = 0.0;
    if (J.load != nullptr && J.amp != nullptr) {
      long long ai = (long long)(*gview(J.counter)) + J.amp_shift;
      ampv = (ai >= 0 && ai < J.namp) ? gview(J.amp)[ai] : 0.0;
    }

    auto load_layer = [&](int cz) {
      const int slot = cz % P;
      const bool zv = cz >= oz && cz < oz + nfz;
      for (int k = tid; k < TYH * TXH; k += NT) {
        int cyl = k / TXH, cxl = k - cyl * TXH;
        int cy = Y0 - p + cyl, cx = X0 - p + cxl;
        double w0 = 0.0, w1 = 0.0, w2 = 0.0;
        if (zv && cy >= oy && cy < oy + nfy && cx >= ox && cx < ox + nfx) {
          long long gi = (long long)(cz - oz) * sxy + (long long)(cy - oy) * nfx + (cx - ox);
          w0 = Ug[gi];
          w1 = Ug[nfree + gi];
          w2 = Ug[2 * nfree + gi];
        }
        ring[0][slot][cyl][cxl] = w0;
        ring[1][slot][cyl][cxl] = w1;
        ring[2][slot][cyl][cxl] = w2;
      }
    };
    auto store_out = [&](int cz, int c, double accv) {
      const int cy = Y0 + cyo, cx = X0 + cxo;
      if (cz >= Z0 && cz < Zend && cy < oy + nfy && cx < ox + nfx) {
        long long gi = (long long)(cz - oz) * sxy + (long long)(cy - oy) * nfx + (cx - ox) + c * nfree;
        double f = (LD != nullptr) ? ampv * LD[gi] : 0.0;
        Rg[gi] = rscale * (f - accv);
      }
    };

    double acc[3][P];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < P; ++a) acc[c][a] = 0.0;

    const int ez0 = max(0, Z0 - p);
    const int ez1 = min(Ez - 1, Zend - 1);
    for (int cz = ez0; cz <= ez0 + p; ++cz) load_layer(cz);
    __syncthreads();

    // z tables at wave-uniform addresses: scalar loads
    const cmem<double>* tzg = cview(J.tab[2]);
    for (int ez = ez0; ez <= ez1; ++ez) {
      for (int gz = 0; gz < Q; ++gz) {
        double nz[P], dz[P];
#pragma unroll
        for (int a = 0; a < P; ++a) {
          nz[a] = tzg[((long long)ez * Q + gz) * P + a];
          dz[a] = tzg[(long long)Ez * Q * P + ((long long)ez * Q + gz) * P + a];
        }
        const double wz = tzg[2ll * Ez * Q * P + (long long)ez * Q + gz];
        // S1
        for (int k = tid; k < 3 * TYH * TXH; k += NT) {
          int c = k / (TYH * TXH), rem = k - c * (TYH * TXH);
          int cyl = rem / TXH, cxl = rem - cyl * TXH;
          double A = 0.0, B = 0.0;
          const double r0 = ring[c][ez % P][cyl][cxl];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            double r = ring[c][(ez + a) % P][cyl][cxl];
            A = fma(nz[a], r, A);
            B = fma(dz[a], r - r0, B);   // sum_a dz[a] = 0: contract differences
          }
          Ab[c][cyl][cxl] = A;
          Bb[c][cyl][cxl] = B;
        }
        __syncthreads();
        // S2
        for (int k = tid; k < 3 * EY * TXH; k += NT) {
          int c = k / (EY * TXH), rem = k - c * (EY * TXH);
          int eyl = rem / TXH, cxl = rem - eyl * TXH;
          double av[P], bv[P];
#pragma unroll
          for (int b = 0; b < P; ++b) {
            av[b] = Ab[c][eyl + b][cxl];
            bv[b] = Bb[c][eyl + b][cxl];
          }
#pragma unroll
          for (int gy = 0; gy < Q; ++gy) {
            double cc = 0.0, dyv = 0.0, dzv = 0.0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
              cc = fma(tyN[eyl][gy][b], av[b], cc);
              dyv = fma(tyD[eyl][gy][b], av[b] - av[0], dyv);
              dzv = fma(tyN[eyl][gy][b], bv[b], dzv);
            }
            S[3 * c + 0][eyl * Q + gy][cxl] = cc;
            S[3 * c + 1][eyl * Q + gy][cxl] = dyv;
            S[3 * c + 2][eyl * Q + gy][cxl] = dzv;
          }
        }
        __syncthreads();
        // S34: gradients, stress, x-backward
        for (int r = rg; r < R; r += 16) {
          const int eyl = r / Q, gy = r - eyl * Q;
          const double wyz = tyW[eyl][gy] * wz;
          double cin[9][P];
#pragma unroll
          for (int ch = 0; ch < 9; ++ch)
#pragma unroll
            for (int a = 0; a < P; ++a) cin[ch][a] = S[ch][r][j + a];
          double o[9][P];
#pragma unroll
          for (int ch = 0; ch < 9; ++ch)
#pragma unroll
            for (int a = 0; a < P; ++a) o[ch][a] = 0.0;
#pragma unroll
          for (int gx = 0; gx < Q; ++gx) {
            double g[3][3];  // g[c][m] = d_m U_c
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
              for (int a = 0; a < P; ++a) {
                d0 = fma(xD[gx][a], cin[3 * c + 0][a] - cin[3 * c + 0][0], d0);
                d1 = fma(xN[gx][a], cin[3 * c + 1][a], d1);
                d2 = fma(xN[gx][a], cin[3 * c + 2][a], d2);
              }
              g[c][0] = d0;
              g[c][1] = d1;
              g[c][2] = d2;
            }
            const double w = xW[gx] * wyz;
            const double ldiv = lam * (g[0][0] + g[1][1] + g[2][2]);
            double sg[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
              for (int m = 0; m < 3; ++m) sg[c][m] = w * (mu * (g[c][m] + g[m][c]) + (c == m ? ldiv : 0.0));
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
              for (int a = 0; a < P; ++a) {
                o[3 * c + 0][a] = fma(xD[gx][a], sg[c][0], o[3 * c + 0][a]);
                o[3 * c + 1][a] = fma(xN[gx][a], sg[c][1], o[3 * c + 1][a]);
                o[3 * c + 2][a] = fma(xN[gx][a], sg[c][2], o[3 * c + 2][a]);
              }
          }
          double res[9];
#pragma unroll
          for (int ch = 0; ch < 9; ++ch) {
            double rr = o[ch][0];
#pragma unroll
            for (int a = 1; a < P; ++a) rr += __shfl_up(o[ch][a], a, 16);
            res[ch] = rr;
          }
          if (j >= p) {
#pragma unroll
            for (int ch = 0; ch < 9; ++ch) S[ch][r][j - p] = res[ch];
          }
        }
        __syncthreads();
        // S5: y- and z-backward per test component
        if (own) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double Ap = 0.0, Bp = 0.0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
              const int eyl = cyo + p - b;
#pragma unroll
              for (int gy = 0; gy < Q; ++gy) {
                const int rr = eyl * Q + gy;
                Ap = fma(tyN[eyl][gy][b], S[3 * c + 0][rr][cxo], Ap);
                Ap = fma(tyD[eyl][gy][b], S[3 * c + 1][rr][cxo], Ap);
                Bp = fma(tyN[eyl][gy][b], S[3 * c + 2][rr][cxo], Bp);
              }
            }
#pragma unroll
            for (int a = 0; a < P; ++a) acc[c][a] = fma(nz[a], Ap, fma(dz[a], Bp, acc[c][a]));
          }
        }
      }
      if (own) {
#pragma unroll
        for (int c = 0; c < 3; ++c) store_out(ez, c, acc[c][0]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int a = 0; a < P - 1; ++a) acc[c][a] = acc[c][a + 1];
        acc[c][P - 1] = 0.0;
      }
      if (ez < ez1) load_layer(ez + P);
      __syncthreads();
    }
    if (own) {
#pragma unroll
      for (int a = 0; a < P - 1; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) store_out(ez1 + 1 + a, c, acc[c][a]);
    }
    __syncthreads();
  }
}

int rhs_el_tile_x(int p) { return 16 - p; }
int rhs_el_tile_y(int p) { return p == 2 ? 6 : 3; }

hipError_t launch_rhs_elastic(int p, const LaunchHdr* d_hdr, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (p == 2) {
    hipLaunchKernelGGL((rhs_elastic_kernel<3, 3>), dim3(grid), dim3(256), 0, s, d_hdr);
  } else if (p == 3) {
    hipLaunchKernelGGL((rhs_elastic_kernel<4, 4>), dim3(grid), dim3(256), 0, s, d_hdr);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ads
