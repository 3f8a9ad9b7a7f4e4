// Right-hand side of the P-wave step by sum-factorized Gauss quadrature
// (Section 2: the tested equation gives (grad B_i, grad w_h) for the
// stiffness action, written as K = K_x(x)M_y(x)M_z + ... in eq. pwave2; here
// it is evaluated element by element at the q^3 Gauss points as a chain of
// 1D contractions instead of assembling K):
//
//   R_i = rscale * ( amp * b_i - sum_e sum_g W_g grad B_i(x_g) . grad w_h(x_g) ),
//   w   = cu*u + cv*v + ca*a   (the Newmark predictor u + tau u' + tau^2/4 u'').
//
// Tiling on gfx950 (owner computes, no atomics, deterministic):
//   * a workgroup owns TX x TY coefficient columns and a z-range of TZ
//     coefficients; it marches over the element layers that touch the range;
//   * per element layer the predictor w is formed once into an LDS ring of
//     p+1 coefficient layers (halo p on each side in x and y);
//   * per z Gauss point: (S1) z-contraction to values/derivatives on the
//     column grid, (S2) y-contraction to the y Gauss rows, (S34) x-forward,
//     weighting and x-backward with one lane per x-element (16-lane groups,
//     one per Gauss row) and a cross-lane shift-and-add that assembles each
//     coefficient from its p+1 elements, (S5) y-backward and z-backward into
//     per-thread accumulators of the owned column (p+1 z-layers in flight);
//   * a z-layer is written when its last contributing element is done.
#include "common.hpp"

namespace ads {

__device__ __forceinline__ int find_job_rhs(const RhsJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int P, int Q>
struct RhsGeom {
  static constexpr int p = P - 1;
  static constexpr int G = 16;          // lanes per Gauss row (x-elements of the tile)
  static constexpr int TX = G - p;      // owned x-coefficients
  static constexpr int TY = 16;         // owned y-coefficients
  static constexpr int TXH = TX + 2 * p;
  static constexpr int TYH = TY + 2 * p;
  static constexpr int EY = TY + p;     // y-elements touching the owned columns
  static constexpr int R = EY * Q;      // y Gauss rows
  static constexpr int NT = 256;
};

template <int P, int Q>
__global__ __launch_bounds__(256) void rhs_pwave_kernel(const RhsJob* __restrict__ jobs, int njobs,
                                                        int total_tiles) {
  using Gm = RhsGeom<P, Q>;
  constexpr int p = Gm::p, TX = Gm::TX, TY = Gm::TY, TXH = Gm::TXH, TYH = Gm::TYH, EY = Gm::EY,
                R = Gm::R, NT = Gm::NT;
  __shared__ double ring[P][TYH][TXH];
  __shared__ double Ab[TYH][TXH];
  __shared__ double Bb[TYH][TXH];
  __shared__ double S[3][R][TXH];
  __shared__ double tyN[EY][Q][P];
  __shared__ double tyD[EY][Q][P];
  __shared__ double tyW[EY][Q];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int j = lane & 15;                        // x-element slot within the Gauss row group
  const int rg = (tid >> 6) * 4 + (lane >> 4);    // Gauss row group 0..15
  const bool own = tid < TX * TY;
  const int cxo = tid % TX, cyo = tid / TX;

  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const RhsJob& J = jobs[find_job_rhs(jobs, njobs, tile)];
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

    // y tables of the tile's y-elements (zero outside the mesh)
    const double* tyg = J.tab[1];
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
    // x tables of this lane's x-element, kept in registers
    const int ex = X0 - p + j;
    const bool exv = ex >= 0 && ex < Ex;
    double xN[Q][P], xD[Q][P], xW[Q];
    {
      const double* txg = J.tab[0];
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
      long long ai = (long long)(*J.counter) + J.amp_shift;
      ampv = (ai >= 0 && ai < J.namp) ? J.amp[ai] : 0.0;
    }

    auto load_layer = [&](int cz) {
      const int slot = cz % P;
      const bool zv = cz >= oz && cz < oz + nfz;
      for (int k = tid; k < TYH * TXH; k += NT) {
        int cyl = k / TXH, cxl = k - cyl * TXH;
        int cy = Y0 - p + cyl, cx = X0 - p + cxl;
        double w = 0.0;
        if (zv && cy >= oy && cy < oy + nfy && cx >= ox && cx < ox + nfx) {
          long long gi = (long long)(cz - oz) * sxy + (long long)(cy - oy) * nfx + (cx - ox);
          w = J.cu * J.u[gi];
          if (J.v != nullptr) w = fma(J.cv, J.v[gi], w);
          if (J.a != nullptr) w = fma(J.ca, J.a[gi], w);
        }
        ring[slot][cyl][cxl] = w;
      }
    };
    auto store_out = [&](int cz, double accv) {
      const int cy = Y0 + cyo, cx = X0 + cxo;
      if (cz >= Z0 && cz < Zend && cy < oy + nfy && cx < ox + nfx) {
        long long gi = (long long)(cz - oz) * sxy + (long long)(cy - oy) * nfx + (cx - ox);
        double f = (J.load != nullptr) ? ampv * J.load[gi] : 0.0;
        J.R[gi] = J.rscale * (f - accv);
      }
    };

    double acc[P];
#pragma unroll
    for (int a = 0; a < P; ++a) acc[a] = 0.0;

    const int ez0 = max(0, Z0 - p);
    const int ez1 = min(Ez - 1, Zend - 1);
    for (int cz = ez0; cz <= ez0 + p; ++cz) load_layer(cz);
    __syncthreads();

    const double* tzg = J.tab[2];
    for (int ez = ez0; ez <= ez1; ++ez) {
      for (int gz = 0; gz < Q; ++gz) {
        double nz[P], dz[P];
#pragma unroll
        for (int a = 0; a < P; ++a) {
          nz[a] = tzg[((long long)ez * Q + gz) * P + a];
          dz[a] = tzg[(long long)Ez * Q * P + ((long long)ez * Q + gz) * P + a];
        }
        const double wz = tzg[2ll * Ez * Q * P + (long long)ez * Q + gz];
        // S1: z-contraction on the halo column grid
        for (int k = tid; k < TYH * TXH; k += NT) {
          int cyl = k / TXH, cxl = k - cyl * TXH;
          double A = 0.0, B = 0.0;
          const double r0 = ring[ez % P][cyl][cxl];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            double r = ring[(ez + a) % P][cyl][cxl];
            A = fma(nz[a], r, A);
            B = fma(dz[a], r - r0, B);   // sum_a dz[a] = 0: contract differences
          }
          Ab[cyl][cxl] = A;
          Bb[cyl][cxl] = B;
        }
        __syncthreads();
        // S2: y-contraction to the Gauss rows of the tile's y-elements
        for (int k = tid; k < EY * TXH; k += NT) {
          int eyl = k / TXH, cxl = k - eyl * TXH;
          double av[P], bv[P];
#pragma unroll
          for (int b = 0; b < P; ++b) {
            av[b] = Ab[eyl + b][cxl];
            bv[b] = Bb[eyl + b][cxl];
          }
#pragma unroll
          for (int gy = 0; gy < Q; ++gy) {
            double c = 0.0, dyv = 0.0, dzv = 0.0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
              c = fma(tyN[eyl][gy][b], av[b], c);
              dyv = fma(tyD[eyl][gy][b], av[b] - av[0], dyv);
              dzv = fma(tyN[eyl][gy][b], bv[b], dzv);
            }
            S[0][eyl * Q + gy][cxl] = c;
            S[1][eyl * Q + gy][cxl] = dyv;
            S[2][eyl * Q + gy][cxl] = dzv;
          }
        }
        __syncthreads();
        // S34: x-forward, weights, x-backward; lanes are x-elements
        for (int r = rg; r < R; r += 16) {
          const int eyl = r / Q, gy = r - eyl * Q;
          const double wyz = tyW[eyl][gy] * wz;
          double c0[P], c1[P], c2[P];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            c0[a] = S[0][r][j + a];
            c1[a] = S[1][r][j + a];
            c2[a] = S[2][r][j + a];
          }
          double o0[P], o1[P], o2[P];
#pragma unroll
          for (int a = 0; a < P; ++a) o0[a] = o1[a] = o2[a] = 0.0;
#pragma unroll
          for (int gx = 0; gx < Q; ++gx) {
            double gX = 0.0, gY = 0.0, gZ = 0.0;
#pragma unroll
            for (int a = 0; a < P; ++a) {
              gX = fma(xD[gx][a], c0[a] - c0[0], gX);
              gY = fma(xN[gx][a], c1[a], gY);
              gZ = fma(xN[gx][a], c2[a], gZ);
            }
            const double w = xW[gx] * wyz;
            gX *= w;
            gY *= w;
            gZ *= w;
#pragma unroll
            for (int a = 0; a < P; ++a) {
              o0[a] = fma(xD[gx][a], gX, o0[a]);
              o1[a] = fma(xN[gx][a], gY, o1[a]);
              o2[a] = fma(xN[gx][a], gZ, o2[a]);
            }
          }
          // coefficient c = ex collects slot a of element ex - a (lane j - a)
          double r0 = o0[0], r1 = o1[0], r2 = o2[0];
#pragma unroll
          for (int a = 1; a < P; ++a) {
            r0 += __shfl_up(o0[a], a, 16);
            r1 += __shfl_up(o1[a], a, 16);
            r2 += __shfl_up(o2[a], a, 16);
          }
          if (j >= p) {
            S[0][r][j - p] = r0;
            S[1][r][j - p] = r1;
            S[2][r][j - p] = r2;
          }
        }
        __syncthreads();
        // S5: y-backward and z-backward into the owned column's accumulators
        if (own) {
          double Ap = 0.0, Bp = 0.0;
#pragma unroll
          for (int b = 0; b < P; ++b) {
            const int eyl = cyo + p - b;
#pragma unroll
            for (int gy = 0; gy < Q; ++gy) {
              const int rr = eyl * Q + gy;
              Ap = fma(tyN[eyl][gy][b], S[0][rr][cxo], Ap);
              Ap = fma(tyD[eyl][gy][b], S[1][rr][cxo], Ap);
              Bp = fma(tyN[eyl][gy][b], S[2][rr][cxo], Bp);
            }
          }
#pragma unroll
          for (int a = 0; a < P; ++a) acc[a] = fma(nz[a], Ap, fma(dz[a], Bp, acc[a]));
        }
      }
      if (own) store_out(ez, acc[0]);
#pragma unroll
      for (int a = 0; a < P - 1; ++a) acc[a] = acc[a + 1];
      acc[P - 1] = 0.0;
      if (ez < ez1) load_layer(ez + P);
      __syncthreads();
    }
    if (own) {
#pragma unroll
      for (int a = 0; a < P - 1; ++a) store_out(ez1 + 1 + a, acc[a]);
    }
    __syncthreads();
  }
}

int rhs_tile_x(int p) { return 16 - p; }
int rhs_tile_y(int) { return 16; }

hipError_t launch_rhs_pwave(int p, const RhsJob* d_jobs, int njobs, int total_tiles, int grid_cap,
                            hipStream_t s) {
  int grid = total_tiles;
  if (grid_cap > 0 && grid > grid_cap) grid = grid_cap;
  if (grid <= 0) return hipSuccess;
  if (p == 2) {
    hipLaunchKernelGGL((rhs_pwave_kernel<3, 3>), dim3(grid), dim3(256), 0, s, d_jobs, njobs, total_tiles);
  } else if (p == 3) {
    hipLaunchKernelGGL((rhs_pwave_kernel<4, 4>), dim3(grid), dim3(256), 0, s, d_jobs, njobs, total_tiles);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ads
