// Right-hand side of the P-wave step by sum-factorized Gauss quadrature
// (Section 2: testing the equation gives (grad B_i, grad w_h) for the
// stiffness action, written as K = K_x(x)M_y(x)M_z + ... in eq. pwave2; here
// it is evaluated element by element at the q^3 Gauss points as a chain of
// 1D contractions instead of assembling K):
//
//   R_i = rscale * ( amp * b_i - sum_e sum_g W_g grad B_i(x_g) . grad w_h(x_g) ),
//   w   = cu*u + cv*v + ca*a   (the Newmark predictor u + tau u' + tau^2/4 u'').
//
// Tiling on gfx950 (owner computes, no atomics, deterministic):
//   * a workgroup owns TX x TY coefficient columns and a z-range of TZ
//     coefficients, and marches over the element layers touching the range;
//   * per element layer the predictor w is formed once (FP64) into an LDS
//     ring of p+1 coefficient layers (halo p on each side in x and y);
//   * per z Gauss point: (S12) z- and y-contraction from the ring to the
//     y Gauss rows of the tile's y-elements (values, y- and z-derivatives),
//     (S34) x-forward, quadrature weight and x-backward with one lane per
//     x-element (16-lane DPP rows, one Gauss row each) and a row-shift
//     add that assembles each coefficient from its p+1 elements, (S5)
//     y-backward and z-backward into FP64 accumulators of the owned column
//     (p+1 z-layers in flight);
//   * the Gauss-row buffer is double-buffered: two barriers per z Gauss
//     point;
//   * a z-layer is written once its last contributing element is done.
// T is the contraction type: double (FP64 mode) or float (mixed mode: FP32
// contractions, FP64 predictor, FP64 z-accumulation and assembly).
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

// Row shift within 16-lane DPP rows: lane i receives lane i-K (0 if none).
template <int K>
__device__ __forceinline__ double row_shr(double x) {
  long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x110 + K, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x110 + K, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int K>
__device__ __forceinline__ float row_shr(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + K, 0xF, 0xF, false));
}

template <typename T, int P, int Q, int TY_, int NT_>
struct RhsGeom {
  static constexpr int p = P - 1;
  static constexpr int G = 16;          // lanes per Gauss row (x-elements of the tile)
  static constexpr int TX = G - p;      // owned x-coefficients
  static constexpr int TY = TY_;        // owned y-coefficients
  static constexpr int TXH = TX + 2 * p;
  static constexpr int TYH = TY + 2 * p;
  static constexpr int EY = TY + p;     // y-elements touching the owned columns
  static constexpr int R = EY * Q;      // y Gauss rows
  static constexpr int NT = NT_;
  static constexpr int NRG = NT / G;    // Gauss-row groups
  static constexpr size_t lds_elems = (size_t)P * TYH * TXH + 2ull * 3 * R * TXH + 2ull * EY * Q * P + EY * Q;
  static constexpr size_t lds_bytes = lds_elems * sizeof(T);
};

template <int K, int P, typename T>
__device__ __forceinline__ T shift_sum(const T (&o)[P]) {
  if constexpr (K >= P) {
    return T(0);
  } else {
    return row_shr<K>(o[K]) + shift_sum<K + 1, P, T>(o);
  }
}

template <typename T, int P, int Q, int TY_, int NT_>
__global__ __launch_bounds__(NT_) void rhs_pwave_kernel(const LaunchHdr* __restrict__ hdr) {
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const RhsJob* __restrict__ jobs = hdr_jobs<RhsJob>(hdr);
  using Gm = RhsGeom<T, P, Q, TY_, NT_>;
  constexpr int p = Gm::p, TX = Gm::TX, TY = Gm::TY, TXH = Gm::TXH, TYH = Gm::TYH, EY = Gm::EY,
                R = Gm::R, NT = Gm::NT, NRG = Gm::NRG;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ring = reinterpret_cast<T*>(smem_raw);            // [P][TYH][TXH]
  T* Sb = ring + P * TYH * TXH;                         // [2][3][R][TXH]
  T* tyN = Sb + 2 * 3 * R * TXH;                        // [EY][Q][P]
  T* tyD = tyN + EY * Q * P;                            // [EY][Q][P]
  T* tyW = tyD + EY * Q * P;                            // [EY][Q]
  auto RING = [&](int s, int y, int x) -> T& { return ring[(s * TYH + y) * TXH + x]; };
  auto SB = [&](int b, int c, int r, int x) -> T& { return Sb[((b * 3 + c) * R + r) * TXH + x]; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int j = lane & 15;                 // x-element slot within the Gauss row group
  const int rg = tid >> 4;                 // Gauss row group
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
      tyN[k] = v ? (T)tyg[(long long)ey * Q * P + rest] : T(0);
      tyD[k] = v ? (T)tyg[(long long)Ey * Q * P + (long long)ey * Q * P + rest] : T(0);
    }
    for (int k = tid; k < EY * Q; k += NT) {
      int eyl = k / Q, g = k - eyl * Q;
      int ey = Y0 - p + eyl;
      tyW[k] = (ey >= 0 && ey < Ey) ? (T)tyg[2ll * Ey * Q * P + (long long)ey * Q + g] : T(0);
    }
    // x tables of this lane's x-element, kept in registers
    const int ex = X0 - p + j;
    const bool exv = ex >= 0 && ex < Ex;
    T xN[Q][P], xD[Q][P], xW[Q];
    {
      const double* txg = J.tab[0];
#pragma unroll
      for (int g = 0; g < Q; ++g) {
#pragma unroll
        for (int a = 0; a < P; ++a) {
          xN[g][a] = exv ? (T)txg[((long long)ex * Q + g) * P + a] : T(0);
          xD[g][a] = exv ? (T)txg[(long long)Ex * Q * P + ((long long)ex * Q + g) * P + a] : T(0);
        }
        xW[g] = exv ? (T)txg[2ll * Ex * Q * P + (long long)ex * Q + g] : T(0);
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
        RING(slot, cyl, cxl) = (T)w;
      }
    };
    // next-layer prefetch: global loads issued one layer ahead, written to
    // the ring after the last z Gauss point of the current layer
    constexpr int NPF = (TYH * TXH + NT - 1) / NT;
    double pf[NPF];
    auto prefetch_layer = [&](int cz) {
      const bool zv = cz >= oz && cz < oz + nfz;
#pragma unroll
      for (int i = 0; i < NPF; ++i) {
        const int k = tid + i * NT;
        double w = 0.0;
        if (k < TYH * TXH) {
          int cyl = k / TXH, cxl = k - cyl * TXH;
          int cy = Y0 - p + cyl, cx = X0 - p + cxl;
          if (zv && cy >= oy && cy < oy + nfy && cx >= ox && cx < ox + nfx) {
            long long gi = (long long)(cz - oz) * sxy + (long long)(cy - oy) * nfx + (cx - ox);
            w = J.cu * J.u[gi];
            if (J.v != nullptr) w = fma(J.cv, J.v[gi], w);
            if (J.a != nullptr) w = fma(J.ca, J.a[gi], w);
          }
        }
        pf[i] = w;
      }
    };
    auto commit_layer = [&](int cz) {
      const int slot = cz % P;
#pragma unroll
      for (int i = 0; i < NPF; ++i) {
        const int k = tid + i * NT;
        if (k < TYH * TXH) ring[slot * TYH * TXH + k] = (T)pf[i];
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
    int buf = 0;
    for (int ez = ez0; ez <= ez1; ++ez) {
      if (ez < ez1) prefetch_layer(ez + P);
      for (int gz = 0; gz < Q; ++gz) {
        T nz[P], dz[P];
#pragma unroll
        for (int a = 0; a < P; ++a) {
          nz[a] = (T)tzg[((long long)ez * Q + gz) * P + a];
          dz[a] = (T)tzg[(long long)Ez * Q * P + ((long long)ez * Q + gz) * P + a];
        }
        const T wz = (T)tzg[2ll * Ez * Q * P + (long long)ez * Q + gz];
        // S12: z- then y-contraction, straight from the coefficient ring
        for (int k = tid; k < EY * TXH; k += NT) {
          const int eyl = k / TXH, cxl = k - eyl * TXH;
          T av[P], bv[P];
#pragma unroll
          for (int b = 0; b < P; ++b) {
            const T r0 = RING(ez % P, eyl + b, cxl);
            T A = T(0), B = T(0);
#pragma unroll
            for (int a = 0; a < P; ++a) {
              const T r = RING((ez + a) % P, eyl + b, cxl);
              A = fma(nz[a], r, A);
              B = fma(dz[a], r - r0, B);     // sum_a dz[a] = 0: contract differences
            }
            av[b] = A;
            bv[b] = B;
          }
          const T* tN = tyN + eyl * Q * P;
          const T* tD = tyD + eyl * Q * P;
#pragma unroll
          for (int gy = 0; gy < Q; ++gy) {
            T c = T(0), dyv = T(0), dzv = T(0);
#pragma unroll
            for (int b = 0; b < P; ++b) {
              c = fma(tN[gy * P + b], av[b], c);
              dyv = fma(tD[gy * P + b], av[b] - av[0], dyv);
              dzv = fma(tN[gy * P + b], bv[b], dzv);
            }
            SB(buf, 0, eyl * Q + gy, cxl) = c;
            SB(buf, 1, eyl * Q + gy, cxl) = dyv;
            SB(buf, 2, eyl * Q + gy, cxl) = dzv;
          }
        }
        __syncthreads();
        // S34: x-forward, weights, x-backward; lanes are x-elements
        for (int r = rg; r < R; r += NRG) {
          const T wyz = tyW[r] * wz;
          T c0[P], c1[P], c2[P];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            c0[a] = SB(buf, 0, r, j + a);
            c1[a] = SB(buf, 1, r, j + a);
            c2[a] = SB(buf, 2, r, j + a);
          }
          T o0[P], o1[P], o2[P];
#pragma unroll
          for (int a = 0; a < P; ++a) o0[a] = o1[a] = o2[a] = T(0);
#pragma unroll
          for (int gx = 0; gx < Q; ++gx) {
            T gX = T(0), gY = T(0), gZ = T(0);
#pragma unroll
            for (int a = 0; a < P; ++a) {
              gX = fma(xD[gx][a], c0[a] - c0[0], gX);
              gY = fma(xN[gx][a], c1[a], gY);
              gZ = fma(xN[gx][a], c2[a], gZ);
            }
            const T w = xW[gx] * wyz;
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
          const T r0v = o0[0] + shift_sum<1, P, T>(o0);
          const T r1v = o1[0] + shift_sum<1, P, T>(o1);
          const T r2v = o2[0] + shift_sum<1, P, T>(o2);
          if (j >= p) {
            SB(buf, 0, r, j - p) = r0v;
            SB(buf, 1, r, j - p) = r1v;
            SB(buf, 2, r, j - p) = r2v;
          }
        }
        // refill the ring slot of layer ez once every z Gauss point has read it
        if (gz == Q - 1 && ez < ez1) commit_layer(ez + P);
        __syncthreads();
        // S5: y-backward and z-backward into the owned column's accumulators
        if (own) {
          T Ap = T(0), Bp = T(0);
#pragma unroll
          for (int b = 0; b < P; ++b) {
            const int eyl = cyo + p - b;
            const T* tN = tyN + eyl * Q * P;
            const T* tD = tyD + eyl * Q * P;
#pragma unroll
            for (int gy = 0; gy < Q; ++gy) {
              const int rr = eyl * Q + gy;
              Ap = fma(tN[gy * P + b], SB(buf, 0, rr, cxo), Ap);
              Ap = fma(tD[gy * P + b], SB(buf, 1, rr, cxo), Ap);
              Bp = fma(tN[gy * P + b], SB(buf, 2, rr, cxo), Bp);
            }
          }
#pragma unroll
          for (int a = 0; a < P; ++a)
            acc[a] = fma((double)nz[a], (double)Ap, fma((double)dz[a], (double)Bp, acc[a]));
        }
        buf ^= 1;
      }
      if (own) store_out(ez, acc[0]);
#pragma unroll
      for (int a = 0; a < P - 1; ++a) acc[a] = acc[a + 1];
      acc[P - 1] = 0.0;
    }
    if (own) {
#pragma unroll
      for (int a = 0; a < P - 1; ++a) store_out(ez1 + 1 + a, acc[a]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// variants (tile height, workgroup size) per degree and arithmetic
struct RhsVariant {
  int TY, NT;
};
// index: variant id; the autotuner in api.cpp times them on the real mesh
static const RhsVariant kVarP2[] = {{14, 256}, {30, 512}, {46, 768}};
static const RhsVariant kVarP3[] = {{13, 256}, {29, 512}, {21, 384}};

int rhs_num_variants(int) { return 3; }
int rhs_tile_x(int p) { return 16 - p; }
int rhs_tile_y(int p, int var) { return p == 2 ? kVarP2[var].TY : kVarP3[var].TY; }

// op 0: launch; op 1: *out = resident workgroups per CU (persistent grids)
template <typename T, int P, int TY, int NT>
static hipError_t launch_one(const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  using Gm = RhsGeom<T, P, P, TY, NT>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)rhs_pwave_kernel<T, P, P, TY, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm::lds_bytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (op == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)rhs_pwave_kernel<T, P, P, TY, NT>, NT,
                                                        Gm::lds_bytes);
  hipLaunchKernelGGL((rhs_pwave_kernel<T, P, P, TY, NT>), dim3(grid), dim3(NT), Gm::lds_bytes, s, d_hdr);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(int p, int var, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  if (p == 2) {
    switch (var) {
      case 0: return launch_one<T, 3, 14, 256>(d_hdr, grid, s, op, out);
      case 1: return launch_one<T, 3, 30, 512>(d_hdr, grid, s, op, out);
      default: return launch_one<T, 3, 46, 768>(d_hdr, grid, s, op, out);
    }
  }
  switch (var) {
    case 0: return launch_one<T, 4, 13, 256>(d_hdr, grid, s, op, out);
    case 1: return launch_one<T, 4, 29, 512>(d_hdr, grid, s, op, out);
    default: return launch_one<T, 4, 21, 384>(d_hdr, grid, s, op, out);
  }
}

hipError_t launch_rhs_pwave(int p, int mixed, int var, const LaunchHdr* d_hdr, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (p != 2 && p != 3) return hipErrorInvalidValue;
  if (var < 0 || var > 2) var = 0;
  return mixed ? launch_t<float>(p, var, d_hdr, grid, s, 0, nullptr)
               : launch_t<double>(p, var, d_hdr, grid, s, 0, nullptr);
}

int rhs_blocks_per_cu(int p, int mixed, int var) {
  int n = 1;
  if (mixed) launch_t<float>(p, var, nullptr, 0, nullptr, 1, &n);
  else launch_t<double>(p, var, nullptr, 0, nullptr, 1, &n);
  return n < 1 ? 1 : n;
}

}  // namespace ads
