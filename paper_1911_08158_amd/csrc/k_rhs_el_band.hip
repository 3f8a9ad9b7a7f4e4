// Right-hand side of the elasticity step in the Kronecker form of the
// operator Upsilon (Section 5, the bilinear form 2 mu (eps(w), eps(u)) +
// lambda (div w, div u) with constant Lame parameters):
//
//   R_i = rscale * ( amp * b_i - sum_k Upsilon_ik U_k ),
//   Upsilon_ii = (2mu+lambda) K_i (x) M (x) M + mu (K_j + K_k terms),
//   Upsilon_ik = mu G_i (x) G_k^T (x) M_j + lambda G_i^T (x) G_k (x) M_j,
//
// each factor a 1D band matrix of width 2p+1 over the free coefficients
// (M mass, K stiffness, G mixed (B_a, B'_c) and its transpose G^T, placed
// in the directions named by their index).  Every term is a product of
// three 1D band passes; the kernel shares them: per source component c the
// x-pass forms four channels M_x U_c, K_x U_c, G_x U_c, G^T_x U_c (twelve
// in all); the y-pass combines them into twelve channels, one per output
// component and z-factor (M_z, K_z, G_z, G^T_z); the z-band scatters them
// into 2p+1 FP64 accumulators per output component.  About 85 multiply-adds
// per component DOF against thousands of the element quadrature: the kernel
// is bound by memory (three fields in, three out).
//
// Tiling as the P-wave's Kronecker-form kernel: a workgroup owns ETX x ETY
// columns and a z-range, and marches over the source layers that reach it;
// per layer the three components with a p-halo in x and y go to LDS (the
// loads of the next one or two layers in flight), the x-pass runs over the halo
// rows (one thread per column), the y-pass
// gives each owned column its twelve channels (band rows from LDS: x-rows
// lane-consecutive, y-rows broadcast within a wave), and the z-band entries of the layer arrive as
// one vector load per wave, read back by readlane.  Each output is computed
// by one thread; no atomics.
//
// Precision: T is the type of the passes with K, G or G^T (double, or float
// in mixed mode).  Those bands act on differences to the centre value (the
// x and y tables hold the row sum in the diagonal slot), so that rounded
// entries still annihilate constants; the differences are formed in the
// channel's own type (FP64 for the components and the mass channels).  The
// mass channels M_x U_c, M_y M_x U_c, the z-pass, the accumulators and the
// output are FP64.
#include "common.hpp"
#include "launch.hpp"

namespace ads {

constexpr int ETX = 32;

// Owned rows per tile: 8 (256 threads), 4 for p >= 4 (128 threads), which
// keeps the static LDS of the FP64 kernel within 64 KiB.
template <int p>
struct ElBandGeom {
  static constexpr int ETY = p >= 4 ? 4 : 8;
  static constexpr int ENT = ETX * ETY;
  static constexpr int B = 2 * p + 1;
  static constexpr int DEPTH = p <= 2 ? 2 : 1;   // source layers whose loads are in flight
  static constexpr int SX = ETX + 2 * p, SY = ETY + 2 * p;
  static constexpr int NS = (SY * SX + ENT - 1) / ENT;    // loads per thread, component and layer
  static constexpr int NXI = (SY * ETX + ENT - 1) / ENT;  // x-pass items per thread
};

__device__ __forceinline__ int find_job_elb(const RhsJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Band matrices of direction d (RhsJob::band[d]): M, K, G, G^T, each
// [nf][2p+1] with entry (i, j) at i*(2p+1) + (j - i + p); in x and y the
// diagonal slots of K, G and G^T hold their row sums.
template <int p>
__device__ __forceinline__ const double* el_band_table(const double* band, int nf, int op) {
  return band + (long long)op * nf * (2 * p + 1);
}

// Band row b applied in difference form to the column c (stride ETX):
// b[p] c[p] + sum_{k != p} b[k] (c[k] - c[p]), in T.
template <typename T, int p, typename C>
__device__ __forceinline__ T band_diff(const double* b, const C* c) {
  constexpr int B = 2 * p + 1;
  const C cc = c[p * ETX];
  T s = (T)b[p] * (T)cc;
#pragma unroll
  for (int k = 0; k < B; ++k)
    if (k != p) s = fma((T)b[k], (T)(c[k * ETX] - cc), s);
  return s;
}
// Mass band row on a column, in the column's type.
template <typename C, int p>
__device__ __forceinline__ C band_plain(const double* b, const C* c) {
  constexpr int B = 2 * p + 1;
  C s = (C)b[0] * c[0];
#pragma unroll
  for (int k = 1; k < B; ++k) s = fma((C)b[k], c[k * ETX], s);
  return s;
}

template <typename T, int p>
__global__ __launch_bounds__(ElBandGeom<p>::ENT, 2) void rhs_elastic_band_kernel(const LaunchHdr* __restrict__ hdr) {
  using Gm = ElBandGeom<p>;
  constexpr int B = Gm::B, SX = Gm::SX, SY = Gm::SY, NS = Gm::NS, NXI = Gm::NXI;
  constexpr int ETY = Gm::ETY, ENT = Gm::ENT, kDepthE = Gm::DEPTH;
  __shared__ double Wl[3][SY * SX];       // the three components of a source layer, with halos
  __shared__ double XM[3][SY * ETX];      // M_x U_c
  __shared__ T XK[3][SY * ETX];           // K_x U_c
  __shared__ T XG[3][SY * ETX];           // G_x U_c
  __shared__ T XT[3][SY * ETX];           // G^T_x U_c
  __shared__ double Xb[4][B][ETX];        // x-band rows M, K, G, G^T of the tile's columns
  __shared__ double Yb[4][ETY][B];        // y-band rows M, K, G, G^T of the tile's rows
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const RhsJob* __restrict__ jobs = hdr_jobs<RhsJob>(hdr);
  const int tid = threadIdx.x, lx = tid % ETX, ly = tid / ETX;

  // XCD-contiguous tile ranges (block b runs on XCD b mod 8; neighbouring
  // tiles share halo rows in that XCD's L2)
  const int full = total_tiles & ~7;
  for (int wi = blockIdx.x; wi < total_tiles; wi += gridDim.x) {
    const int tile = wi >= full ? wi : (wi & 7) * (full >> 3) + (wi >> 3);
    const RhsJob& J = jobs[find_job_elb(jobs, njobs, tile)];
    const int t = tile - J.tile0;
    const int tx = t % J.tiles[0];
    const int t2 = t / J.tiles[0];
    const int ty = t2 % J.tiles[1];
    const int tz = t2 / J.tiles[1];
    const int nfx = J.nf[0], nfy = J.nf[1], nfz = J.nf[2];
    const int x0 = tx * ETX, y0 = ty * ETY, Z0 = tz * J.TZ;
    const int Zend = min(Z0 + J.TZ, nfz);
    const long long sxy = (long long)nfx * nfy;
    const long long nfree = sxy * nfz;
    const gmem<double>* __restrict__ U = gview(J.u);
    const gmem<double>* __restrict__ LD = gview(J.load);
    gmem<double>* __restrict__ R = gview(J.R);
    const double rscale = J.rscale;
    const double mu = J.mu, lam = J.lam, c2 = 2.0 * J.mu + J.lam;

    // band rows of the tile's columns (x) and rows (y) in LDS, zero beyond
    // the field; read after the first barrier of the first layer
    for (int k = tid; k < 4 * B * ETX; k += ENT) {
      const int op = k / (B * ETX), r = k - op * (B * ETX);
      const int c = r / ETX, col = r - c * ETX;
      const int gx = x0 + col;
      (&Xb[0][0][0])[k] = gx < nfx ? gview(el_band_table<p>(J.band[0], nfx, op))[(long long)gx * B + c] : 0.0;
    }
    for (int k = tid; k < 4 * ETY * B; k += ENT) {
      const int op = k / (ETY * B), r = k - op * (ETY * B);
      const int row = r / B, c = r - row * B;
      const int gy = y0 + row;
      (&Yb[0][0][0])[k] = gy < nfy ? gview(el_band_table<p>(J.band[1], nfy, op))[(long long)gy * B + c] : 0.0;
    }
    // z-band entries of a source layer s: lane op*B + k holds factor op's
    // entry (s-p+k, s), op = M, K, G, G^T (zero outside the free range)
    const int zlane = threadIdx.x & 63;
    const int zop = zlane / B, zk = zlane - zop * B;
    const gmem<double>* bzg = gview(el_band_table<p>(J.band[2], nfz, zop < 4 ? zop : 0));
    double ampv = 0.0;
    if (J.load != nullptr && J.amp != nullptr) {
      long long ai = (long long)(*gview(J.counter)) + J.amp_shift;
      ampv = (ai >= 0 && ai < J.namp) ? gview(J.amp)[ai] : 0.0;
    }

    long long prow[NS];
    bool pval[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int k = tid + i * ENT;
      const int r = k / SX, c = k - r * SX;
      const int gy = y0 - p + r, gxx = x0 - p + c;
      pval[i] = k < SY * SX && gy >= 0 && gy < nfy && gxx >= 0 && gxx < nfx;
      prow[i] = pval[i] ? (long long)gy * nfx + gxx : 0;
    }
    const bool own = x0 + lx < nfx && y0 + ly < nfy;
    const long long ocol = own ? (long long)(y0 + ly) * nfx + (x0 + lx) : 0;

    double pf[kDepthE][3][NS];
    double pzb[kDepthE];
    // loads only: nothing consumes them before the layer is committed (the
    // z-band entry outside the free range is replaced by zero then), so that
    // they stay in flight meanwhile
    auto zband_ok = [&](int s) {
      const int o = s - p + zk;
      return zlane < 4 * B && o >= 0 && o < nfz;
    };
    auto prefetch = [&](int s, double (&pf)[3][NS], double& pz) {
      {
        const int o = s - p + zk;
        pz = bzg[zband_ok(s) ? (long long)o * B + (2 * p - zk) : 0];
      }
      const long long zo = (long long)s * sxy;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < NS; ++i) pf[c][i] = U[c * nfree + (pval[i] ? zo + prow[i] : 0)];
    };
    auto commit = [&](const double (&pf)[3][NS]) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int k = tid + i * ENT;
          if (k < SY * SX) Wl[c][k] = pval[i] ? pf[c][i] : 0.0;
        }
    };
    // output o of component c (the load vector is read here: one value per
    // output, off the critical path of the layers)
    auto store = [&](int o, int c, double a) {
      if (own && o >= Z0 && o < Zend) {
        const long long go = c * nfree + (long long)o * sxy + ocol;
        const double ld = LD != nullptr ? LD[go] : 0.0;
        R[go] = rscale * (ampv * ld - a);
      }
    };

    double acc[3][B];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < B; ++k) acc[c][k] = 0.0;

    auto process = [&](int s, double zbv) {
      __syncthreads();
      // x-pass: four channels per component over the halo rows; each band
      // entry is read once for the three components
#pragma unroll 1
      for (int i = 0; i < NXI; ++i) {
        const int r = ly + i * (ENT / ETX);
        if (r < SY) {
          double wc[3], am[3];
          T ak[3], ag[3], at[3];
          const double bmp = Xb[0][p][lx], bkp = Xb[1][p][lx], bgp = Xb[2][p][lx], btp = Xb[3][p][lx];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            wc[c] = Wl[c][r * SX + lx + p];
            am[c] = bmp * wc[c];
            ak[c] = (T)bkp * (T)wc[c];
            ag[c] = (T)bgp * (T)wc[c];
            at[c] = (T)btp * (T)wc[c];
          }
#pragma unroll
          for (int k = 0; k < B; ++k) {
            if (k == p) continue;
            const double bm = Xb[0][k][lx];
            const T bk = (T)Xb[1][k][lx], bg = (T)Xb[2][k][lx], bt = (T)Xb[3][k][lx];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double w = Wl[c][r * SX + lx + k];
              const T d = (T)(w - wc[c]);
              am[c] = fma(bm, w, am[c]);
              ak[c] = fma(bk, d, ak[c]);
              ag[c] = fma(bg, d, ag[c]);
              at[c] = fma(bt, d, at[c]);
            }
          }
          const int o = r * ETX + lx;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            XM[c][o] = am[c];
            XK[c][o] = ak[c];
            XG[c][o] = ag[c];
            XT[c][o] = at[c];
          }
        }
      }
      __syncthreads();
      // y-pass of the owned column, one output component at a time: its
      // channels for the z-factors M, K, G, G^T, scattered at once by the
      // layer's z-band entries
      const int co = ly * ETX + lx;
      const double* yM = Yb[0][ly];
      const double* yK = Yb[1][ly];
      const double* yG = Yb[2][ly];
      const double* yT = Yb[3][ly];
      const long long zbb = __double_as_longlong(zbv);
      const int zlo = (int)(zbb & 0xffffffffll), zhi = (int)(zbb >> 32);
      auto lane_d = [&](int l) {
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane(zlo, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane(zhi, l);
        return __longlong_as_double(((long long)hi << 32) | lo);
      };
      auto scatter = [&](double (&a)[B], double zm, double zkk, double zg, double zt) {
#pragma unroll
        for (int k = 0; k < B; ++k)
          a[k] = fma(lane_d(k), zm, fma(lane_d(B + k), zkk, fma(lane_d(2 * B + k), zg, fma(lane_d(3 * B + k), zt, a[k]))));
      };
      {
        const T zm = (T)c2 * band_plain<T, p>(yM, &XK[0][co]) + (T)mu * band_diff<T, p>(yK, &XM[0][co]) +
                     (T)mu * band_diff<T, p>(yT, &XG[1][co]) + (T)lam * band_diff<T, p>(yG, &XT[1][co]);
        const double zkk = mu * band_plain<double, p>(yM, &XM[0][co]);
        const T zt = (T)mu * band_plain<T, p>(yM, &XG[2][co]);
        const T zg = (T)lam * band_plain<T, p>(yM, &XT[2][co]);
        scatter(acc[0], (double)zm, zkk, (double)zg, (double)zt);
      }
      {
        const T zm = (T)c2 * band_diff<T, p>(yK, &XM[1][co]) + (T)mu * band_plain<T, p>(yM, &XK[1][co]) +
                     (T)mu * band_diff<T, p>(yG, &XT[0][co]) + (T)lam * band_diff<T, p>(yT, &XG[0][co]);
        const double zkk = mu * band_plain<double, p>(yM, &XM[1][co]);
        const T zt = (T)mu * band_diff<T, p>(yG, &XM[2][co]);
        const T zg = (T)lam * band_diff<T, p>(yT, &XM[2][co]);
        scatter(acc[1], (double)zm, zkk, (double)zg, (double)zt);
      }
      {
        const T zm = (T)mu * (band_plain<T, p>(yM, &XK[2][co]) + band_diff<T, p>(yK, &XM[2][co]));
        const double zkk = c2 * band_plain<double, p>(yM, &XM[2][co]);
        const T zg = (T)mu * (band_plain<T, p>(yM, &XT[0][co]) + band_diff<T, p>(yT, &XM[1][co]));
        const T zt = (T)lam * (band_plain<T, p>(yM, &XG[0][co]) + band_diff<T, p>(yG, &XM[1][co]));
        scatter(acc[2], (double)zm, zkk, (double)zg, (double)zt);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        store(s - p, c, acc[c][0]);
#pragma unroll
        for (int k = 0; k < B - 1; ++k) acc[c][k] = acc[c][k + 1];
        acc[c][B - 1] = 0.0;
      }
    };

    const int sb = max(0, Z0 - p), se = min(nfz - 1, Zend - 1 + p);
#pragma unroll
    for (int d = 0; d < kDepthE; ++d)
      if (sb + d <= se) prefetch(sb + d, pf[d], pzb[d]);
    for (int s0 = sb; s0 <= se; s0 += kDepthE) {
#pragma unroll
      for (int d = 0; d < kDepthE; ++d) {
        const int s = s0 + d;
        if (s > se) break;
        commit(pf[d]);
        const double zbv = zband_ok(s) ? pzb[d] : 0.0;
        if (s + kDepthE <= se) prefetch(s + kDepthE, pf[d], pzb[d]);
        process(s, zbv);
      }
    }
    // outputs se - p + 1 .. se + p
#pragma unroll
    for (int k = 0; k < B - 1; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) store(se - p + 1 + k, c, acc[c][k]);
    __syncthreads();
  }
}

template <typename T, int p>
static hipError_t elb_one(const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  constexpr int ENT = ElBandGeom<p>::ENT;
  if (op == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)rhs_elastic_band_kernel<T, p>, ENT, 0);
  hipLaunchKernelGGL((rhs_elastic_band_kernel<T, p>), dim3(grid), dim3(ENT), 0, s, d_hdr);
  return hipGetLastError();
}

template <int p>
static hipError_t elb_p(int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  return mixed ? elb_one<float, p>(d_hdr, grid, s, op, out) : elb_one<double, p>(d_hdr, grid, s, op, out);
}

static hipError_t elb_dispatch(int p, int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  switch (p) {
    case 1: return elb_p<1>(mixed, d_hdr, grid, s, op, out);
    case 2: return elb_p<2>(mixed, d_hdr, grid, s, op, out);
    case 3: return elb_p<3>(mixed, d_hdr, grid, s, op, out);
    case 4: return elb_p<4>(mixed, d_hdr, grid, s, op, out);
    case 5: return elb_p<5>(mixed, d_hdr, grid, s, op, out);
    default: return hipErrorInvalidValue;
  }
}

int rhs_el_band_tile_x() { return ETX; }
int rhs_el_band_tile_y(int p) { return p >= 4 ? ElBandGeom<4>::ETY : ElBandGeom<2>::ETY; }

hipError_t launch_rhs_elastic_band(int p, int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  return elb_dispatch(p, mixed, d_hdr, grid, s, 0, nullptr);
}

int rhs_el_band_blocks_per_cu(int p, int mixed) {
  int n = 1;
  (void)elb_dispatch(p, mixed, nullptr, 0, nullptr, 1, &n);
  return n < 1 ? 1 : n;
}

}  // namespace ads
