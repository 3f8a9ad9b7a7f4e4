// Right-hand side of the P-wave step without a wave-speed field, in the
// Kronecker form of the stiffness matrix (Section 2, eq. pwave2, in 3D):
// with constant coefficients the Galerkin stiffness is a sum of three
// tensor products of assembled 1D matrices of bandwidth 2p+1 (restricted
// to the free coefficients),
//
//   K = K_x(x)M_y(x)M_z + M_x(x)K_y(x)M_z + M_x(x)M_y(x)K_z,
//   R = rscale * ( amp * b - K w ),   w = cu*u + cv*v + ca*a,
//
// applied as three band passes with two channels each (the stiffness
// bands of the x- and y-passes in difference form, see band_table):
//   x:  X1 = K_x w,            X2 = M_x w
//   y:  YM = M_y X1 + K_y X2,  YK = M_y X2
//   z:  K w = M_z YM + K_z YK
// i.e. 7(2p+1) multiply-adds per coefficient, against the hundreds of the
// element quadrature; the 1D matrices are the same Gauss sums (exact for
// q = p+1), so the result is the quadrature's up to rounding.  The kernel
// is bound by HBM (three state fields in, one out).
//
// Tiling on gfx950: a workgroup owns BTX x BTY columns and a z-range of TZ
// outputs and marches over the source layers that reach them (TZ + 2p).
// Per source layer: the predictor of the layer with a p-halo in x and y
// (formed in FP64 from the three fields, coalesced rows) goes to LDS, the
// next kDepth layers' loads already in flight; the x-pass runs over the halo rows
// (LDS -> LDS, one thread per column, its band rows in registers); the
// y-pass gives each owned column its two channels, which the z-band
// scatters into 2p+1 FP64 accumulators (outputs s-p .. s+p of source
// layer s; the layer's z-band entries are one vector load per wave issued
// with its predictor, one entry per lane, broadcast by readlane, since
// scalar loads would share their wait counter with the LDS traffic).  The oldest
// accumulator is complete after each layer and is written.  Two barriers
// per layer, no atomics, each output computed by one thread.  Tiles are
// spread over the XCDs in contiguous ranges (halo re-reads hit the L2).
// T is the type of the x- and y-stiffness passes K_x w, K_y X2 and of
// M_y X1 (double, or float in mixed mode, on differences formed in FP64);
// the predictor, the mass channel X2 = M_x w and YK = M_y X2, the
// z-accumulation and the output are FP64.
#include "common.hpp"
#include "launch.hpp"

namespace ads {

constexpr int BTX = 32, BTY = 8, BNT = BTX * BTY;
constexpr int kDepth = 2;   // source layers whose loads are in flight

template <typename T, int p>
struct BandGeom {
  static constexpr int B = 2 * p + 1;
  static constexpr int P = p + 1;
  static constexpr int SX = BTX + 2 * p, SY = BTY + 2 * p;
  static constexpr int NS = (SY * SX + BNT - 1) / BNT;    // predictor loads per thread and layer
  static constexpr int NXI = (SY * BTX + BNT - 1) / BNT;  // x-pass items per thread
};

__device__ __forceinline__ int find_job_band(const RhsJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// x rounded to the nearest BF16 value (ties to even), as an FP32 value
__device__ __forceinline__ float bf16_round_band(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Assembled 1D matrices of direction d (RhsJob::band[d], after the element
// tables of that direction): M [nf][2p+1], then K [nf][2p+1]; entry (i, j)
// at i*(2p+1) + (j - i + p), zero where j leaves the free range.  In x and
// y the diagonal slot of K holds the row sum s_i instead, for the
// difference form
//   (K v)_i = s_i v_i + sum_{j != i} K_ij (v_j - v_i),
// in which FP32-rounded entries still annihilate constants (s_i is zero
// away from eliminated boundary coefficients); z keeps K (FP64 pass).

// waves per SIMD: four at p <= 2 (FP32 at five spills registers and runs
// slower), four (FP32) or three (FP64) at p = 3, two above
template <typename T, int p>
__global__ __launch_bounds__(BNT, p <= 2 ? 4 : (p == 3 ? (sizeof(T) == 4 ? 4 : 3) : 2)) void rhs_band_kernel(const LaunchHdr* __restrict__ hdr) {
  using Gm = BandGeom<T, p>;
  constexpr int B = Gm::B, SX = Gm::SX, SY = Gm::SY, NS = Gm::NS, NXI = Gm::NXI;
  // The predictor and the mass channel stay FP64 in every mode: a stiffness
  // band applied to differences of FP32-rounded values would turn their
  // rounding (relative to the values) into an error of the stiffness action
  // larger by about (wavelength / h)^2.  In mixed mode only the stiffness
  // passes K_x w and K_y X2, and M_y X1, run in FP32, on differences formed
  // in FP64.
  __shared__ double Wl[SY * SX];   // predictor layer with halos
  __shared__ T X1[SY * BTX];       // K_x w
  __shared__ double X2[SY * BTX];  // M_x w
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const RhsJob* __restrict__ jobs = hdr_jobs<RhsJob>(hdr);
  const int tid = threadIdx.x, lx = tid % BTX, ly = tid / BTX;

  // Workgroups are dispatched to the eight XCDs in turn (block b on XCD
  // b mod 8), each XCD with its own L2: work item w is mapped so that every
  // XCD takes one contiguous range of tiles (x fastest, then y, then the
  // z-chunk), whose neighbours share their halo rows in that L2.  The
  // remainder of total_tiles mod 8 keeps its order.
  const int full = total_tiles & ~7;
  for (int wi = blockIdx.x; wi < total_tiles; wi += gridDim.x) {
    const int tile = wi >= full ? wi : (wi & 7) * (full >> 3) + (wi >> 3);
    const RhsJob& J = jobs[find_job_band(jobs, njobs, tile)];
    const int t = tile - J.tile0;
    const int tx = t % J.tiles[0];
    const int t2 = t / J.tiles[0];
    const int ty = t2 % J.tiles[1];
    const int tz = t2 / J.tiles[1];
    const int nfx = J.nf[0], nfy = J.nf[1], nfz = J.nf[2];
    const int x0 = tx * BTX, y0 = ty * BTY, Z0 = tz * J.TZ;
    const int Zend = min(Z0 + J.TZ, nfz);
    const long long sxy = (long long)nfx * nfy;
    const gmem<double>* __restrict__ U = gview(J.u);
    const gmem<double>* __restrict__ V = gview(J.v);
    const gmem<double>* __restrict__ A = gview(J.a);
    const double cu = J.cu, cv = J.cv, ca = J.ca;
    const gmem<double>* __restrict__ LD = gview(J.load);
    gmem<double>* __restrict__ R = gview(J.R);
    const double rscale = J.rscale;
    const bool accumulate = J.accumulate != 0;
    const int wsplit = J.wsplit;

    // band rows of this thread's x-column (x-pass) and y-row (y-pass)
    T kx[B], ky[B], my[B];
    double mx[B], myd[B];
    {
      const gmem<double>* bx = gview(J.band[0]);
      const gmem<double>* by = gview(J.band[1]);
      const int gx = x0 + lx, gy = y0 + ly;
      const bool vx = gx < nfx, vy = gy < nfy;
      const long long ix = (long long)(vx ? gx : 0) * B, iy = (long long)(vy ? gy : 0) * B;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        mx[k] = vx ? bx[ix + k] : 0.0;
        kx[k] = vx ? (T)bx[(long long)nfx * B + ix + k] : T(0);
        myd[k] = vy ? by[iy + k] : 0.0;
        my[k] = (T)myd[k];
        ky[k] = vy ? (T)by[(long long)nfy * B + iy + k] : T(0);
      }
    }
    // z-band entries of a source layer s, one per lane of every wave: lane
    // k < 2p+1 holds M_z(s-p+k, s), lane 2p+1+k holds K_z(s-p+k, s) (zero
    // outside the free range); loaded with the layer's predictor and read
    // back with readlane
    const gmem<double>* bzg = gview(J.band[2]);
    const int zlane = threadIdx.x & 63;
    const int zk = zlane < B ? zlane : zlane - B;
    const long long zoff = zlane < B ? 0ll : (long long)nfz * B;
    double ampv = 0.0;
    if (J.load != nullptr && J.amp != nullptr) {
      long long ai = (long long)(*gview(J.counter)) + J.amp_shift;
      ampv = (ai >= 0 && ai < J.namp) ? gview(J.amp)[ai] : 0.0;
    }

    // predictor positions of this thread (zero outside the free range;
    // those load offset 0 so that no branch surrounds the loads)
    long long prow[NS];
    bool pval[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int k = tid + i * BNT;
      const int r = k / SX, c = k - r * SX;
      const int gy = y0 - p + r, gx = x0 - p + c;
      pval[i] = k < SY * SX && gy >= 0 && gy < nfy && gx >= 0 && gx < nfx;
      prow[i] = pval[i] ? (long long)gy * nfx + gx : 0;
    }
    // owned output column
    const bool own = x0 + lx < nfx && y0 + ly < nfy;
    const long long ocol = own ? (long long)(y0 + ly) * nfx + (x0 + lx) : 0;

    // kDepth layers of loads in flight: register set d holds the layers
    // s = sb + d (mod kDepth), with the load vector and the previous R of
    // the output its layer completes
    double pf[kDepth][NS];
    double pld[kDepth], prr[kDepth], pzb[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) pld[d] = prr[d] = 0.0;
    auto prefetch = [&](int s, double (&pf)[NS], double& pld, double& prr, double& pzb) {
      {
        const int o = s - p + zk;
        const bool ok = zlane < 2 * B && o >= 0 && o < nfz;
        pzb = bzg[ok ? zoff + (long long)o * B + (2 * p - zk) : 0];
        pzb = ok ? pzb : 0.0;
      }
      const long long zo = (long long)s * sxy;
      long long gi[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) gi[i] = pval[i] ? zo + prow[i] : 0;
#pragma unroll
      for (int i = 0; i < NS; ++i) pf[i] = cu * U[gi[i]];
      if (V != nullptr) {
#pragma unroll
        for (int i = 0; i < NS; ++i) pf[i] = fma(cv, V[gi[i]], pf[i]);
      }
      if (A != nullptr) {
#pragma unroll
        for (int i = 0; i < NS; ++i) pf[i] = fma(ca, A[gi[i]], pf[i]);
      }
      // output completed by source layer s: s - p
      const int o = s - p;
      const bool ov = own && o >= Z0 && o < Zend;
      const long long go = ov ? (long long)o * sxy + ocol : 0;
      if (LD != nullptr) pld = ov ? LD[go] : 0.0;
      if (accumulate) prr = ov ? R[go] : 0.0;
    };
    // W is free when a layer is committed: every thread passed the second
    // barrier of the previous layer after its x-pass
    auto commit = [&](const double (&pf)[NS]) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int k = tid + i * BNT;
        double w = pval[i] ? pf[i] : 0.0;
        if (wsplit != 0) {
          const double hi = (double)bf16_round_band((float)w);
          w = wsplit == 1 ? hi : w - hi;
        }
        if (k < SY * SX) Wl[k] = w;
      }
    };
    auto store = [&](int o, double accv, double ldv, double rv) {
      if (own && o >= Z0 && o < Zend) {
        const double r = rscale * (ampv * ldv - accv);
        R[(long long)o * sxy + ocol] = accumulate ? rv + r : r;
      }
    };

    double acc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) acc[k] = 0.0;
    // x-, y- and z-passes of committed source layer s
    auto process = [&](int s, double ldv, double rv, double zbv) {
      __syncthreads();
      // x-pass over the halo rows
#pragma unroll
      for (int i = 0; i < NXI; ++i) {
        const int r = ly + i * (BNT / BTX);
        if (r < SY) {
          const double* w = Wl + r * SX + lx;
          const double wc = w[p];
          T a1 = kx[p] * (T)wc;
          double a2 = mx[0] * w[0];
#pragma unroll
          for (int k = 0; k < B; ++k) {
            if (k != p) a1 = fma(kx[k], (T)(w[k] - wc), a1);
            if (k > 0) a2 = fma(mx[k], w[k], a2);
          }
          X1[r * BTX + lx] = a1;
          X2[r * BTX + lx] = a2;
        }
      }
      __syncthreads();
      // y-pass of the owned column, then the z-band into the accumulators
      {
        const T* c1 = X1 + ly * BTX + lx;
        const double* c2 = X2 + ly * BTX + lx;
        const double v2c = c2[p * BTX];
        T ym = my[0] * c1[0];
        double yk = myd[0] * c2[0];
        ym = fma(ky[p], (T)v2c, ym);
#pragma unroll
        for (int k = 0; k < B; ++k) {
          const T v1 = c1[k * BTX];
          const double v2 = c2[k * BTX];
          if (k > 0) {
            ym = fma(my[k], v1, ym);
            yk = fma(myd[k], v2, yk);
          }
          if (k != p) ym = fma(ky[k], (T)(v2 - v2c), ym);
        }
        const double dym = (double)ym, dyk = yk;
        // output o = s - p + k takes column s of its z-band rows: entry
        // (o, s) at o*(2p+1) + (s - o + p) = o*(2p+1) + 2p - k
        const long long zbb = __double_as_longlong(zbv);
        const int zlo = (int)(zbb & 0xffffffffll), zhi = (int)(zbb >> 32);
        auto lane_d = [&](int l) {
          const unsigned lo = (unsigned)__builtin_amdgcn_readlane(zlo, l);
          const unsigned hi = (unsigned)__builtin_amdgcn_readlane(zhi, l);
          return __longlong_as_double(((long long)hi << 32) | lo);
        };
#pragma unroll
        for (int k = 0; k < B; ++k) acc[k] = fma(lane_d(k), dym, fma(lane_d(B + k), dyk, acc[k]));
      }
      store(s - p, acc[0], ldv, rv);
#pragma unroll
      for (int k = 0; k < B - 1; ++k) acc[k] = acc[k + 1];
      acc[B - 1] = 0.0;
    };

    const int sb = max(0, Z0 - p), se = min(nfz - 1, Zend - 1 + p);
#pragma unroll
    for (int d = 0; d < kDepth; ++d)
      if (sb + d <= se) prefetch(sb + d, pf[d], pld[d], prr[d], pzb[d]);
    for (int s0 = sb; s0 <= se; s0 += kDepth) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        const int s = s0 + d;
        if (s > se) break;
        commit(pf[d]);
        const double ldv = pld[d], rv = prr[d], zbv = pzb[d];
        if (s + kDepth <= se) prefetch(s + kDepth, pf[d], pld[d], prr[d], pzb[d]);
        process(s, ldv, rv, zbv);
      }
    }
    // outputs se - p + 1 .. se + p: loads at store time (the tail of the range)
#pragma unroll
    for (int k = 0; k < B - 1; ++k) {
      const int o = se - p + 1 + k;
      if (own && o >= Z0 && o < Zend) {
        const long long go = (long long)o * sxy + ocol;
        store(o, acc[k], LD != nullptr ? LD[go] : 0.0, accumulate ? R[go] : 0.0);
      }
    }
    __syncthreads();
  }
}

template <typename T, int p>
static hipError_t band_one(const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  if (op == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)rhs_band_kernel<T, p>, BNT, 0);
  hipLaunchKernelGGL((rhs_band_kernel<T, p>), dim3(grid), dim3(BNT), 0, s, d_hdr);
  return hipGetLastError();
}

template <int p>
static hipError_t band_p(int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  return mixed ? band_one<float, p>(d_hdr, grid, s, op, out) : band_one<double, p>(d_hdr, grid, s, op, out);
}

static hipError_t band_dispatch(int p, int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  switch (p) {
    case 1: return band_p<1>(mixed, d_hdr, grid, s, op, out);
    case 2: return band_p<2>(mixed, d_hdr, grid, s, op, out);
    case 3: return band_p<3>(mixed, d_hdr, grid, s, op, out);
    case 4: return band_p<4>(mixed, d_hdr, grid, s, op, out);
    case 5: return band_p<5>(mixed, d_hdr, grid, s, op, out);
    default: return hipErrorInvalidValue;
  }
}

int rhs_band_tile_x() { return BTX; }
int rhs_band_tile_y() { return BTY; }

hipError_t launch_rhs_band(int p, int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  return band_dispatch(p, mixed, d_hdr, grid, s, 0, nullptr);
}

int rhs_band_blocks_per_cu(int p, int mixed) {
  int n = 1;
  (void)band_dispatch(p, mixed, nullptr, 0, nullptr, 1, &n);
  return n < 1 ? 1 : n;
}

}  // namespace ads
