// Right-hand side of the P-wave step without a wave-speed field, in the
// Kronecker form of the stiffness matrix (Section 2, eq. pwave2, in 3D):
// with constant coefficients the Galerkin stiffness is a sum of three
// tensor products of assembled 1D matrices of bandwidth 2p+1 (restricted
// to the free coefficients),
//
//   K = K_x(x)M_y(x)M_z + M_x(x)K_y(x)M_z + M_x(x)M_y(x)K_z,
//   R = rscale * ( amp * b - K w ),   w = cu * src,
//
// src being the time step's predictor field (or the state, for the start
// and the energy diagnostic), applied as three band passes with two
// channels each:
//   x:  X1 = K_x w,            X2 = M_x w
//   y:  YM = M_y X1 + K_y X2,  YK = M_y X2
//   z:  K w = M_z YM + K_z YK
// i.e. 7(2p+1) multiply-adds per coefficient, against the hundreds of the
// element quadrature; the 1D matrices are the same Gauss sums (exact for
// q = p+1), so the result is the quadrature's up to rounding.  One field
// in, one out.
//
// Tiling on gfx950: a workgroup of eight waves owns BTX x BTY = 64 x 8
// columns (a wave per row) and a z-range of TZ outputs and marches over the
// source layers that reach them (TZ + 2p).  Per source layer: the layer
// with a p-halo in x and y (coalesced rows) goes to LDS, its loads issued
// kDepth layers ahead and consumed only then (no arithmetic or select on a
// load in flight, which would wait for it at once); the x-pass runs over
// the halo rows (LDS -> LDS, one thread per column, its band rows in
// registers); the y-pass gives each owned column its two channels (the
// wave's y-band rows are scalars: one row per wave), which the z-band
// scatters into 2p+1 FP64 accumulators (outputs s-p .. s+p of source layer
// s; the layer's 2(2p+1) z-band entries are loaded by as many threads with
// the layer and pass through LDS, read back as one broadcast per wave).
// The oldest accumulator is complete after each layer and is written.  Two
// barriers per layer, no atomics, each output computed by one thread.
// Tiles are spread over the XCDs in contiguous ranges (halo re-reads hit
// the L2).  T is the type of the x- and y-stiffness passes K_x w, K_y X2
// and of M_y X1: double, or float in mixed mode (on differences formed in
// FP64, the stored bands holding the row sum in the diagonal slot); the
// field, the mass channel X2 = M_x w and YK = M_y X2, the z-accumulation and
// the output are FP64.
#include "common.hpp"
#include "launch.hpp"

namespace ads {

constexpr int BTX = 64, BTY = 8, BNT = BTX * BTY;
constexpr int kDepth = 2;   // source layers whose loads are in flight

template <bool V>
struct BoolC {
  static constexpr bool value = V;
};

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

// at least two waves per SIMD at p <= 3 (the second launch-bounds argument
// is waves per SIMD); at p = 2 the registers (128) allow four, i.e. two
// workgroups per CU
template <typename T, int p>
__global__ __launch_bounds__(BNT, p <= 3 ? 2 : 1) void rhs_band_kernel(const LaunchHdr* __restrict__ hdr) {
  using Gm = BandGeom<T, p>;
  constexpr int B = Gm::B, SX = Gm::SX, SY = Gm::SY, NS = Gm::NS, NXI = Gm::NXI;
  constexpr bool F64 = sizeof(T) == 8;
  // The predictor and the mass channel stay FP64 in every mode: a stiffness
  // band applied to differences of FP32-rounded values would turn their
  // rounding (relative to the values) into an error of the stiffness action
  // larger by about (wavelength / h)^2.  In mixed mode only the stiffness
  // passes K_x w and K_y X2, and M_y X1, run in FP32, on differences formed
  // in FP64.  In FP64 the x- and y-stiffness passes use the plain band (its
  // diagonal recovered from the stored row sum), one multiply-add per entry.
  __shared__ double Wl[SY * SX];   // predictor layer with halos
  __shared__ T X1[SY * BTX];       // K_x w
  __shared__ double X2[SY * BTX];  // M_x w
  __shared__ double Zl[2][2 * B];  // z-band entries of the layer (two in turn): M_z, K_z column
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const RhsJob* __restrict__ jobs = hdr_jobs<RhsJob>(hdr);
  // a wave is one row of the tile (BTX = 64): ly is wave-uniform, so the
  // y-band rows of the y-pass are scalar values
  const int tid = threadIdx.x, lx = tid % BTX, ly = __builtin_amdgcn_readfirstlane(tid / BTX);

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
    // the source field w = cu * u (the step's predictor field, or the
    // state field of the start and of the energy diagnostic)
    const gmem<double>* __restrict__ U = gview(J.u);
    const double cu = J.cu;
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
      const cmem<double>* by = cview(J.band[1]);
      const int gx = x0 + lx, gy = y0 + ly;
      const bool vx = gx < nfx, vy = gy < nfy;
      const long long ix = (long long)(vx ? gx : 0) * B, iy = (long long)(vy ? gy : 0) * B;
      double kxd[B], kyd[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        mx[k] = vx ? bx[ix + k] : 0.0;
        kxd[k] = vx ? bx[(long long)nfx * B + ix + k] : 0.0;
        myd[k] = vy ? by[iy + k] : 0.0;
        kyd[k] = vy ? by[(long long)nfy * B + iy + k] : 0.0;
      }
      if constexpr (F64) {
        // plain form: the diagonal is the row sum minus the off-diagonal
        // entries (the stored band holds the row sum in its diagonal slot)
        double dx = kxd[p], dy = kyd[p];
#pragma unroll
        for (int k = 0; k < B; ++k)
          if (k != p) {
            dx -= kxd[k];
            dy -= kyd[k];
          }
        kxd[p] = dx;
        kyd[p] = dy;
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        kx[k] = (T)kxd[k];
        ky[k] = (T)kyd[k];
        my[k] = (T)myd[k];
      }
    }
    // z-band entries of a source layer s: thread k < 2p+1 loads M_z(s-p+k, s),
    // thread 2p+1+k loads K_z(s-p+k, s) (zero outside the free range); they
    // reach the other threads through LDS (Zl), written when the layer is
    // committed and read after its first barrier
    const gmem<double>* bzg = gview(J.band[2]);
    const bool zload = tid < 2 * B;
    const int zk = tid < B ? tid : tid - B;
    const long long zoff = tid < B ? 0ll : (long long)nfz * B;
    double ampv = 0.0;
    if (J.load != nullptr && J.amp != nullptr) {
      long long ai = (long long)(*gview(J.counter)) + J.amp_shift;
      ampv = (ai >= 0 && ai < J.namp) ? gview(J.amp)[ai] : 0.0;
    }

    // predictor positions of this thread as byte offsets in a z-layer (a
    // layer holds at most 4101^2 coefficients: the offsets fit 32 bits; zero
    // outside the free range: such positions load the layer's first entry
    // and are replaced by zero when committed, so no branch surrounds the
    // loads)
    unsigned pofs[NS];
    bool pval[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int k = tid + i * BNT;
      const int r = k / SX, c = k - r * SX;
      const int gy = y0 - p + r, gx = x0 - p + c;
      pval[i] = k < SY * SX && gy >= 0 && gy < nfy && gx >= 0 && gx < nfx;
      pofs[i] = pval[i] ? (unsigned)(gy * nfx + gx) * 8u : 0u;
    }
    // owned output column
    const bool own = x0 + lx < nfx && y0 + ly < nfy;
    const long long ocol = own ? (long long)(y0 + ly) * nfx + (x0 + lx) : 0;

    // W and the layer's Zl slot are free when a layer is committed: every
    // thread passed the second barrier of the previous layer after its
    // x-pass, and the first barrier of the previous layer after its z-pass
    // of the layer before (the slot's last reader)
    auto commit = [&](int s, const double (&qu)[NS], double zbv) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int k = tid + i * BNT;
        double w = pval[i] ? cu * qu[i] : 0.0;
        if (wsplit != 0) {
          const double hi = (double)bf16_round_band((float)w);
          w = wsplit == 1 ? hi : w - hi;
        }
        if (k < SY * SX) Wl[k] = w;
      }
      if (zload) {
        const int o = s - p + zk;
        Zl[s & 1][tid] = (o >= 0 && o < nfz) ? zbv : 0.0;
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
    auto process = [&](int s, double ldv, double rv) {
      __syncthreads();
      // x-pass over the halo rows
#pragma unroll
      for (int i = 0; i < NXI; ++i) {
        const int r = ly + i * (BNT / BTX);
        if (r < SY) {
          const double* w = Wl + r * SX + lx;
          T a1;
          double a2 = mx[0] * w[0];
          if constexpr (F64) {
            a1 = kx[0] * w[0];
#pragma unroll
            for (int k = 1; k < B; ++k) {
              a1 = fma(kx[k], w[k], a1);
              a2 = fma(mx[k], w[k], a2);
            }
          } else {
            const double wc = w[p];
            a1 = kx[p] * (T)wc;
#pragma unroll
            for (int k = 0; k < B; ++k) {
              if (k != p) a1 = fma(kx[k], (T)(w[k] - wc), a1);
              if (k > 0) a2 = fma(mx[k], w[k], a2);
            }
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
        T ym = my[0] * c1[0];
        double yk = myd[0] * c2[0];
        if constexpr (F64) {
          ym = fma(ky[0], c2[0], ym);
#pragma unroll
          for (int k = 1; k < B; ++k) {
            const double v1 = c1[k * BTX], v2 = c2[k * BTX];
            ym = fma(my[k], v1, ym);
            ym = fma(ky[k], v2, ym);
            yk = fma(myd[k], v2, yk);
          }
        } else {
          const double v2c = c2[p * BTX];
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
        }
        const double dym = (double)ym, dyk = yk;
        // output o = s - p + k takes column s of its z-band rows (entries
        // read from LDS at one address per wave: a broadcast)
        const double* zb = Zl[s & 1];
#pragma unroll
        for (int k = 0; k < B; ++k) acc[k] = fma(zb[k], dym, fma(zb[B + k], dyk, acc[k]));
      }
      store(s - p, acc[0], ldv, rv);
#pragma unroll
      for (int k = 0; k < B - 1; ++k) acc[k] = acc[k + 1];
      acc[B - 1] = 0.0;
    };

    const int sb = max(0, Z0 - p), se = min(nfz - 1, Zend - 1 + p);
    // kDepth layers of loads in flight: register set d holds the raw loads
    // of layer s = sb + d (mod kDepth) (the source field, the z-band entry,
    // and with EX the load vector and the previous R at the output the layer
    // completes); nothing consumes them before the layer is committed,
    // kDepth layers later, so the loads stay in flight meanwhile.  EX is
    // false for jobs without a load vector and without accumulation (no
    // per-output loads at all).  With EX the per-output loads are
    // unconditional (offset 0 where the output is not this thread's; a
    // missing load vector reads R instead and is replaced by zero at use),
    // so that no select waits for them early.
    auto layers = [&](auto ex) {
      constexpr bool EX = decltype(ex)::value;
      const gmem<double>* __restrict__ LDp = LD != nullptr ? LD : R;
      double pu[kDepth][NS];
      double pld[kDepth], prr[kDepth], pzb[kDepth];
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        pld[d] = prr[d] = pzb[d] = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) pu[d][i] = 0.0;
      }
      auto prefetch = [&](int s, double (&qu)[NS], double& pld, double& prr, double& pzb) {
        if (zload) {
          const int o = s - p + zk;
          const bool ok = o >= 0 && o < nfz;
          pzb = bzg[ok ? zoff + (long long)o * B + (2 * p - zk) : 0];
        }
        const gmem<char>* Ub = (const gmem<char>*)(U + (long long)s * sxy);
#pragma unroll
        for (int i = 0; i < NS; ++i) qu[i] = *(const gmem<double>*)(Ub + pofs[i]);
        if constexpr (EX) {
          // output completed by source layer s: s - p
          const int o = s - p;
          const bool ov = own && o >= Z0 && o < Zend;
          const long long go = ov ? (long long)o * sxy + ocol : 0;
          pld = LDp[go];
          prr = R[go];
        }
      };
#pragma unroll
      for (int d = 0; d < kDepth; ++d)
        if (sb + d <= se) prefetch(sb + d, pu[d], pld[d], prr[d], pzb[d]);
      for (int s0 = sb; s0 <= se; s0 += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d) {
          const int s = s0 + d;
          if (s > se) break;
          commit(s, pu[d], pzb[d]);
          const double ldv = (EX && LD != nullptr) ? pld[d] : 0.0;
          const double rv = (EX && accumulate) ? prr[d] : 0.0;
          if (s + kDepth <= se) prefetch(s + kDepth, pu[d], pld[d], prr[d], pzb[d]);
          process(s, ldv, rv);
        }
      }
    };
    if (LD != nullptr || accumulate) layers(BoolC<true>{});
    else layers(BoolC<false>{});
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
