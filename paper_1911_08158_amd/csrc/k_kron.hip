// Sum of tensor products of 1D banded matrices applied to fields
// (elasticity couplings of the alternating-triangular stages, eq. pre /
// eq. corr:  rho M Y_i  and  Upsilon_ij Y_j = mu G(x)G^T(x)M + lambda
// G^T(x)G(x)M in the directions of i and j):
//
//   out = alpha * base + sum_t coef_t * (T^t_x (x) T^t_y (x) T^t_z) src_t
//
// Sum factorization on gfx950: a workgroup owns a KTX x KTY column tile and
// a z-range of outputs and walks the source layers that reach the range.
// Per source layer it stages the layer of every term (with a p-halo in x
// and y) in LDS, applies the x-bands (LDS -> LDS), then per term the y-band
// (one thread per owned column) and scatters the result through the z-band
// into 2p+1 register accumulators (outputs zs-p .. zs+p); the oldest
// accumulator is complete after each layer and is written out.  The next
// layer's global loads, all terms at once, are in flight while the current
// one is contracted (one load latency and two barriers per layer).  The
// band rows of every term for the tile's columns are staged once per tile.
#include <algorithm>

#include "common.hpp"

namespace ads {

constexpr int KTX = 32, KTY = 8, KNT = KTX * KTY;
constexpr int kKronMaxTerms = 6;   // KronJob::term

__device__ __forceinline__ int find_job_kron(const KronJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int p>
struct KronGeom {
  static constexpr int B = 2 * p + 1;
  static constexpr int SX = KTX + 2 * p, SY = KTY + 2 * p;
  static constexpr int NS = (SY * SX + KNT - 1) / KNT;   // layer loads per thread
  static constexpr int NX = (SY * KTX + KNT - 1) / KNT;  // x-band items per thread and term
  // LDS: S [terms][SY][SX], X [terms][SY][KTX], band rows [terms][KTX + KTY][B]
  static constexpr size_t lds_elems =
      (size_t)kKronMaxTerms * (SY * SX + SY * KTX) + (size_t)kKronMaxTerms * (KTX + KTY) * B;
};

template <int p>
__device__ void kron_tile(const KronJob& J, int t, double* lds) {
  using Gm = KronGeom<p>;
  constexpr int B = Gm::B, SX = Gm::SX, SY = Gm::SY, NS = Gm::NS, NX = Gm::NX;
  constexpr int MT = kKronMaxTerms;
  double* S = lds;                      // [MT][SY][SX]
  double* X = S + MT * SY * SX;         // [MT][SY][KTX]
  double* Tb = X + MT * SY * KTX;
  const int tid = threadIdx.x, lx = tid % KTX, ly = tid / KTX;
  const int tx = t % J.tiles[0], t2 = t / J.tiles[0];
  const int ty = t2 % J.tiles[1], tz = t2 / J.tiles[1];
  const int nx = J.nx, ny = J.ny, nz = J.nz, nt = J.nterm;
  const int X0 = tx * KTX, Y0 = ty * KTY, Z0 = tz * J.TZ, Z1 = min(Z0 + J.TZ, nz);
  // band rows of every term for the tile's x and y indices (zero outside)
  for (int k = tid; k < nt * (KTX + KTY) * B; k += KNT) {
    const int term = k / ((KTX + KTY) * B), r = k - term * ((KTX + KTY) * B);
    const int row = r / B, c = r - row * B;
    double v = 0.0;
    if (row < KTX) {
      const int x = X0 + row;
      if (x < nx) v = gview(J.term[term].T[0])[(long long)x * B + c];
    } else {
      const int y = Y0 + row - KTX;
      if (y < ny) v = gview(J.term[term].T[1])[(long long)y * B + c];
    }
    Tb[k] = v;
  }
  // source-layer loads of this thread: positions k = tid + i*KNT of [SY][SX]
  long long soff[NS];
  bool sval[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int k = tid + i * KNT;
    const int yy = k / SX, xx = k - yy * SX;
    const int x = X0 - p + xx, y = Y0 - p + yy;
    sval[i] = k < SY * SX && x >= 0 && x < nx && y >= 0 && y < ny;
    soff[i] = (long long)y * nx + x;
  }
  const long long sxy = (long long)nx * ny;
  double pf[MT][NS];
  // layer zs of every term (positions outside the field load offset 0 of
  // the layer, no branch around the loads, and are zeroed when the layer is
  // written to LDS: nothing consumes a load before then, so that the loads
  // stay in flight during the previous layer's contractions)
  auto prefetch = [&](int zs) {
#pragma unroll
    for (int term = 0; term < MT; ++term) {
      if (term < nt) {
        const gmem<double>* src = gview(J.term[term].src) + (long long)zs * sxy;
#pragma unroll
        for (int i = 0; i < NS; ++i) pf[term][i] = src[sval[i] ? soff[i] : 0];
      }
    }
  };
  const bool ocol = X0 + lx < nx && Y0 + ly < ny;
  const long long obase = (long long)(Y0 + ly) * nx + X0 + lx;
  gmem<double>* __restrict__ out = gview(J.out);
  const gmem<double>* __restrict__ bse = gview(J.base);
  const double alpha = J.alpha;
  auto store = [&](int z, double v) {
    if (ocol && z >= Z0 && z < Z1) {
      const long long g = (long long)z * sxy + obase;
      out[g] = (bse != nullptr) ? fma(alpha, bse[g], v) : v;
    }
  };
  double acc[B];
#pragma unroll
  for (int k = 0; k < B; ++k) acc[k] = 0.0;
  // window: acc[k] is output z = zs - p + k
  const int zs0 = max(0, Z0 - p), zs1 = min(nz - 1, Z1 - 1 + p);
  prefetch(zs0);
  for (int zs = zs0; zs <= zs1; ++zs) {
#pragma unroll
    for (int term = 0; term < MT; ++term) {
      if (term < nt) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int k = tid + i * KNT;
          if (k < SY * SX) S[term * (SY * SX) + k] = sval[i] ? pf[term][i] : 0.0;
        }
      }
    }
    __syncthreads();
    // the next layer in flight during the contractions
    if (zs < zs1) prefetch(zs + 1);
    for (int term = 0; term < nt; ++term) {
      const double* tbx = Tb + term * ((KTX + KTY) * B);
      const double* St = S + term * (SY * SX);
      double* Xt = X + term * (SY * KTX);
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        const int k = tid + i * KNT;
        if (k < SY * KTX) {
          const int yy = k / KTX, xo = k - yy * KTX;
          const double* srow = St + yy * SX + xo;
          double s = tbx[xo * B] * srow[0];
#pragma unroll
          for (int a = 1; a < B; ++a) s = fma(tbx[xo * B + a], srow[a], s);
          Xt[k] = s;
        }
      }
    }
    __syncthreads();
    for (int term = 0; term < nt; ++term) {
      const double* tby = Tb + term * ((KTX + KTY) * B) + KTX * B + ly * B;
      const double* Xt = X + term * (SY * KTX);
      double sy = tby[0] * Xt[ly * KTX + lx];
#pragma unroll
      for (int b = 1; b < B; ++b) sy = fma(tby[b], Xt[(ly + b) * KTX + lx], sy);
      sy *= J.term[term].coef;
      // z band at wave-uniform rows: scalar loads
      const cmem<double>* Tz = cview(J.term[term].T[2]);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int z = zs - p + k;
        if (z >= 0 && z < nz) acc[k] = fma(Tz[(long long)z * B + (2 * p - k)], sy, acc[k]);
      }
    }
    // output zs - p has all its source layers
    store(zs - p, acc[0]);
#pragma unroll
    for (int k = 0; k < B - 1; ++k) acc[k] = acc[k + 1];
    acc[B - 1] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < B - 1; ++k) store(zs1 + 1 - p + k, acc[k]);
  __syncthreads();   // LDS is reused by the next tile
}

// Jobs of different degrees may share a launch: the degree is taken per
// tile (HI instantiation: every degree 1 to 5, for launches that hold
// p = 4 or 5; else 1 to 3; the LDS is sized for the largest degree of the
// launch).
template <bool HI>
__global__ __launch_bounds__(KNT) void kron_kernel(const LaunchHdr* __restrict__ hdr) {
  extern __shared__ double lds[];
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const KronJob* __restrict__ jobs = hdr_jobs<KronJob>(hdr);
  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const KronJob& J = jobs[find_job_kron(jobs, njobs, tile)];
    if constexpr (HI) {
      if (J.p == 5) {
        kron_tile<5>(J, tile - J.tile0, lds);
        continue;
      }
      if (J.p == 4) {
        kron_tile<4>(J, tile - J.tile0, lds);
        continue;
      }
    }
    {
      if (J.p == 1) kron_tile<1>(J, tile - J.tile0, lds);
      else if (J.p == 2) kron_tile<2>(J, tile - J.tile0, lds);
      else kron_tile<3>(J, tile - J.tile0, lds);
    }
  }
}

int kron_tile_x() { return KTX; }
int kron_tile_y() { return KTY; }

static size_t kron_lds_elems(int p) {
  switch (p) {
    case 1: return KronGeom<1>::lds_elems;
    case 2: return KronGeom<2>::lds_elems;
    case 3: return KronGeom<3>::lds_elems;
    case 4: return KronGeom<4>::lds_elems;
    default: return KronGeom<5>::lds_elems;
  }
}
// LDS of a launch whose largest degree is pmax (the layout of every degree
// up to pmax fits)
static size_t kron_lds_bytes(int pmax) {
  size_t e = 0;
  for (int p = 1; p <= pmax; ++p) e = std::max(e, kron_lds_elems(p));
  return e * sizeof(double);
}

int kron_blocks_per_cu(int pmax) {
  int n = 0;
  const void* k = pmax >= 4 ? (const void*)kron_kernel<true> : (const void*)kron_kernel<false>;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, KNT, kron_lds_bytes(pmax));
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t kron_set_attributes() {
  for (const void* k : {(const void*)kron_kernel<false>, (const void*)kron_kernel<true>}) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_kron(const LaunchHdr* d_hdr, int grid, int pmax, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (pmax < 1 || pmax > kMaxP) return hipErrorInvalidValue;
  if (pmax >= 4) hipLaunchKernelGGL(kron_kernel<true>, dim3(grid), dim3(KNT), kron_lds_bytes(pmax), s, d_hdr);
  else hipLaunchKernelGGL(kron_kernel<false>, dim3(grid), dim3(KNT), kron_lds_bytes(pmax), s, d_hdr);
  return hipGetLastError();
}

}  // namespace ads
