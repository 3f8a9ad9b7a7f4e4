// Sum of tensor products of 1D banded matrices applied to fields
// (elasticity couplings of the alternating-triangular stages, eq. pre /
// eq. corr:  rho M Y_i  and  Upsilon_ij Y_j = mu G(x)G^T(x)M + lambda
// G^T(x)G(x)M in the directions of i and j):
//
//   out = alpha * base + sum_t coef_t * (T^t_x (x) T^t_y (x) T^t_z) src_t
//
// One thread per output coefficient; the (2p+1)^3 stencil is evaluated by
// sum factorization in registers (x-rows, then y, then z).
#include "common.hpp"

namespace ads {

constexpr int kKronPts = 256;

__device__ __forceinline__ int find_job_kron(const KronJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int p>
__device__ double kron_term(const KronTerm& T, int x, int y, int z, int nx, int ny, int nz) {
  constexpr int B = 2 * p + 1;
  const double* Tx = T.T[0] + (long long)x * B;
  const double* Ty = T.T[1] + (long long)y * B;
  const double* Tz = T.T[2] + (long long)z * B;
  double sz = 0.0;
  for (int c = -p; c <= p; ++c) {
    int zz = z + c;
    if (zz < 0 || zz >= nz) continue;
    double sy = 0.0;
    for (int b = -p; b <= p; ++b) {
      int yy = y + b;
      if (yy < 0 || yy >= ny) continue;
      const double* row = T.src + ((long long)zz * ny + yy) * nx;
      double sx = 0.0;
#pragma unroll
      for (int a = -p; a <= p; ++a) {
        int xx = x + a;
        if (xx >= 0 && xx < nx) sx = fma(Tx[a + p], row[xx], sx);
      }
      sy = fma(Ty[b + p], sx, sy);
    }
    sz = fma(Tz[c + p], sy, sz);
  }
  return sz;
}

__global__ __launch_bounds__(kKronPts) void kron_kernel(const LaunchHdr* __restrict__ hdr) {
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const KronJob* __restrict__ jobs = hdr_jobs<KronJob>(hdr);
  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const KronJob& J = jobs[find_job_kron(jobs, njobs, tile)];
    const long long idx = (long long)(tile - J.tile0) * kKronPts + threadIdx.x;
    const long long n = (long long)J.nx * J.ny * J.nz;
    if (idx >= n) continue;
    const int x = (int)(idx % J.nx);
    const long long r = idx / J.nx;
    const int y = (int)(r % J.ny), z = (int)(r / J.ny);
    double s = (J.base != nullptr) ? J.alpha * J.base[idx] : 0.0;
    for (int t = 0; t < J.nterm; ++t) {
      double v = (J.p == 2) ? kron_term<2>(J.term[t], x, y, z, J.nx, J.ny, J.nz)
                            : kron_term<3>(J.term[t], x, y, z, J.nx, J.ny, J.nz);
      s = fma(J.term[t].coef, v, s);
    }
    J.out[idx] = s;
  }
}

int kron_tile_points() { return kKronPts; }

hipError_t launch_kron(const LaunchHdr* d_hdr, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(kron_kernel, dim3(grid), dim3(kKronPts), 0, s, d_hdr);
  return hipGetLastError();
}

}  // namespace ads
