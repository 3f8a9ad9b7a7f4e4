// Direction sweeps: banded forward/back substitution along every grid line
// of one direction (Appendix: the x-, y- and z-problems are 1D banded
// systems with one right-hand side per line; the factor is shared).
//
// Mapping on gfx950: a tile is W lines (W = 64, one wave64; 32 or 16 for
// lines longer than 128), one lane per line.  The tile is staged in LDS
// [i][lane] with an XOR swizzle so that both the line-major global access
// of x-lines (contiguous in memory, loaded cooperatively and transposed
// through LDS) and the lane-parallel substitution are bank-conflict free.
// y- and z-lines are read lane-parallel straight from HBM (consecutive lanes
// are consecutive x, so every row of the tile is one coalesced access).
// The factor entries are uniform across the tile and come through the
// scalar cache.  The forward result overwrites the tile in LDS, the backward
// result overwrites it again, then the epilogue writes it out (optionally
// fused with the Newmark or three-level time update).
#include "common.hpp"

namespace ads {

__device__ __forceinline__ int find_job_sweep(const SweepJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int W>
__device__ __forceinline__ int sidx(int i, int l) { return i * W + (l ^ (i & (W - 1))); }

// Global offset of element i of line `line` and the element stride.
__device__ __forceinline__ void line_geom(const SweepJob& J, int line, long long& base, long long& stride) {
  if (J.dir == 0) {
    base = (long long)line * J.nx;
    stride = 1;
  } else if (J.dir == 1) {
    int z = line / J.nx, x = line - z * J.nx;
    base = (long long)z * J.nx * J.ny + x;
    stride = J.nx;
  } else {
    base = line;
    stride = (long long)J.nx * J.ny;
  }
}

__device__ __forceinline__ void epilogue(const SweepJob& J, long long g, double x) {
  if (J.epi == EPI_STORE) {
    J.out[g] = x;
  } else if (J.epi == EPI_NEWMARK) {
    double u = J.e0[g], v = J.e1[g], a = J.e2[g];
    double s = a + x;
    J.e1[g] = v + 0.5 * J.c0 * s;
    J.e0[g] = u + J.c0 * v + J.c1 * s;
    J.e2[g] = x;
  } else {  // EPI_THREELEVEL
    double un = J.e0[g], um = J.e1[g];
    J.out[g] = x;
    J.e1[g] = un;
    J.e0[g] = 2.0 * un - um + x;
  }
}

// Forward (L, unit diagonal) then backward (U) substitution on one lane's
// line held in LDS.  The dependency chain per step is a single FMA on the
// most recent value; the older terms are folded in first.
template <int W, int P>
__device__ __forceinline__ void substitute(double* lds, int lane, int m, const Factor1D& f) {
  constexpr int p = P;
  double h[p];
#pragma unroll
  for (int k = 0; k < p; ++k) h[k] = 0.0;
  for (int i = 0; i < m; ++i) {
    const double* Li = f.L + (long long)i * p;
    double s = lds[sidx<W>(i, lane)];
#pragma unroll
    for (int k = p - 1; k >= 0; --k) s = fma(-Li[k], h[k], s);
#pragma unroll
    for (int k = p - 1; k > 0; --k) h[k] = h[k - 1];
    h[0] = s;
    lds[sidx<W>(i, lane)] = s;
  }
#pragma unroll
  for (int k = 0; k < p; ++k) h[k] = 0.0;
  for (int i = m - 1; i >= 0; --i) {
    const double* Ui = f.U + (long long)i * p;
    double s = lds[sidx<W>(i, lane)];
#pragma unroll
    for (int k = p - 1; k >= 0; --k) s = fma(-Ui[k], h[k], s);
    s *= f.rd[i];
#pragma unroll
    for (int k = p - 1; k > 0; --k) h[k] = h[k - 1];
    h[0] = s;
    lds[sidx<W>(i, lane)] = s;
  }
}

template <int W>
__global__ __launch_bounds__(W) void sweep_kernel(const SweepJob* __restrict__ jobs, int njobs, int total_tiles) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const int jb = find_job_sweep(jobs, njobs, tile);
    const SweepJob& J = jobs[jb];
    const int t = tile - J.tile0;
    const int m = J.f.m;
    const int line0 = t * W;
    const int nl = min(W, J.nlines - line0);
    const int line = line0 + lane;
    const bool active = lane < nl;
    long long base = 0, stride = 0;
    if (J.dir == 0) {
      // x-lines: the nl lines of the tile are one contiguous block of nl*m
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      for (int fidx = lane; fidx < tot; fidx += W) {
        int l = fidx / m, i = fidx - l * m;
        lds[sidx<W>(i, l)] = J.scale * J.in[gb + fidx];
      }
    } else if (active) {
      line_geom(J, line, base, stride);
      for (int i = 0; i < m; ++i) lds[sidx<W>(i, lane)] = J.scale * J.in[base + i * stride];
    }
    __syncthreads();
    if (active) {
      switch (J.p) {
        case 1: substitute<W, 1>(lds, lane, m, J.f); break;
        case 2: substitute<W, 2>(lds, lane, m, J.f); break;
        default: substitute<W, 3>(lds, lane, m, J.f); break;
      }
    }
    __syncthreads();
    if (J.dir == 0) {
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      for (int fidx = lane; fidx < tot; fidx += W) {
        int l = fidx / m, i = fidx - l * m;
        epilogue(J, gb + fidx, lds[sidx<W>(i, l)]);
      }
    } else if (active) {
      for (int i = 0; i < m; ++i) epilogue(J, base + i * stride, lds[sidx<W>(i, lane)]);
    }
    if (t == 0 && lane == 0 && J.counter != nullptr) *J.counter += 1ull;
    __syncthreads();
  }
}

// Tiles per job for a lines-per-tile width W.
int sweep_width_for(int max_m) {
  if (max_m <= 128) return 64;
  if (max_m <= 256) return 32;
  return 16;
}

hipError_t launch_sweeps(const SweepJob* d_jobs, int njobs, int total_tiles, int max_m, int grid_cap,
                         hipStream_t s) {
  const int W = sweep_width_for(max_m);
  size_t lds = (size_t)W * max_m * sizeof(double);
  int grid = total_tiles;
  if (grid_cap > 0 && grid > grid_cap) grid = grid_cap;
  if (grid <= 0) return hipSuccess;
  if (W == 64) {
    hipLaunchKernelGGL(sweep_kernel<64>, dim3(grid), dim3(64), lds, s, d_jobs, njobs, total_tiles);
  } else if (W == 32) {
    hipLaunchKernelGGL(sweep_kernel<32>, dim3(grid), dim3(32), lds, s, d_jobs, njobs, total_tiles);
  } else {
    hipLaunchKernelGGL(sweep_kernel<16>, dim3(grid), dim3(16), lds, s, d_jobs, njobs, total_tiles);
  }
  return hipGetLastError();
}

hipError_t sweep_set_attributes() {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)sweep_kernel<64>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)sweep_kernel<32>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)sweep_kernel<16>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
}

}  // namespace ads
