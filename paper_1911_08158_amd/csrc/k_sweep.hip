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

constexpr int kChunk = 32;   // global loads in flight per lane while staging a tile

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

// Epilogue on K solved values at global offsets g[k] (ok[k] false = skip);
// all old-state loads of the batch are issued before any is used.
constexpr int kEpi = 8;
__device__ __forceinline__ void epilogue_batch(const SweepJob& J, const long long* g, const double* x,
                                               const bool* ok) {
  if (J.epi == EPI_STORE) {
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) J.out[g[k]] = x[k];
  } else if (J.epi == EPI_NEWMARK) {
    double u[kEpi], v[kEpi], a[kEpi];
#pragma unroll
    for (int k = 0; k < kEpi; ++k) {
      u[k] = ok[k] ? J.e0[g[k]] : 0.0;
      v[k] = ok[k] ? J.e1[g[k]] : 0.0;
      a[k] = ok[k] ? J.e2[g[k]] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) {
        double s = a[k] + x[k];
        J.e1[g[k]] = v[k] + 0.5 * J.c0 * s;
        J.e0[g[k]] = u[k] + J.c0 * v[k] + J.c1 * s;
        J.e2[g[k]] = x[k];
      }
  } else {  // EPI_THREELEVEL
    double un[kEpi], um[kEpi];
#pragma unroll
    for (int k = 0; k < kEpi; ++k) {
      un[k] = ok[k] ? J.e0[g[k]] : 0.0;
      um[k] = ok[k] ? J.e1[g[k]] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) {
        J.out[g[k]] = x[k];
        J.e1[g[k]] = un[k];
        J.e0[g[k]] = 2.0 * un[k] - um[k] + x[k];
      }
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
#pragma unroll 8
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
#pragma unroll 8
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
__global__ __launch_bounds__(W) void sweep_kernel(const LaunchHdr* __restrict__ hdr) {
  extern __shared__ double lds[];
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const SweepJob* __restrict__ jobs = hdr_jobs<SweepJob>(hdr);
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
      // x-lines: the nl lines of the tile are one contiguous block of nl*m;
      // kChunk loads per lane are issued before any is consumed
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      for (int f0 = 0; f0 < tot; f0 += kChunk * W) {
        double r[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          int fidx = f0 + k * W + lane;
          r[k] = fidx < tot ? J.in[gb + fidx] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          int fidx = f0 + k * W + lane;
          if (fidx < tot) {
            int l = fidx / m, i = fidx - l * m;
            lds[sidx<W>(i, l)] = J.scale * r[k];
          }
        }
      }
    } else if (active) {
      line_geom(J, line, base, stride);
      for (int i0 = 0; i0 < m; i0 += kChunk) {
        double r[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) r[k] = (i0 + k < m) ? J.in[base + (i0 + k) * stride] : 0.0;
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
          if (i0 + k < m) lds[sidx<W>(i0 + k, lane)] = J.scale * r[k];
      }
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
      for (int f0 = 0; f0 < tot; f0 += kEpi * W) {
        long long g[kEpi];
        double x[kEpi];
        bool ok[kEpi];
#pragma unroll
        for (int k = 0; k < kEpi; ++k) {
          int fidx = f0 + k * W + lane;
          ok[k] = fidx < tot;
          int l = ok[k] ? fidx / m : 0, i = ok[k] ? fidx - l * m : 0;
          g[k] = gb + fidx;
          x[k] = ok[k] ? lds[sidx<W>(i, l)] : 0.0;
        }
        epilogue_batch(J, g, x, ok);
      }
    } else if (active) {
      for (int i0 = 0; i0 < m; i0 += kEpi) {
        long long g[kEpi];
        double x[kEpi];
        bool ok[kEpi];
#pragma unroll
        for (int k = 0; k < kEpi; ++k) {
          ok[k] = i0 + k < m;
          g[k] = base + (long long)(i0 + k) * stride;
          x[k] = ok[k] ? lds[sidx<W>(i0 + k, lane)] : 0.0;
        }
        epilogue_batch(J, g, x, ok);
      }
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

hipError_t launch_sweeps(const LaunchHdr* d_hdr, int grid, int max_m, hipStream_t s) {
  const int W = sweep_width_for(max_m);
  size_t lds = (size_t)W * max_m * sizeof(double);
  if (grid <= 0) return hipSuccess;
  if (W == 64) {
    hipLaunchKernelGGL(sweep_kernel<64>, dim3(grid), dim3(64), lds, s, d_hdr);
  } else if (W == 32) {
    hipLaunchKernelGGL(sweep_kernel<32>, dim3(grid), dim3(32), lds, s, d_hdr);
  } else {
    hipLaunchKernelGGL(sweep_kernel<16>, dim3(grid), dim3(16), lds, s, d_hdr);
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
