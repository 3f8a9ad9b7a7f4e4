// Direction sweeps: banded forward/back substitution along every grid line
// of one direction (Appendix: the x-, y- and z-problems are 1D banded
// systems with one right-hand side per line; the factor is shared).
//
// Mapping on gfx950: a block is one wave64 and a tile is W lines (W = 16 by
// default, 32 or 64 selectable).  All 64 lanes stage the tile into LDS
// [i][line] with an XOR swizzle: x-lines (contiguous in memory) as one flat
// cooperative block, y- and z-lines with 64/W lanes per line so that each
// load instruction reads 64/W rows of W consecutive x.  The first W lanes
// then run the substitution, one line each, with the factor rows staged in
// LDS behind the tile and read as broadcasts.  Small tiles give several
// waves per CU that overlap one another's load, solve and store phases; the
// tile loads are issued kChunk at a time per lane before any is consumed.
// The forward result overwrites the tile in LDS, the backward result
// overwrites it again, then all 64 lanes write it out (optionally fused with
// the Newmark or three-level time update).
#include <cstdlib>

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
__device__ __forceinline__ void substitute(double* lds, int lane, int m, const double* fl) {
  constexpr int p = P;
  // factor rows staged in LDS behind the tile: L[m*p], U[m*p], rd[m]
  const double* Lf = fl;
  const double* Uf = fl + m * p;
  const double* rdf = fl + 2 * m * p;
  double h[p];
#pragma unroll
  for (int k = 0; k < p; ++k) h[k] = 0.0;
#pragma unroll 8
  for (int i = 0; i < m; ++i) {
    const double* Li = Lf + i * p;
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
    const double* Ui = Uf + i * p;
    double s = lds[sidx<W>(i, lane)];
#pragma unroll
    for (int k = p - 1; k >= 0; --k) s = fma(-Ui[k], h[k], s);
    s *= rdf[i];
#pragma unroll
    for (int k = p - 1; k > 0; --k) h[k] = h[k - 1];
    h[0] = s;
    lds[sidx<W>(i, lane)] = s;
  }
}

constexpr int kNT = 64;   // threads per block: one wave64

// A tile is W lines (W divides 64).  All 64 lanes of the block stage the
// tile: x-lines cooperatively as one contiguous block, y/z-lines with 64/W
// lanes per line (consecutive lanes = consecutive lines = consecutive x, so
// each instruction reads 64/W rows of W contiguous doubles).  The first W
// lanes run the substitution, one line each.  Small W gives many small
// waves (several per CU) that overlap each other's load, solve and store.
template <int W>
__global__ __launch_bounds__(kNT) void sweep_kernel(const LaunchHdr* __restrict__ hdr) {
  static_assert(kNT % W == 0, "W must divide the wave size");
  constexpr int RL = kNT / W;   // lanes per line in the cooperative y/z access
  extern __shared__ double lds[];
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const SweepJob* __restrict__ jobs = hdr_jobs<SweepJob>(hdr);
  const int tid = threadIdx.x;
  const int ll = tid % W, lq = tid / W;   // cooperative y/z access: line ll, row phase lq
  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const int jb = find_job_sweep(jobs, njobs, tile);
    const SweepJob& J = jobs[jb];
    const int t = tile - J.tile0;
    const int m = J.f.m;
    const int line0 = t * W;
    const int nl = min(W, J.nlines - line0);
    const bool lact = ll < nl;
    long long base = 0, stride = 0;
    if (J.dir != 0 && lact) line_geom(J, line0 + ll, base, stride);
    if (J.dir == 0) {
      // x-lines: the nl lines of the tile are one contiguous block of nl*m
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      for (int f0 = 0; f0 < tot; f0 += kChunk * kNT) {
        double r[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          int fidx = f0 + k * kNT + tid;
          r[k] = fidx < tot ? J.in[gb + fidx] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          int fidx = f0 + k * kNT + tid;
          if (fidx < tot) {
            int l = fidx / m, i = fidx - l * m;
            lds[sidx<W>(i, l)] = J.scale * r[k];
          }
        }
      }
    } else if (lact) {
      for (int i0 = lq; i0 < m; i0 += kChunk * RL) {
        double r[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          int i = i0 + k * RL;
          r[k] = i < m ? J.in[base + (long long)i * stride] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          int i = i0 + k * RL;
          if (i < m) lds[sidx<W>(i, ll)] = J.scale * r[k];
        }
      }
    }
    // stage the factor rows behind the tile (read as LDS broadcasts)
    double* fl = lds + W * m;
    {
      const int mp = m * J.p;
      for (int k = tid; k < mp; k += kNT) {
        fl[k] = J.f.L[k];
        fl[mp + k] = J.f.U[k];
      }
      for (int k = tid; k < m; k += kNT) fl[2 * mp + k] = J.f.rd[k];
    }
    __syncthreads();
    if (tid < nl) {
      switch (J.p) {
        case 1: substitute<W, 1>(lds, tid, m, fl); break;
        case 2: substitute<W, 2>(lds, tid, m, fl); break;
        default: substitute<W, 3>(lds, tid, m, fl); break;
      }
    }
    __syncthreads();
    if (J.dir == 0) {
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      for (int f0 = 0; f0 < tot; f0 += kEpi * kNT) {
        long long g[kEpi];
        double x[kEpi];
        bool ok[kEpi];
#pragma unroll
        for (int k = 0; k < kEpi; ++k) {
          int fidx = f0 + k * kNT + tid;
          ok[k] = fidx < tot;
          int l = ok[k] ? fidx / m : 0, i = ok[k] ? fidx - l * m : 0;
          g[k] = gb + fidx;
          x[k] = ok[k] ? lds[sidx<W>(i, l)] : 0.0;
        }
        epilogue_batch(J, g, x, ok);
      }
    } else if (lact) {
      for (int i0 = lq; i0 < m; i0 += kEpi * RL) {
        long long g[kEpi];
        double x[kEpi];
        bool ok[kEpi];
#pragma unroll
        for (int k = 0; k < kEpi; ++k) {
          int i = i0 + k * RL;
          ok[k] = i < m;
          g[k] = base + (long long)i * stride;
          x[k] = ok[k] ? lds[sidx<W>(i, ll)] : 0.0;
        }
        epilogue_batch(J, g, x, ok);
      }
    }
    if (t == 0 && tid == 0 && J.counter != nullptr) *J.counter += 1ull;
    __syncthreads();
  }
}

// Lines per tile (16, 32 or 64; ADS_SWEEP_W overrides the default 16).
int sweep_width() {
  static int w = [] {
    const char* e = std::getenv("ADS_SWEEP_W");
    int v = e ? std::atoi(e) : 16;
    return (v == 32 || v == 64) ? v : 16;
  }();
  return w;
}
int sweep_width_for(int) { return sweep_width(); }

// Dynamic LDS: the tile (W lines x m) + the factor rows (2p+1 <= 7 per
// line position).
static size_t sweep_lds_bytes(int W, int max_m) { return (size_t)(W + 2 * kMaxP + 1) * max_m * sizeof(double); }

// Resident sweep blocks per CU for lines of at most max_m unknowns (the
// persistent grid of a merged launch is this times the CU count).
int sweep_blocks_per_cu(int max_m) {
  const int W = sweep_width();
  const size_t lds = sweep_lds_bytes(W, max_m);
  int n = 0;
  hipError_t e;
  if (W == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)sweep_kernel<64>, kNT, lds);
  else if (W == 32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)sweep_kernel<32>, kNT, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)sweep_kernel<16>, kNT, lds);
  return (e == hipSuccess && n > 0) ? n : 2;
}

hipError_t launch_sweeps(const LaunchHdr* d_hdr, int grid, int max_m, hipStream_t s) {
  const int W = sweep_width();
  const size_t lds = sweep_lds_bytes(W, max_m);
  if (grid <= 0) return hipSuccess;
  if (W == 64) {
    hipLaunchKernelGGL(sweep_kernel<64>, dim3(grid), dim3(kNT), lds, s, d_hdr);
  } else if (W == 32) {
    hipLaunchKernelGGL(sweep_kernel<32>, dim3(grid), dim3(kNT), lds, s, d_hdr);
  } else {
    hipLaunchKernelGGL(sweep_kernel<16>, dim3(grid), dim3(kNT), lds, s, d_hdr);
  }
  return hipGetLastError();
}

hipError_t sweep_set_attributes() {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)sweep_kernel<64>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)sweep_kernel<32>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)sweep_kernel<16>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace ads
