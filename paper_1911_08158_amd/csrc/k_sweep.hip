// Direction sweeps: banded forward/back substitution along every grid line
// of one direction (Appendix: the x-, y- and z-problems are 1D banded
// systems with one right-hand side per line; the factor is shared).
//
// Mapping on gfx950: a workgroup is four wave64s and takes a group of 4W
// consecutive lines of one job; each wave owns a tile of W lines (W = 16,
// or 8 / 4 for launches with few lines).  The wave
// stages its tile in LDS [i][line] (rows padded to W+1): x-lines (contiguous
// in memory) as one flat cooperative block, y- and z-lines with 64/W lanes
// per line so that each load reads 64/W rows of W consecutive x.  The first
// W lanes then run the substitution, one line each, reading the factor rows
// as LDS broadcasts; all 64 lanes write the result (optionally fused with
// the Newmark or three-level time update).  The factor rows are staged
// once per workgroup and again only when a group belongs to another job,
// so inside a job the four waves never wait for each other: one wave's
// loads, substitution and stores overlap the others'.
#include <algorithm>
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

// Completes this wave's LDS writes before its lanes read each other's
// values (LDS operations of one wave execute in order).
__device__ __forceinline__ void wave_sync_sw() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile layout in LDS: row i (one value per line) at i*(W+1): the padding
// makes both the row reads of the substitution (W consecutive values) and
// the column writes of the x-line staging (stride W+1) free of bank
// conflicts, and every access an immediate offset from one base.
template <int W>
__device__ __forceinline__ int sidx(int i, int l) { return i * (W + 1) + l; }

constexpr int kChunk = 32;   // global loads in flight per lane while staging a tile
constexpr int kWaves = 4;    // waves per workgroup (one tile each)
constexpr int kNT = 64 * kWaves;

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

// A job's output side, read once per group: the pointers as global views.
struct EpiView {
  gmem<double>* out;
  gmem<double>* e0;
  gmem<double>* e1;
  gmem<double>* e2;
  double c0, c1;
  int epi;
};

// Epilogue on K solved values at global offsets g[k] (ok[k] false = skip;
// g[k] is then still a valid offset of the field, so the old-state loads
// need no branch); all loads of the batch are issued before any is used.
constexpr int kEpi = 8;
__device__ __forceinline__ void epilogue_batch(const EpiView& E, const long long* g, const double* x,
                                               const bool* ok) {
  if (E.epi == EPI_STORE) {
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) E.out[g[k]] = x[k];
  } else if (E.epi == EPI_NEWMARK) {
    double w[kEpi], b[kEpi];
#pragma unroll
    for (int k = 0; k < kEpi; ++k) {
      w[k] = E.e0[g[k]];
      b[k] = E.e1[g[k]];
    }
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) {
        E.e0[g[k]] = fma(E.c1, x[k], fma(E.c0, b[k], w[k]));
        E.e1[g[k]] = fma(E.c0, x[k], b[k]);
        E.e2[g[k]] = x[k];
      }
  } else if (E.epi == EPI_NEWMARK_LITERAL) {
    double w[kEpi], v[kEpi];
#pragma unroll
    for (int k = 0; k < kEpi; ++k) {
      w[k] = E.e0[g[k]];
      v[k] = E.e1[g[k]];
    }
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) {
        const double vn = v[k] + 0.5 * E.c0 * x[k];
        E.e0[g[k]] = fma(E.c0, vn, w[k]);
        E.e1[g[k]] = vn;
        E.e2[g[k]] = x[k];
      }
  } else {  // EPI_THREELEVEL
    double un[kEpi], um[kEpi];
#pragma unroll
    for (int k = 0; k < kEpi; ++k) {
      un[k] = E.e0[g[k]];
      um[k] = E.e1[g[k]];
    }
#pragma unroll
    for (int k = 0; k < kEpi; ++k)
      if (ok[k]) {
        E.out[g[k]] = x[k];
        E.e1[g[k]] = un[k];
        E.e0[g[k]] = 2.0 * un[k] - um[k] + x[k];
      }
  }
}

// Forward (L, unit diagonal) then backward (U) substitution on one lane's
// line held in LDS.  The dependency chain per step is a single FMA on the
// most recent value; the older terms are folded in first.  Rows go in
// blocks of kSB: the block's values and factor rows are read into registers
// first (one LDS wait per block), the chain runs in registers, the results
// are written back.
constexpr int kSB = 8;

template <int W, int P>
__device__ __forceinline__ void substitute(double* tl, int lane, int m, const double* fl) {
  constexpr int TP = W + 1;
  // factor rows: L[m*p], U[m*p], rd[m]
  const double* Lf = fl;
  const double* Uf = fl + m * P;
  const double* rdf = fl + 2 * m * P;
  const int nb = m / kSB;          // full blocks; rows nb*kSB .. m-1 are the tail
  double h[P];
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = 0.0;
  double* col = tl + lane;
  for (int b = 0; b < nb; ++b) {
    double* rb = col + b * kSB * TP;
    const double* Lb = Lf + b * kSB * P;
    double v[kSB], f[kSB][P];
#pragma unroll
    for (int k = 0; k < kSB; ++k) {
      v[k] = rb[k * TP];
#pragma unroll
      for (int j = 0; j < P; ++j) f[k][j] = Lb[k * P + j];
    }
#pragma unroll
    for (int k = 0; k < kSB; ++k) {
      double s = v[k];
#pragma unroll
      for (int j = P - 1; j >= 0; --j) s = fma(-f[k][j], h[j], s);
#pragma unroll
      for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
      h[0] = s;
      rb[k * TP] = s;
    }
  }
  for (int i = nb * kSB; i < m; ++i) {
    double s = col[i * TP];
#pragma unroll
    for (int j = P - 1; j >= 0; --j) s = fma(-Lf[i * P + j], h[j], s);
#pragma unroll
    for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
    h[0] = s;
    col[i * TP] = s;
  }
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = 0.0;
  for (int i = m - 1; i >= nb * kSB; --i) {
    double s = col[i * TP];
#pragma unroll
    for (int j = P - 1; j >= 0; --j) s = fma(-Uf[i * P + j], h[j], s);
    s *= rdf[i];
#pragma unroll
    for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
    h[0] = s;
    col[i * TP] = s;
  }
  for (int b = nb - 1; b >= 0; --b) {
    double* rb = col + b * kSB * TP;
    const double* Ub = Uf + b * kSB * P;
    const double* rdb = rdf + b * kSB;
    double v[kSB], f[kSB][P], r[kSB];
#pragma unroll
    for (int k = 0; k < kSB; ++k) {
      v[k] = rb[k * TP];
      r[k] = rdb[k];
#pragma unroll
      for (int j = 0; j < P; ++j) f[k][j] = Ub[k * P + j];
    }
#pragma unroll
    for (int k = kSB - 1; k >= 0; --k) {
      double s = v[k];
#pragma unroll
      for (int j = P - 1; j >= 0; --j) s = fma(-f[k][j], h[j], s);
      s *= r[k];
#pragma unroll
      for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
      h[0] = s;
      rb[k * TP] = s;
    }
  }
}

// Job tiling: SweepJob.tile0 / ntiles count groups of 4W lines; the header's
// total_tiles is the number of groups of the launch.
// Substitution of degree p: HI instantiations take every degree 1 to 5
// (launches whose jobs include p = 4 or 5), the others p = 1, 2, 3 (two
// kernels, so that the registers of the high degrees do not weigh on the
// common ones).
template <int W, bool HI>
__device__ __forceinline__ void substitute_p(int p, double* tl, int lane, int m, const double* fl) {
  if constexpr (HI) {
    if (p == 5) return substitute<W, 5>(tl, lane, m, fl);
    if (p == 4) return substitute<W, 4>(tl, lane, m, fl);
  }
  if (p == 1) substitute<W, 1>(tl, lane, m, fl);
  else if (p == 2) substitute<W, 2>(tl, lane, m, fl);
  else substitute<W, 3>(tl, lane, m, fl);
}

// frows: factor rows per line position in LDS, 2 pmax + 1 for the largest
// degree pmax of the launch's jobs.
template <int W, bool HI>
__global__ __launch_bounds__(kNT, 2) void sweep_kernel(const LaunchHdr* __restrict__ hdr, int max_m, int frows) {
  static_assert(64 % W == 0, "W must divide the wave size");
  constexpr int RL = 64 / W;   // lanes per line in the cooperative y/z access
  extern __shared__ double lds[];
  const int njobs = hdr->njobs, total_groups = hdr->total_tiles;
  const SweepJob* __restrict__ jobs = hdr_jobs<SweepJob>(hdr);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int ll = lane % W, lq = lane / W;   // cooperative y/z access: line ll, row phase lq
  double* fl = lds;                                             // factor rows
  double* tl = lds + frows * max_m + wv * (W + 1) * max_m;      // this wave's tile
  int staged = -1;                                              // job whose factor is in LDS
  for (int grp = blockIdx.x; grp < total_groups; grp += gridDim.x) {
    const int jb = find_job_sweep(jobs, njobs, grp);
    const SweepJob& J = jobs[jb];
    const int m = J.f.m;
    if (jb != staged) {   // uniform over the workgroup
      __syncthreads();    // no wave still reads the previous factor
      const int mp = m * J.p;
      const gmem<double>* fL = gview(J.f.L);
      const gmem<double>* fU = gview(J.f.U);
      const gmem<double>* frd = gview(J.f.rd);
      for (int k = tid; k < mp; k += kNT) {
        fl[k] = fL[k];
        fl[mp + k] = fU[k];
      }
      for (int k = tid; k < m; k += kNT) fl[2 * mp + k] = frd[k];
      __syncthreads();
      staged = jb;
    }
    const int line0 = ((grp - J.tile0) * kWaves + wv) * W;
    if (line0 >= J.nlines) continue;   // the job's last group may be partial
    const int nl = min(W, J.nlines - line0);
    const bool lact = ll < nl;
    const int dir = J.dir;
    const double scale = J.scale;
    const gmem<double>* __restrict__ gin = gview(J.in);
    const EpiView E{gview(J.out), gview(J.e0), gview(J.e1), gview(J.e2), J.c0, J.c1, J.epi};
    // inactive lanes of a partial tile take line 0 of the tile: every
    // address below stays inside the field (loads need no branch)
    long long base = 0, stride = 0;
    if (dir != 0) line_geom(J, line0 + (lact ? ll : 0), base, stride);
    if (dir == 0) {
      // x-lines: the nl lines of the tile are one contiguous block of nl*m
      // (loads past its end re-read its last element)
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      int l = lane / m, i = lane - l * m;   // (line, row) of flat index f0 + lane
      for (int f0 = 0; f0 < tot; f0 += kChunk * 64) {
        double c[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) c[k] = gin[gb + min(f0 + k * 64 + lane, tot - 1)];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          if (f0 + k * 64 + lane < tot) tl[sidx<W>(i, l)] = scale * c[k];
          i += 64;
          while (i >= m) {   // at most once for m >= 64
            i -= m;
            ++l;
          }
        }
      }
    } else if (lact) {
      for (int i0 = lq; i0 < m; i0 += kChunk * RL) {
        double c[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) c[k] = gin[base + (long long)min(i0 + k * RL, m - 1) * stride];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          const int i = i0 + k * RL;
          if (i < m) tl[sidx<W>(i, ll)] = scale * c[k];
        }
      }
    }
    wave_sync_sw();
    if (lane < nl) substitute_p<W, HI>(J.p, tl, lane, m, fl);
    wave_sync_sw();
    if (dir == 0) {
      const long long gb = (long long)line0 * m;
      const int tot = nl * m;
      int l = lane / m, i = lane - l * m;   // (line, row) of flat index f0 + lane
      for (int f0 = 0; f0 < tot; f0 += kEpi * 64) {
        long long g[kEpi];
        double x[kEpi];
        bool ok[kEpi];
#pragma unroll
        for (int k = 0; k < kEpi; ++k) {
          const int fidx = f0 + k * 64 + lane;
          ok[k] = fidx < tot;
          g[k] = gb + (ok[k] ? fidx : 0);
          x[k] = ok[k] ? tl[sidx<W>(i, l)] : 0.0;
          i += 64;
          while (i >= m) {
            i -= m;
            ++l;
          }
        }
        epilogue_batch(E, g, x, ok);
      }
    } else if (lact) {
      for (int i0 = lq; i0 < m; i0 += kEpi * RL) {
        long long g[kEpi];
        double x[kEpi];
        bool ok[kEpi];
#pragma unroll
        for (int k = 0; k < kEpi; ++k) {
          const int i = i0 + k * RL;
          ok[k] = i < m;
          g[k] = base + (long long)(ok[k] ? i : 0) * stride;
          x[k] = ok[k] ? tl[sidx<W>(i, ll)] : 0.0;
        }
        epilogue_batch(E, g, x, ok);
      }
    }
    if (line0 == 0 && lane == 0 && J.counter != nullptr) *gview(J.counter) += 1ull;
    // the next tile of this wave overwrites the tile region: every lane's
    // epilogue reads of it come first
    wave_sync_sw();
  }
}

// ---------------------------------------------------------------------------
// In-plane sweeps.  The 160 KiB LDS of a CU holds a whole z-plane of up to
// 128 x 128 FP64 unknowns (padded rows of nx + 1) with the x- and y-factor
// rows, so one workgroup solves the x-lines and then the y-lines of a plane
// without writing the intermediate to memory: 16 B per unknown instead of
// 32 for the two sweeps, a thread per x-line, then a thread per y-line.
// The memory traffic rides on the recurrences: the x-forward pass reads its
// line from global memory with the next chunk in flight, and the y-backward
// pass stores each final value as it is produced.  With the odd row pitch
// the x-lines' LDS accesses (lanes a row apart) and the y-lines' (lanes
// adjacent) are free of bank conflicts.

constexpr int kPT = 256;    // threads per plane workgroup
constexpr int kPTC = 512;   // ... with coupling terms (more loads in flight)
// coupled input (plane_couple): the largest plane it takes
constexpr int kCoupleMaxN = 4608;

__device__ __forceinline__ int find_job_plane(const PlaneJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Substitution passes of one line with element i at col[i * st] in LDS;
// factor rows fl = L[m*P], U[m*P], rd[m] in LDS (broadcast reads).  The
// arithmetic and its order are those of `substitute`.  Forward pass:
template <int P>
__device__ __forceinline__ void fwd_st(double* col, int st, int m, const double* fl) {
  const double* Lf = fl;
  const int nb = m / kSB;
  double h[P];
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = 0.0;
  for (int b = 0; b < nb; ++b) {
    double* rb = col + b * kSB * st;
    const double* Lb = Lf + b * kSB * P;
    double v[kSB], f[kSB][P];
#pragma unroll
    for (int k = 0; k < kSB; ++k) {
      v[k] = rb[k * st];
#pragma unroll
      for (int j = 0; j < P; ++j) f[k][j] = Lb[k * P + j];
    }
#pragma unroll
    for (int k = 0; k < kSB; ++k) {
      double s = v[k];
#pragma unroll
      for (int j = P - 1; j >= 0; --j) s = fma(-f[k][j], h[j], s);
#pragma unroll
      for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
      h[0] = s;
      rb[k * st] = s;
    }
  }
  for (int i = nb * kSB; i < m; ++i) {
    double s = col[i * st];
#pragma unroll
    for (int j = P - 1; j >= 0; --j) s = fma(-Lf[i * P + j], h[j], s);
#pragma unroll
    for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
    h[0] = s;
    col[i * st] = s;
  }
}

// Forward pass fed from global memory: element i is scale * src[i]; the
// results go to col[i] in LDS.  The line is read in chunks of 2 kSB values,
// the next chunk's loads in flight while the current one is substituted,
// so that the plane's loads overlap the forward recurrences.
template <int P>
__device__ __forceinline__ void fwd_from_global(const gmem<double>* __restrict__ src, double scale, double* col,
                                                int m, const double* fl) {
  constexpr int C = 2 * kSB;
  const double* Lf = fl;
  const int nc = m / C;
  double h[P];
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = 0.0;
  double va[C], vb[C];
  auto load = [&](double (&v)[C], int c) {
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = src[c * C + k];
  };
  auto run = [&](const double (&v)[C], int c) {
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      const int r0 = c * C + hb * kSB;
      const double* Lb = Lf + r0 * P;
      double f[kSB][P];
#pragma unroll
      for (int k = 0; k < kSB; ++k)
#pragma unroll
        for (int j = 0; j < P; ++j) f[k][j] = Lb[k * P + j];
#pragma unroll
      for (int k = 0; k < kSB; ++k) {
        double s = scale * v[hb * kSB + k];
#pragma unroll
        for (int j = P - 1; j >= 0; --j) s = fma(-f[k][j], h[j], s);
#pragma unroll
        for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
        h[0] = s;
        col[r0 + k] = s;
      }
    }
  };
  // chunks in pairs, each chunk's loads issued before the other chunk is
  // substituted (every use unconditional, so that no load is moved next to
  // its use; past the end the va reload re-reads the last chunk); the
  // scheduling barriers keep the loads ahead of the substitution
  if (nc > 0) load(va, 0);
  int c = 0;
  for (; c + 1 < nc; c += 2) {
    load(vb, c + 1);
    __builtin_amdgcn_sched_barrier(0);
    run(va, c);
    load(va, min(c + 2, nc - 1));
    __builtin_amdgcn_sched_barrier(0);
    run(vb, c + 1);
  }
  if (c < nc) run(va, c);
  for (int i = nc * C; i < m; ++i) {
    double s = scale * src[i];
#pragma unroll
    for (int j = P - 1; j >= 0; --j) s = fma(-Lf[i * P + j], h[j], s);
#pragma unroll
    for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
    h[0] = s;
    col[i] = s;
  }
}

// Backward pass on the LDS line; each result is stored to dst[i * ds] in
// global memory (ToGlobal) or back to col[i * st].
template <int P, bool ToGlobal>
__device__ __forceinline__ void bwd_st(double* col, int st, gmem<double>* __restrict__ dst, long long ds, int m,
                                       const double* fl) {
  const double* Uf = fl + m * P;
  const double* rdf = fl + 2 * m * P;
  const int nb = m / kSB;
  double h[P];
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = 0.0;
  for (int i = m - 1; i >= nb * kSB; --i) {
    double s = col[i * st];
#pragma unroll
    for (int j = P - 1; j >= 0; --j) s = fma(-Uf[i * P + j], h[j], s);
    s *= rdf[i];
#pragma unroll
    for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
    h[0] = s;
    if constexpr (ToGlobal) dst[i * ds] = s;
    else col[i * st] = s;
  }
  for (int b = nb - 1; b >= 0; --b) {
    double* rb = col + b * kSB * st;
    const double* Ub = Uf + b * kSB * P;
    const double* rdb = rdf + b * kSB;
    double v[kSB], f[kSB][P], r[kSB];
#pragma unroll
    for (int k = 0; k < kSB; ++k) {
      v[k] = rb[k * st];
      r[k] = rdb[k];
#pragma unroll
      for (int j = 0; j < P; ++j) f[k][j] = Ub[k * P + j];
    }
#pragma unroll
    for (int k = kSB - 1; k >= 0; --k) {
      double s = v[k];
#pragma unroll
      for (int j = P - 1; j >= 0; --j) s = fma(-f[k][j], h[j], s);
      s *= r[k];
#pragma unroll
      for (int j = P - 1; j > 0; --j) h[j] = h[j - 1];
      h[0] = s;
      if constexpr (ToGlobal) dst[(b * kSB + k) * ds] = s;
      else rb[k * st] = s;
    }
  }
}

// LDS: plane [ny][nx + 1], then the x-factor rows (2p+1 per x) and the
// y-factor rows (2p+1 per y).
size_t plane_lds_bytes(int nx, int ny, int p) {
  return ((size_t)ny * (nx + 1) + (size_t)(2 * p + 1) * (nx + ny)) * sizeof(double);
}
bool plane_fits(int nx, int ny, int p) { return plane_lds_bytes(nx, ny, p) <= (size_t)160 * 1024; }
// With coupling terms: the work space of plane_couple after the factor rows.
size_t plane_lds_bytes(int nx, int ny, int p, bool coupled) {
  size_t b = plane_lds_bytes(nx, ny, p);
  if (coupled) b += (2 * (size_t)nx * ny + 2 * (size_t)(2 * p + 1) * (nx + ny)) * sizeof(double);
  return b;
}
bool plane_couple_fits(int nx, int ny, int p) {
  return (long long)nx * ny <= kCoupleMaxN && plane_lds_bytes(nx, ny, p, true) <= (size_t)160 * 1024;
}

// x-lines of a plane: forward pass from global memory, backward in LDS
template <int P>
__device__ __forceinline__ void plane_x(const gmem<double>* __restrict__ src, double scale, double* col, int nx,
                                        const double* fxl) {
  fwd_from_global<P>(src, scale, col, nx, fxl);
  bwd_st<P, false>(col, 1, nullptr, 0, nx, fxl);
}
// y-lines of a plane: forward pass in LDS, backward pass storing the results
template <int P>
__device__ __forceinline__ void plane_y(double* col, int PX, gmem<double>* __restrict__ dst, int nx, int ny,
                                        const double* fyl) {
  fwd_st<P>(col, PX, ny, fyl);
  bwd_st<P, true>(col, PX, dst, nx, ny, fyl);
}

// Degree dispatch as in substitute_p (HI: every degree, else 1 to 3).
template <bool HI>
__device__ __forceinline__ void plane_x_p(int p, const gmem<double>* __restrict__ src, double scale, double* col,
                                          int nx, const double* fxl) {
  if constexpr (HI) {
    if (p == 5) return plane_x<5>(src, scale, col, nx, fxl);
    if (p == 4) return plane_x<4>(src, scale, col, nx, fxl);
  }
  if (p == 1) plane_x<1>(src, scale, col, nx, fxl);
  else if (p == 2) plane_x<2>(src, scale, col, nx, fxl);
  else plane_x<3>(src, scale, col, nx, fxl);
}
template <bool HI>
__device__ __forceinline__ void plane_y_p(int p, double* col, int PX, gmem<double>* __restrict__ dst, int nx,
                                          int ny, const double* fyl) {
  if constexpr (HI) {
    if (p == 5) return plane_y<5>(col, PX, dst, nx, ny, fyl);
    if (p == 4) return plane_y<4>(col, PX, dst, nx, ny, fyl);
  }
  if (p == 1) plane_y<1>(col, PX, dst, nx, ny, fyl);
  else if (p == 2) plane_y<2>(col, PX, dst, nx, ny, fyl);
  else plane_y<3>(col, PX, dst, nx, ny, fyl);
}

// Coupled input of plane z (PlaneJob with nterm > 0), written to the plane
// buffer pl as scale * (in + sum_t coef_t (T^t_x (x) T^t_y (x) T^t_z) src_t).
// Sum factorization over the whole plane, z first: per term the 2p+1 source
// planes that reach z are combined with row z of T_z into A (terms with the
// source and z-band of the term before them reuse its A), the x-band takes
// A to B, and the y-band of B is accumulated into pl (which holds the base
// input from the first term on).  A thread owns the positions tid + i NT
// of the plane and takes them in groups of G, the loads of a group in
// flight together.  Work space wk (after the factor rows): A [n], B [n],
// the band rows of two terms [2][(nx + ny)(2p+1)] (double-buffered, so that
// staging the next term's rows needs no barrier of its own).  Two barriers
// per term.
template <int P, int NT>
__device__ void plane_couple(const PlaneJob& J, int z, double* pl, double* wk) {
  constexpr int B = 2 * P + 1;
  constexpr int NC = (kCoupleMaxN + NT - 1) / NT;   // positions per thread
  constexpr int G = P <= 2 ? 5 : 3;   // positions per group (global loads)
  constexpr int GL = 3;               // ... in the LDS passes
  const int nx = J.nx, ny = J.ny, nz = J.nz, n = nx * ny, PX = nx + 1;
  const int tid = threadIdx.x;
  // (y, x) of position k + NT from those of k
  const int dy = NT / nx, dx = NT - dy * nx;
  auto next = [&](int& y, int& x) {
    y += dy;
    x += dx;
    if (x >= nx) {
      x -= nx;
      ++y;
    }
  };
  const int ty0 = tid / nx, tx0 = tid - ty0 * nx;
  double* A = wk;
  double* Bx = A + n;
  double* TB = Bx + n;
  const int tbs = (nx + ny) * B;
  for (int t = 0; t < J.nterm; ++t) {
    const KronTerm& T = J.term[t];
    double* tb = TB + (t & 1) * tbs;
    {
      const gmem<double>* tx = gview(T.T[0]);
      const gmem<double>* ty = gview(T.T[1]);
      for (int k0 = 0; k0 < tbs; k0 += 4 * NT) {
        double v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = min(k0 + tid + r * NT, tbs - 1);
          v[r] = k < nx * B ? tx[k] : ty[k - nx * B];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (k0 + tid + r * NT < tbs) tb[k0 + tid + r * NT] = v[r];
      }
    }
    if (t == 0 || T.src != J.term[t - 1].src || T.T[2] != J.term[t - 1].T[2]) {
      // A = sum_zs T_z[z][zs] src(zs): row z of the z-band (wave-uniform:
      // scalar loads); planes outside the field read a plane of it with
      // weight zero, and positions past the plane its last position, so
      // that no load waits behind a branch.  The first term also moves the
      // base input into pl.
      const cmem<double>* tz = cview(T.T[2]) + (long long)z * B;
      const gmem<double>* src = gview(T.src);
      const gmem<double>* in = (t == 0 && J.in != nullptr) ? gview(J.in) + (long long)z * n : nullptr;
      double w[B];
      long long zo[B];
#pragma unroll
      for (int kk = 0; kk < B; ++kk) {
        const int zs = z + kk - P;
        const bool ok = zs >= 0 && zs < nz;
        w[kk] = ok ? tz[kk] : 0.0;
        zo[kk] = (long long)(ok ? zs : z) * n;
      }
      int y = ty0, x = tx0;
#pragma unroll 1
      for (int i0 = 0; i0 < NC; i0 += G) {
        const int kb = tid + i0 * NT;
        if (kb >= n) break;
        double a[G], b[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
          a[j] = 0.0;
          b[j] = in != nullptr ? in[min(kb + j * NT, n - 1)] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < B; ++kk) {
          const gmem<double>* sp = src + zo[kk];
#pragma unroll
          for (int j = 0; j < G; ++j) a[j] = fma(w[kk], sp[min(kb + j * NT, n - 1)], a[j]);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
          if (kb + j * NT < n) {
            A[kb + j * NT] = a[j];
            if (t == 0) pl[y * PX + x] = b[j];
          }
          next(y, x);
        }
      }
    }
    __syncthreads();
    // B = x-band of A (columns outside the line read an edge value with
    // weight zero)
    {
      int y = ty0, x = tx0;
#pragma unroll 1
      for (int i0 = 0; i0 < NC; i0 += GL) {
        const int kb = tid + i0 * NT;
        if (kb >= n) break;
#pragma unroll
        for (int j = 0; j < GL; ++j) {
          const int k = kb + j * NT;
          if (k < n) {
            const double* tr = tb + x * B;
            const double* ar = A + y * nx;
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < B; ++c) {
              const int xs = x + c - P;
              v = fma((xs >= 0 && xs < nx) ? tr[c] : 0.0, ar[min(max(xs, 0), nx - 1)], v);
            }
            Bx[k] = v;
          }
          next(y, x);
        }
      }
    }
    __syncthreads();
    // pl += coef * y-band of B
    {
      const double cf = T.coef;
      int y = ty0, x = tx0;
#pragma unroll 1
      for (int i0 = 0; i0 < NC; i0 += GL) {
        const int kb = tid + i0 * NT;
        if (kb >= n) break;
#pragma unroll
        for (int j = 0; j < GL; ++j) {
          const int k = kb + j * NT;
          if (k < n) {
            const double* tr = tb + (nx + y) * B;
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < B; ++c) {
              const int ys = y + c - P;
              v = fma((ys >= 0 && ys < ny) ? tr[c] : 0.0, Bx[min(max(ys, 0), ny - 1) * nx + x], v);
            }
            double* o = pl + y * PX + x;
            *o = fma(cf, v, *o);
          }
          next(y, x);
        }
      }
    }
  }
  // the scale of the solve's input
  const double scale = J.scale;
  {
    int y = ty0, x = tx0;
    for (int k = tid; k < n; k += NT) {
      pl[y * PX + x] *= scale;
      next(y, x);
    }
  }
}

template <bool HI>
__device__ __forceinline__ void plane_couple_p(const PlaneJob& J, int z, double* pl, double* wk) {
  if constexpr (HI) {
    if (J.p == 5) return plane_couple<5, kPTC>(J, z, pl, wk);
    if (J.p == 4) return plane_couple<4, kPTC>(J, z, pl, wk);
  }
  if (J.p == 1) plane_couple<1, kPTC>(J, z, pl, wk);
  else if (J.p == 2) plane_couple<2, kPTC>(J, z, pl, wk);
  else plane_couple<3, kPTC>(J, z, pl, wk);
}

// x-lines of a plane already in LDS (the coupled input): both passes in LDS
template <int P>
__device__ __forceinline__ void plane_x_lds(double* col, int nx, const double* fxl) {
  fwd_st<P>(col, 1, nx, fxl);
  bwd_st<P, false>(col, 1, nullptr, 0, nx, fxl);
}
template <bool HI>
__device__ __forceinline__ void plane_x_lds_p(int p, double* col, int nx, const double* fxl) {
  if constexpr (HI) {
    if (p == 5) return plane_x_lds<5>(col, nx, fxl);
    if (p == 4) return plane_x_lds<4>(col, nx, fxl);
  }
  if (p == 1) plane_x_lds<1>(col, nx, fxl);
  else if (p == 2) plane_x_lds<2>(col, nx, fxl);
  else plane_x_lds<3>(col, nx, fxl);
}

// CPL: the launch holds jobs with coupling terms (a separate instantiation,
// so that the plain in-plane sweeps keep their registers).
template <bool HI, bool CPL>
__global__ __launch_bounds__(CPL ? kPTC : kPT, 1) void sweep_plane_kernel(const LaunchHdr* __restrict__ hdr) {
  constexpr int NT = CPL ? kPTC : kPT;
  extern __shared__ double lds[];
  const int njobs = hdr->njobs, total = hdr->total_tiles;
  const PlaneJob* __restrict__ jobs = hdr_jobs<PlaneJob>(hdr);
  const int tid = threadIdx.x;
  int staged = -1;   // job whose factor rows are in LDS
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int jb = find_job_plane(jobs, njobs, t);
    const PlaneJob& J = jobs[jb];
    const int nx = J.nx, ny = J.ny, p = J.p, PX = nx + 1, n = nx * ny;
    double* pl = lds;
    double* fxl = pl + (size_t)ny * PX;
    double* fyl = fxl + (2 * p + 1) * nx;
    __syncthreads();   // the previous plane's last reads of the LDS are done
    if (jb != staged) {
      const gmem<double>* lx = gview(J.fx.L);
      const gmem<double>* ux = gview(J.fx.U);
      const gmem<double>* rx = gview(J.fx.rd);
      const gmem<double>* ly = gview(J.fy.L);
      const gmem<double>* uy = gview(J.fy.U);
      const gmem<double>* ry = gview(J.fy.rd);
      for (int k = tid; k < nx * p; k += NT) {
        fxl[k] = lx[k];
        fxl[nx * p + k] = ux[k];
      }
      for (int k = tid; k < nx; k += NT) fxl[2 * nx * p + k] = rx[k];
      for (int k = tid; k < ny * p; k += NT) {
        fyl[k] = ly[k];
        fyl[ny * p + k] = uy[k];
      }
      for (int k = tid; k < ny; k += NT) fyl[2 * ny * p + k] = ry[k];
      staged = jb;
      __syncthreads();
    }
    const long long gb = (long long)(t - J.tile0) * n;
    gmem<double>* __restrict__ gout = gview(J.out) + gb;
    if (CPL && J.nterm > 0) {
      // coupled input formed in LDS, then the x-lines in LDS
      plane_couple_p<HI>(J, t - J.tile0, pl, fyl + (2 * p + 1) * ny);
      __syncthreads();
      for (int y = tid; y < ny; y += NT) plane_x_lds_p<HI>(p, pl + y * PX, nx, fxl);
    } else {
      const gmem<double>* __restrict__ gin = gview(J.in) + gb;
      const double scale = J.scale;
      // x-lines: the forward pass reads the line from global memory (the
      // plane's loads overlap the recurrences), the backward pass works in
      // LDS; a thread per line, lanes a padded row apart
      for (int y = tid; y < ny; y += NT) {
        double* col = pl + y * PX;
        const gmem<double>* src = gin + (long long)y * nx;
        plane_x_p<HI>(p, src, scale, col, nx, fxl);
      }
    }
    __syncthreads();
    // y-lines: forward pass in LDS, the backward pass stores each final
    // value (a row of adjacent lanes: coalesced) instead of writing it back
    for (int x = tid; x < nx; x += NT) {
      plane_y_p<HI>(p, pl + x, PX, gout + x, nx, ny, fyl);
    }
  }
}

// Launches whose jobs have a degree above 3 take the HI instantiations.
static bool hi_degree(int pmax) { return pmax >= 4; }

template <bool CPL>
static const void* plane_fn(int pmax) {
  return hi_degree(pmax) ? (const void*)sweep_plane_kernel<true, CPL> : (const void*)sweep_plane_kernel<false, CPL>;
}

int plane_blocks_per_cu(size_t lds_bytes, int pmax, bool coupled) {
  int n = 0;
  const void* k = coupled ? plane_fn<true>(pmax) : plane_fn<false>(pmax);
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, coupled ? kPTC : kPT, lds_bytes);
  const int by_lds = (int)((160 * 1024) / std::max<size_t>(lds_bytes, 1));
  if (e != hipSuccess || n <= 0) n = by_lds;
  return std::max(1, std::min(n, by_lds));
}

hipError_t launch_planes(const LaunchHdr* d_hdr, int grid, size_t lds_bytes, int pmax, bool coupled, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (lds_bytes > (size_t)160 * 1024) return hipErrorInvalidValue;
  if (pmax < 1 || pmax > kMaxP) return hipErrorInvalidValue;
  const bool hi = hi_degree(pmax);
  if (coupled) {
    if (hi) hipLaunchKernelGGL((sweep_plane_kernel<true, true>), dim3(grid), dim3(kPTC), lds_bytes, s, d_hdr);
    else hipLaunchKernelGGL((sweep_plane_kernel<false, true>), dim3(grid), dim3(kPTC), lds_bytes, s, d_hdr);
  } else {
    if (hi) hipLaunchKernelGGL((sweep_plane_kernel<true, false>), dim3(grid), dim3(kPT), lds_bytes, s, d_hdr);
    else hipLaunchKernelGGL((sweep_plane_kernel<false, false>), dim3(grid), dim3(kPT), lds_bytes, s, d_hdr);
  }
  return hipGetLastError();
}

// Dynamic LDS of a workgroup: the factor rows (2 pmax + 1 per line
// position) and kWaves tiles of max_m rows of pitch W + 1.
static size_t sweep_lds_bytes(int W, int max_m, int pmax) {
  return (size_t)(2 * pmax + 1 + kWaves * (W + 1)) * max_m * sizeof(double);
}

template <bool HI>
static const void* sweep_fn(int W) {
  if (W == 16) return (const void*)sweep_kernel<16, HI>;
  if (W == 8) return (const void*)sweep_kernel<8, HI>;
  return (const void*)sweep_kernel<4, HI>;
}

// Resident workgroups per CU for lines of at most max_m unknowns.
static int sweep_resident(int W, int max_m, int pmax) {
  const size_t lds = sweep_lds_bytes(W, max_m, pmax);
  int n = 0;
  const void* k = hi_degree(pmax) ? sweep_fn<true>(W) : sweep_fn<false>(W);
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kNT, lds);
  const int by_lds = (int)((160 * 1024) / std::max<size_t>(lds, 1));
  if (e != hipSuccess || n <= 0) n = by_lds;
  return std::max(1, std::min(n, by_lds));
}

bool sweep_width_fits(int W, int max_m, int pmax) {
  return (W == 4 || W == 8 || W == 16) && sweep_lds_bytes(W, max_m, pmax) <= (size_t)160 * 1024;
}

// Default tile width for a launch over `lines` lines of at most max_m
// unknowns on ncu CUs (the pool's autotuner and ads_set_launch_shape may
// choose another).  Measured on 128-long lines: W = 16 (rows of 128
// contiguous bytes in the y/z access) beats 8 and 4 both for one 128^3
// simulation and for a batch of four; narrower tiles remain for launches
// with too few lines to give every CU a group, and for lines too long for
// four 16-line tiles in LDS.
int sweep_width_for(long long lines, int max_m, int ncu, int pmax) {
  for (int W : {16, 8}) {
    if (sweep_width_fits(W, max_m, pmax) && lines >= (long long)ncu * kWaves * W) return W;
  }
  return 4;   // fits for lines up to 728 long at p = 5 (the library accepts up to 512)
}

// Groups of 4W lines in a job of `lines` lines.
int sweep_groups(long long lines, int W) { return (int)((lines + (long long)kWaves * W - 1) / (kWaves * W)); }

int sweep_blocks_per_cu(int W, int max_m, int pmax) { return sweep_resident(W, max_m, pmax); }

hipError_t launch_sweeps(const LaunchHdr* d_hdr, int grid, int W, int max_m, int pmax, hipStream_t s) {
  const size_t lds = sweep_lds_bytes(W, max_m, pmax);
  if (grid <= 0) return hipSuccess;
  if (W != 16 && W != 8 && W != 4) return hipErrorInvalidValue;
  if (pmax < 1 || pmax > kMaxP) return hipErrorInvalidValue;
  const int frows = 2 * pmax + 1;
  const bool hi = hi_degree(pmax);
  if (W == 16) {
    if (hi) hipLaunchKernelGGL((sweep_kernel<16, true>), dim3(grid), dim3(kNT), lds, s, d_hdr, max_m, frows);
    else hipLaunchKernelGGL((sweep_kernel<16, false>), dim3(grid), dim3(kNT), lds, s, d_hdr, max_m, frows);
  } else if (W == 8) {
    if (hi) hipLaunchKernelGGL((sweep_kernel<8, true>), dim3(grid), dim3(kNT), lds, s, d_hdr, max_m, frows);
    else hipLaunchKernelGGL((sweep_kernel<8, false>), dim3(grid), dim3(kNT), lds, s, d_hdr, max_m, frows);
  } else {
    if (hi) hipLaunchKernelGGL((sweep_kernel<4, true>), dim3(grid), dim3(kNT), lds, s, d_hdr, max_m, frows);
    else hipLaunchKernelGGL((sweep_kernel<4, false>), dim3(grid), dim3(kNT), lds, s, d_hdr, max_m, frows);
  }
  return hipGetLastError();
}

hipError_t sweep_set_attributes() {
  const void* ks[] = {plane_fn<false>(1), plane_fn<false>(5), plane_fn<true>(1), plane_fn<true>(5),
                      sweep_fn<false>(16), sweep_fn<false>(8), sweep_fn<false>(4),
                      sweep_fn<true>(16), sweep_fn<true>(8), sweep_fn<true>(4)};
  for (const void* k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ads
