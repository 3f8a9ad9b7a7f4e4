// Internal types shared by the host side and the gfx950 kernels.
//
// Field layout on the device: FREE coefficients only (zero-Dirichlet
// eliminated), nf_x * nf_y * nf_z doubles per component, [z][y][x] with x
// fastest.  Full-index coefficient c of direction d has free index
// c - off[d] (off = 1 for zero Dirichlet).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ads {

constexpr int kMaxP = 5;          // spline degrees 1 to 5 are instantiated

// Every launch reads its job count and tile count from a device-side header
// that precedes its job table, so that a captured graph can be replayed
// while the tables are rewritten (batches that change between replays).
struct alignas(256) LaunchHdr {
  int njobs;
  int total_tiles;
};
template <class Job>
__host__ __device__ inline const Job* hdr_jobs(const LaunchHdr* h) {
  return reinterpret_cast<const Job*>(h + 1);
}

// Global-memory views of the device pointers held in job tables.  Through a
// plain pointer read from memory the compiler cannot tell global memory from
// LDS and emits flat loads and stores, which count on the same wait counter
// as LDS and scalar loads: every LDS wait would then also wait for all
// global loads in flight (no prefetch survives it).  Accesses through these
// views are global loads and stores, waited for on their own counter.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ const gmem<T>* gview(const T* p) {
  return (const gmem<T>*)p;
}
template <class T>
__device__ __forceinline__ gmem<T>* gview(T* p) {
  return (gmem<T>*)p;
}

// Read-only view (constant address space) of tables that no kernel writes
// while it runs: loads at wave-uniform addresses become scalar loads, which
// neither occupy vector registers nor wait behind vector loads in flight.
template <class T>
using cmem = __attribute__((address_space(4))) T;
template <class T>
__device__ __forceinline__ const cmem<T>* cview(const T* p) {
  return (const cmem<T>*)p;
}

// One 1D banded factor (banded LU without pivoting of a free-row block):
// L[i*p + k-1] = l_{i,i-k}, U[i*p + k-1] = u_{i,i+k} (zero where the index
// leaves the matrix), rd[i] = 1 / u_{ii}.
struct Factor1D {
  const double* L;
  const double* U;
  const double* rd;
  int m;
};

// Epilogue applied by a sweep to every solved value x at global offset g.
enum SweepEpi : int {
  EPI_STORE = 0,     // out[g] = x
  // Newmark on the state (w, b, a): w = u + tau v + eta a the predictor of
  // the next step, b = v + tau/2 a the half-step velocity (v = b - tau/2 a,
  // u = w - tau v - eta a).  With a' = x, v' = v + tau/2 (a + a') and
  // u' = w + eta a' (eta = tau^2/4) they advance as
  //   w' = u' + tau v' + eta a' = w + tau b + tau^2 a',  b' = b + tau a'
  // (two fields read, three written: a' is kept for the state's readers)
  EPI_NEWMARK = 1,
  EPI_THREELEVEL = 2, // out[g] = x; U^{n-1} <- U^n; U^n <- 2 U^n - U^{n-1} + x
  // printed coefficient set on (w, v, a), w = u + tau v:
  //   a' = x; u' = w (u + tau v, old v); v' = v + tau/2 a'; w' = u' + tau v'
  EPI_NEWMARK_LITERAL = 3
};

// One set of line solves of a field along one direction.
struct SweepJob {
  const double* in;
  double* out;
  Factor1D f;
  int dir;          // 0: x-lines (contiguous), 1: y-lines, 2: z-lines
  int p;
  int nx, ny, nz;   // free sizes of the field
  int nlines;
  int tile0;        // first global tile index of this job
  int ntiles;
  int epi;
  double scale;     // the input is multiplied by this before the solve
  double c0, c1;    // EPI_NEWMARK: tau, tau^2   EPI_NEWMARK_LITERAL: tau
  double* e0;       // EPI_NEWMARK(_LITERAL): w   EPI_THREELEVEL: U^n
  double* e1;       // EPI_NEWMARK: b (literal: v)   EPI_THREELEVEL: U^{n-1}
  double* e2;       // EPI_NEWMARK(_LITERAL): a
  unsigned long long* counter;  // incremented once by the job (end of a step)
};

// One tensor-product term coef * (T_x (x) T_y (x) T_z) src of an elasticity
// coupling.
struct KronTerm {
  const double* src;
  const double* T[3];     // banded [m][2p+1], band[i*(2p+1) + (j-i+p)]
  double coef;
};
constexpr int kPlaneMaxTerms = 5;   // PlaneJob::term

// The x- then the y-sweep of every z-plane of a field, the plane held in
// LDS (the in-plane pair of a direction-split solve).  With nterm > 0 the
// input of plane z is  in + sum_t coef_t (T^t_x (x) T^t_y (x) T^t_z) src_t
// at that plane (in may then be null: no base), formed in LDS before the
// solve (the coupling of an alternating-triangular stage fused into the
// solve that consumes it).
struct PlaneJob {
  const double* in;
  double* out;
  Factor1D fx, fy;
  int p;
  int nx, ny, nz;   // free sizes of the field
  double scale;     // the input is multiplied by this before the solve
  int tile0;        // first global tile (plane) index of this job
  int ntiles;       // = nz
  int nterm;
  KronTerm term[kPlaneMaxTerms];
};

// Right-hand side by sum-factorized Gauss quadrature on one field
// (P-wave) or three fields (elasticity).
struct RhsJob {
  // state: P-wave w = cu*u + cv*v + ca*a (free layout; the Kronecker-form
  // kernel takes v = a = null); elasticity uses u as U^n (3 components,
  // comp stride nfree) and ignores v, a.
  const double* u;
  const double* v;
  const double* a;
  double cu, cv, ca;
  double* R;              // output (free layout, comps as input)
  const double* load;     // load vector (free layout) or null
  const double* amp;      // amplitude table or null
  int namp;
  int amp_shift;          // amplitude index = *counter + amp_shift
  const unsigned long long* counter;
  double rscale;          // R = rscale * (amp * load - A(w))
  int wsplit;             // P-wave: contract w (0), its BF16 rounding hi (1), or w - hi (2)
  int accumulate;         // 1: R += rscale * (amp * load - A(w)) instead of R =
  const double* coef;     // P-wave: c^2 at every Gauss point [Ez q][Ey q][Ex q], or null (c^2 = 1)
  double lam, mu;         // elasticity Lame constants
  const double* tab[3];   // per direction: N, D [E][q][P], W [E][q], W*N, W*D [E][q][P], M_e, K_e [E][P][P]
  const double* band[3];  // per direction: the assembled bands M, K (elasticity: G, G^T) [nf][2p+1] after them
  int E[3], nf[3], off[3];
  int tiles[3];           // tiles along x, y, and z-chunks
  int TZ;                 // owned z-coefficients per chunk
  int tile0, ntiles;
};

// Apply of a sum of tensor products of 1D banded matrices (elasticity
// couplings):  out = alpha*base + sum_t coef_t * (T^t_x (x) T^t_y (x) T^t_z) src_t
struct KronJob {
  double* out;
  const double* base;
  double alpha;
  KronTerm term[6];
  int nterm;
  int p;
  int nx, ny, nz;
  int TZ;           // output z-layers per tile
  int tiles[3];     // tiles per direction (x, y: column tiles; z: chunks)
  int tile0, ntiles;
};

}  // namespace ads
