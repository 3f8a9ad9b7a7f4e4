// Layout copies, projection contractions, counters.
#include "common.hpp"

namespace ads {

// Free (Dirichlet-eliminated) <-> full coefficient layouts, ncomp components.
__global__ void full_to_free_kernel(const double* __restrict__ full, double* __restrict__ fr, int n0, int n1,
                                    int n2, int f0, int f1, int f2, int o0, int o1, int o2, int ncomp) {
  const long long nfree = (long long)f0 * f1 * f2, nfull = (long long)n0 * n1 * n2;
  const long long tot = nfree * ncomp;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    long long c = idx / nfree, r = idx - c * nfree;
    int x = (int)(r % f0);
    long long r2 = r / f0;
    int y = (int)(r2 % f1), z = (int)(r2 / f1);
    fr[idx] = full ? full[c * nfull + ((long long)(z + o2) * n1 + (y + o1)) * n0 + (x + o0)] : 0.0;
  }
}

__global__ void free_to_full_kernel(const double* __restrict__ fr, double* __restrict__ full, int n0, int n1,
                                    int n2, int f0, int f1, int f2, int o0, int o1, int o2, int ncomp) {
  const long long nfree = (long long)f0 * f1 * f2, nfull = (long long)n0 * n1 * n2;
  const long long tot = nfull * ncomp;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    long long c = idx / nfull, r = idx - c * nfull;
    int x = (int)(r % n0);
    long long r2 = r / n0;
    int y = (int)(r2 % n1), z = (int)(r2 / n1);
    int fx = x - o0, fy = y - o1, fz = z - o2;
    double v = 0.0;
    if (fx >= 0 && fx < f0 && fy >= 0 && fy < f1 && fz >= 0 && fz < f2)
      v = fr[c * nfree + ((long long)fz * f1 + fy) * f0 + fx];
    full[idx] = v;
  }
}

// One direction of the projection right-hand side b_i = int B_i g:
// out[o][c][i] = sum over elements e touching coefficient c+off and their Gauss
// points g of N[e][g][c+off-e] * W[e][g] * in[o][e*q+g][i].
__global__ void proj_contract_kernel(const double* __restrict__ in, double* __restrict__ out, long long outer,
                                     int E, int q, int P, int nf, int off, long long inner,
                                     const double* __restrict__ tab) {
  const long long tot = outer * nf * inner;
  const double* N = tab;
  const double* W = tab + 2ll * E * q * P;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    long long i = idx % inner, r = idx / inner;
    int c = (int)(r % nf);
    long long o = r / nf;
    int cf = c + off;
    double s = 0.0;
    for (int a = 0; a < P; ++a) {
      int e = cf - a;
      if (e < 0 || e >= E) continue;
      for (int g = 0; g < q; ++g)
        s += N[((long long)e * q + g) * P + a] * W[(long long)e * q + g] *
             in[(o * ((long long)E * q) + (long long)e * q + g) * inner + i];
    }
    out[idx] = s;
  }
}

__global__ void set_u64_kernel(unsigned long long* p, unsigned long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void fill_kernel(double* p, long long n, double v) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x)
    p[idx] = v;
}

__global__ void axpby_kernel(double* out, const double* x, const double* y, double a, double b, long long n) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x)
    out[idx] = a * x[idx] + (y ? b * y[idx] : 0.0);
}

// out = x + b y + c z (z optional), as fma(c, z, fma(b, y, x)): the
// Newmark predictor w = u + tau v + eta a of a state, and back u = w -
// tau v - eta a.
__global__ void lin3_kernel(double* out, const double* x, const double* y, const double* z, double b, double c,
                            long long n) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const double t = fma(b, y[idx], x[idx]);
    out[idx] = z ? fma(c, z[idx], t) : t;
  }
}

// Count non-finite entries (any positive count means failure).
__global__ void nonfinite_kernel(const double* x, long long n, unsigned long long* cnt) {
  unsigned long long local = 0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x)
    if (!isfinite(x[idx])) local++;
  if (local) atomicAdd(cnt, local);
}

// Dot product in a fixed order (deterministic): every block sums a
// grid-stride slice and reduces it by a fixed tree; one block then reduces
// the kDotBlocks partial sums the same way.
constexpr int kDotBlocks = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(256) void dot_partial_kernel(const double* x, const double* y, long long n,
                                                          double* partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    acc = fma(x[i], y[i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void dot_final_kernel(const double* partial, int nb, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = t;
}

static inline int grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_full_to_free(const double* full, double* fr, const int n[3], const int nf[3], const int off[3],
                               int ncomp, hipStream_t s) {
  long long tot = (long long)nf[0] * nf[1] * nf[2] * ncomp;
  hipLaunchKernelGGL(full_to_free_kernel, dim3(grid_for(tot)), dim3(256), 0, s, full, fr, n[0], n[1], n[2],
                     nf[0], nf[1], nf[2], off[0], off[1], off[2], ncomp);
  return hipGetLastError();
}

hipError_t launch_free_to_full(const double* fr, double* full, const int n[3], const int nf[3], const int off[3],
                               int ncomp, hipStream_t s) {
  long long tot = (long long)n[0] * n[1] * n[2] * ncomp;
  hipLaunchKernelGGL(free_to_full_kernel, dim3(grid_for(tot)), dim3(256), 0, s, fr, full, n[0], n[1], n[2],
                     nf[0], nf[1], nf[2], off[0], off[1], off[2], ncomp);
  return hipGetLastError();
}

hipError_t launch_proj_contract(const double* in, double* out, long long outer, int E, int q, int P, int nf,
                                int off, long long inner, const double* tab, hipStream_t s) {
  long long tot = outer * nf * inner;
  hipLaunchKernelGGL(proj_contract_kernel, dim3(grid_for(tot)), dim3(256), 0, s, in, out, outer, E, q, P, nf,
                     off, inner, tab);
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_axpby(double* out, const double* x, const double* y, double a, double b, long long n,
                        hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, out, x, y, a, b, n);
  return hipGetLastError();
}

hipError_t launch_lin3(double* out, const double* x, const double* y, const double* z, double b, double c,
                       long long n, hipStream_t s) {
  hipLaunchKernelGGL(lin3_kernel, dim3(grid_for(n)), dim3(256), 0, s, out, x, y, z, b, c, n);
  return hipGetLastError();
}

int dot_scratch_doubles() { return kDotBlocks; }

hipError_t launch_dot(const double* x, const double* y, long long n, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks), dim3(256), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, partial, kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double* x, long long n, unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, cnt);
  return hipGetLastError();
}

}  // namespace ads
