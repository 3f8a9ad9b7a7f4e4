// Right-hand side of the P-wave step by sum-factorized Gauss quadrature
// (Section 2: testing the equation gives (grad B_i, grad w_h) for the
// stiffness action, written as K = K_x(x)M_y(x)M_z + ... in eq. pwave2; here
// it is evaluated element by element at the q^3 Gauss points as a chain of
// 1D contractions instead of assembling K):
//
//   R_i = rscale * ( amp * b_i - sum_e sum_g W_g grad B_i(x_g) . grad w_h(x_g) ),
//   w   = cu*u + cv*v + ca*a   (the Newmark predictor u + tau u' + tau^2/4 u'').
//
// Tiling on gfx950 (owner computes, no atomics, deterministic):
//   * a workgroup owns TX x TY coefficient columns and a z-range of TZ
//     coefficients, and marches over the element layers touching the range;
//   * the predictor w is formed once per coefficient (FP64) into an LDS ring
//     of p+1 coefficient layers (halo p on each side in x and y), the next
//     layer's global loads in flight while the current one is processed;
//   * per element layer (Z): the z-contraction of every ring column at all q
//     z Gauss points (value and z-derivative), once per column;
//   * per z Gauss point: (Y) y-contraction to the y Gauss rows of the tile's
//     y-elements (value, y- and z-derivative); (X) x-forward, x-weights and
//     x-backward with one lane per x-element (16-lane DPP rows, one Gauss row
//     each) and a row-shift Horner sum that assembles each coefficient from
//     its p+1 elements; (B) y-backward (y-weights folded into per-thread
//     tables) and z-backward (z-weights folded into the z tables) into FP64
//     accumulators of the owned column (p+1 z-layers in flight);
//   * the Gauss-row buffer is double-buffered: two barriers per z Gauss point
//     and one per element layer;
//   * a z-layer is written once its last contributing element is done.
// With a wave-speed field (c^2 at the Gauss points) the three point
// gradients are scaled by it between the x-forward and x-backward stages.
// Variant MX (FP32 with a field) runs that x-stage on the matrix cores: one
// 4x4x1 MFMA block per x-element (16 per wave), its four columns four Gauss
// rows, the element's own x-tables as the A operand (boundary elements need
// no special case); the forward result lands in the registers that the
// backward contraction takes as its B operand, and the backward result is
// assembled across elements with lane permutes.  It is slower than the
// VALU form (its chain of dependent MFMAs and permutes per row group is
// latency-bound), so the autotuner keeps it only where it measures faster.
// Without one (CF false) nothing pointwise separates a channel's forward and
// backward contraction in any direction, and each pair collapses to an
// element matrix, M_d = sum_g w_g N_g N_g^T or K_d = sum_g w_g D_g D_g^T:
// the element's contribution is (K_x(x)M_y(x)M_z + M_x(x)K_y(x)M_z +
// M_x(x)M_y(x)K_z) w_e, the same sum up to rounding (q = p+1 is exact).
// The stages keep their places: (Z) M_z r and K_z r per column, the loop
// over z Gauss points runs over the element's local z-slots; (Y) M_y of the
// z-value channel and K_y of it plus M_y of the z-derivative channel,
// summed (both meet M_x next); (X) K_x and M_x in one chain, one assembled
// value per row; (B) plain sums into the FP64 accumulators.
// Derivative tables satisfy sum_a D_a = 0 on every element (partition of
// unity), so the forward derivative contractions use differences against
// the first coefficient and the backward x-derivative slot 0 is minus the
// sum of the others; likewise the stiffness matrices act on differences.
// T is the contraction type: double (FP64 mode) or float (mixed mode: FP32
// contractions, FP64 predictor, FP64 z-accumulation and assembly).
#include "common.hpp"
#include "launch.hpp"

namespace ads {

__device__ __forceinline__ int find_job_rhs(const RhsJob* jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Row shift within 16-lane DPP rows: lane i receives lane i-1; lane 0 of
// each row reads 0 (bound_ctrl), so no "old" value has to be set up.
__device__ __forceinline__ double row_shr1(double x) {
  long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xF, 0xF, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float row_shr1(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xF, 0xF, true));
}

// x rounded to the nearest BF16 value (ties to even), as an FP32 value;
// finite inputs only (the predictor of a finite state)
__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// sum_a o[a] of lane i-a, as a Horner chain of one-lane shifts
template <int P, typename T>
__device__ __forceinline__ T horner_shift(const T (&o)[P]) {
  T t = o[P - 1];
#pragma unroll
  for (int a = P - 2; a >= 0; --a) t = o[a] + row_shr1(t);
  return t;
}

// Completes this wave's LDS writes before its lanes read each other's
// values (LDS operations of one wave execute in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef float f4 __attribute__((ext_vector_type(4)));

// One 4x4x1 MFMA step over 16 blocks: block b (lanes 4b..4b+3) adds the
// outer product of a (lane 4b+i gives row i) and b (lane 4b+j gives column
// j); lane 4b+j holds column j of its block, element i in register i.
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// value of lane - 4 (the previous 4x4 block); lanes 0-3 get lanes 60-63
__device__ __forceinline__ float lane_sub4(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane - 4) & 63) << 2, __float_as_int(v)));
}

template <typename T, int P, int Q, int TY_, int NT_, bool CF>
struct RhsGeom {
  static constexpr int p = P - 1;
  static constexpr int G = 16;          // lanes per Gauss row (x-elements of the tile)
  static constexpr int TX = G - p;      // owned x-coefficients
  static constexpr int TY = TY_;        // owned y-coefficients
  static constexpr int TXH = TX + 2 * p;
  static constexpr int TYH = TY + 2 * p;
  static constexpr int NC = TYH * TXH;  // coefficient positions of one layer
  static constexpr int EY = TY + p;     // y-elements touching the owned columns
  static constexpr int R = EY * Q;      // y Gauss rows
  static constexpr int NT = NT_;
  static constexpr int NW = NT / 64;    // waves
  static constexpr int WE = 4;          // y-elements per wave
  static constexpr int WR = WE + p;     // coefficient rows a wave's y-elements touch
  static constexpr int NZW = WR * TXH;  // z-stage items of one wave
  static constexpr int NZ = (NZW + 63) / 64;
  static constexpr int NF = (NC + NT - 1) / NT;   // predictor loads per thread
  // Gauss-row buffer: row r, column x at (r & 1) * H + (r >> 1) * RP + x;
  // H = 16 (mod 32) puts the two rows read by one half-wave (rows r, r+1 of
  // the x-stage) on disjoint LDS banks.  In FP32 the row pitch RP keeps
  // rows r and r + q, which one half-wave of the y-stage stores, 16 banks
  // apart as well: RP = 0 (mod 32) for odd q, RP = 8 (mod 16) for even q
  static constexpr int RP = sizeof(T) != 4 ? TXH
                            : (Q % 2) ? (TXH + 31) / 32 * 32
                                      : (TXH + 7) / 16 * 16 + 8;
  static constexpr int HR = (R / 2) * RP;
  static constexpr int H = HR + ((16 - HR % 32) + 32) % 32;
  static constexpr int SBC = 2 * H;     // one component plane
  static constexpr int TS = 2 * Q * P + (sizeof(T) == 4 ? (4 - (2 * Q * P) % 4) % 4 : 0);
  // channels of a Gauss row: three with a wave-speed field; two without
  // (the collapsed form sums the y- and z-derivative channels)
  static constexpr int NCH = CF ? 3 : 2;
  // LDS: ring [P][NC], zc [NW][Q][2][NZW], sb [2][NCH][SBC], ty [EY][TS]
  static constexpr size_t lds_elems =
      (size_t)P * NC + (size_t)NW * Q * 2 * NZW + 2ull * NCH * SBC + (size_t)EY * TS;
  static constexpr size_t lds_bytes = lds_elems * sizeof(T);
  static_assert(EY == WE * NW, "every wave owns WE y-elements");
  static_assert((WE * Q) % 4 == 0, "a wave's Gauss rows split over its four row groups");
  static_assert(R % 2 == 0, "rows come in even/odd pairs");
  static_assert(TX * TY <= NT, "every owned column needs a thread");
  static_assert(lds_bytes <= 160 * 1024, "LDS budget of one workgroup");
};

// FP32 p = 2: at least four waves per SIMD (three with a field; five for
// the four-wave workgroups without one, whose LDS allows five per CU).  CF:
// the jobs carry a wave-speed field (a separate instantiation, so that the
// constant coefficient kernels keep their registers).
template <typename T, int P, int Q, int TY_, int NT_, bool CF, bool MX = false>
__global__ __launch_bounds__(NT_, (sizeof(T) == 4 && P == 3) ? (CF ? 3 : (NT_ <= 256 ? 5 : 4)) : 1) void rhs_pwave_kernel(
    const LaunchHdr* __restrict__ hdr) {
  const int njobs = hdr->njobs, total_tiles = hdr->total_tiles;
  const RhsJob* __restrict__ jobs = hdr_jobs<RhsJob>(hdr);
  using Gm = RhsGeom<T, P, Q, TY_, NT_, CF>;
  constexpr int p = Gm::p, TX = Gm::TX, TY = Gm::TY, TXH = Gm::TXH, TYH = Gm::TYH, NC = Gm::NC, EY = Gm::EY,
                RP = Gm::RP,
                NT = Gm::NT, NW = Gm::NW, WE = Gm::WE, NZW = Gm::NZW, NZ = Gm::NZ,
                NF = Gm::NF, H = Gm::H, SBC = Gm::SBC, TS = Gm::TS;
  constexpr int NRW = WE * Q / 4;       // Gauss rows per row group
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ring = reinterpret_cast<T*>(smem_raw);   // [P][NC]
  T* zcall = ring + P * NC;                    // [NW][Q][2][NZW]
  T* sb = zcall + NW * Q * 2 * NZW;            // [2][NCH][SBC]
  T* tyl = sb + 2 * Gm::NCH * SBC;             // [EY][TS]: N[Q][P] then D[Q][P] (My, Ky without a field)
  auto rowpos = [](int r) { return (r & 1) * H + (r >> 1) * RP; };
  // position of row r0 + k from that of row r0 (par = r0 & 1)
  auto rowstep = [](int pos0, int par, int k) {
    const int even = (k & 1) * H + (k >> 1) * RP;
    const int odd = (k & 1) ? ((k + 1) >> 1) * RP - H : (k >> 1) * RP;
    return pos0 + (par ? odd : even);
  };

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int j = lane & 15;                // x-element slot within the Gauss row group
  const int grp = lane >> 4;              // row group within the wave
  const bool own = tid < TX * TY;
  const int cxo = tid % TX, cyo = tid / TX;
  T* zc = zcall + wv * (Q * 2 * NZW);     // this wave's z-contracted rows
  // y-stage, full pass: lane = (wave y-element el, column cxl < 16), all
  // Gauss points; extra pass: the p columns 16.. as (el, column, gy) items
  constexpr int NYX = p * WE * Q;
  static_assert(WE * 16 == 64 && NYX <= 64, "y-stage lane mapping");
  const int yel = lane >> 4;
  const int yr0 = (wv * WE + yel) * Q;
  const int ysb = rowpos(yr0) + j, ypar = yr0 & 1, yty = (wv * WE + yel) * TS, yzc = yel * TXH + j;
  const bool xok = lane < NYX;
  int xsb, xty, xzc, xa;
  {
    const int gy = lane % Q, rest = lane / Q;
    const int el = rest / p, cx = 16 + rest % p;
    xsb = rowpos((wv * WE + el) * Q + gy) + cx;
    xty = (wv * WE + el) * TS + gy * P;
    xzc = el * TXH + cx;
    xa = gy;   // without a field: the row's local y-slot
  }
  // x-stage rows of this row group: wave rows 4i + grp (same parity as
  // grp, so row i sits 2i rows of RP further on)
  const int xrow0 = rowpos(wv * WE * Q + grp);
  // MFMA x-stage (variant MX): lane = 4 * (x-element slot mb) + mj, mj the
  // Gauss row of the group of four for the B operand and the output, and
  // the Gauss point (forward) or slot (backward) row of the A operand
  constexpr bool MF = MX && CF && sizeof(T) == 4;
  static_assert(!MF || (P <= 4 && Q <= 4), "an element's x-tables fit one 4x4 block");
  const int mb = lane >> 2, mj = lane & 3;
  const int xrowm0 = rowpos(wv * WE * Q + mj) + mb;
  // b-stage rows of the owned column: cyo*Q + (p - b)*Q + gy
  const int brow0 = rowpos(cyo * Q) + cxo, bpar = (cyo * Q) & 1;

  // each XCD (block b runs on XCD b mod 8) takes one contiguous range of
  // tiles, whose neighbours share their halo columns in its L2; the
  // remainder of total_tiles mod 8 keeps its order
  const int full = total_tiles & ~7;
  for (int wi = blockIdx.x; wi < total_tiles; wi += gridDim.x) {
    const int tile = wi >= full ? wi : (wi & 7) * (full >> 3) + (wi >> 3);
    const RhsJob& J = jobs[find_job_rhs(jobs, njobs, tile)];
    const int t = tile - J.tile0;
    const int tx = t % J.tiles[0];
    const int t2 = t / J.tiles[0];
    const int ty = t2 % J.tiles[1];
    const int tz = t2 / J.tiles[1];
    const int Ex = J.E[0], Ey = J.E[1], Ez = J.E[2];
    const int nfx = J.nf[0], nfy = J.nf[1], nfz = J.nf[2];
    const int ox = J.off[0], oy = J.off[1], oz = J.off[2];
    const int X0 = ox + tx * TX, Y0 = oy + ty * TY, Z0 = oz + tz * J.TZ;
    const int Zend = min(Z0 + J.TZ, oz + nfz);
    const long long sxy = (long long)nfx * nfy;
    const gmem<double>* __restrict__ U = gview(J.u);
    const gmem<double>* __restrict__ V = gview(J.v);
    const gmem<double>* __restrict__ A = gview(J.a);
    const double cu = J.cu, cv = J.cv, ca = J.ca;
    const gmem<double>* __restrict__ C = gview(J.coef);
    const gmem<double>* __restrict__ LD = gview(J.load);
    gmem<double>* __restrict__ R = gview(J.R);
    const double rscale = J.rscale;
    const bool accumulate = J.accumulate != 0;

    const gmem<double>* tyg = gview(J.tab[1]);
    if constexpr (CF) {
      // forward y tables of the tile's y-elements (zero outside the mesh)
      for (int k = tid; k < EY * Q * P; k += NT) {
        const int eyl = k / (Q * P), rest = k - eyl * (Q * P);
        const int ey = Y0 - p + eyl;
        const bool v = ey >= 0 && ey < Ey;
        tyl[eyl * TS + rest] = v ? (T)tyg[(long long)ey * Q * P + rest] : T(0);
        tyl[eyl * TS + Q * P + rest] = v ? (T)tyg[(long long)(Ey + ey) * Q * P + rest] : T(0);
      }
    } else {
      // Without a field the y-forward and y-backward contractions of a
      // channel collapse as in x: per y-element the mass matrix
      // My = sum_g w_g N_g N_g^T, then the stiffness Ky = sum_g w_g D_g D_g^T
      // (columns 1.., acting on differences), formed in FP64 (zero outside
      // the mesh).  Rows of the Gauss-row buffer then hold the local y-slots
      // of an element.
      constexpr int NM = P * P + P * (P - 1);
      static_assert(NM <= 2 * Q * P, "element matrices fit the table stride");
      for (int k = tid; k < EY * NM; k += NT) {
        const int eyl = k / NM, r = k - eyl * NM;
        const int ey = Y0 - p + eyl;
        const bool mass = r < P * P;
        const int rr = mass ? r : r - P * P;
        const int a = mass ? rr / P : rr / (P - 1), b = mass ? rr % P : rr % (P - 1) + 1;
        const long long tb = mass ? 0 : (long long)Ey * Q * P;
        double sm = 0.0;
        if (ey >= 0 && ey < Ey) {
          for (int g = 0; g < Q; ++g) {
            const double w = tyg[2ll * Ey * Q * P + (long long)ey * Q + g];
            const long long o = tb + ((long long)ey * Q + g) * P;
            sm = fma(w * tyg[o + a], tyg[o + b], sm);
          }
        }
        tyl[eyl * TS + r] = (T)sm;
      }
    }
    // backward y tables of the owned column, y-weights folded in:
    // slot b of y-element cyo + p - b at Gauss point gy
    T bN[P][Q], bD[P][Q];
    if constexpr (CF)
#pragma unroll
    for (int b = 0; b < P; ++b) {
      const int ey = Y0 + cyo - b;
      const bool v = own && ey >= 0 && ey < Ey;
#pragma unroll
      for (int gy = 0; gy < Q; ++gy) {
        const double w = v ? tyg[2ll * Ey * Q * P + (long long)ey * Q + gy] : 0.0;
        bN[b][gy] = v ? (T)(w * tyg[((long long)ey * Q + gy) * P + b]) : T(0);
        bD[b][gy] = v ? (T)(w * tyg[((long long)(Ey + ey) * Q + gy) * P + b]) : T(0);
      }
    }
    // x tables of this lane's x-element, kept in registers: forward N, D;
    // backward ones with the x-weights folded in (FP32), or the weights
    // alone, applied to the point values (FP64: fewer registers)
    constexpr bool kFoldX = sizeof(T) == 4;
    constexpr int QW = kFoldX ? Q : 1, QX = kFoldX ? 1 : Q;
    const int ex = X0 - p + j;
    const bool exv = ex >= 0 && ex < Ex;
    T xN[Q][P], xD[Q][P], xNw[QW][P], xDw[QW][P], xW[QX];
    // MFMA x-stage: the tables of x-element mb as A operands: forward
    // N[g = mj][k], D[g = mj][k]; backward (x-weights folded in)
    // w_k N[k][a = mj], w_k D[k][a = mj]; zero in padding rows
    const int exm = X0 - p + mb;
    const bool exvm = exm >= 0 && exm < Ex;
    float mfN[P], mfD[P], mbN[Q], mbD[Q];
    if constexpr (MF) {
      const gmem<double>* txg = gview(J.tab[0]);
      const bool fv = exvm && mj < Q, bv = exvm && mj < P;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        mfN[k] = fv ? (float)txg[((long long)exm * Q + mj) * P + k] : 0.f;
        mfD[k] = fv ? (float)txg[((long long)(Ex + exm) * Q + mj) * P + k] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const double w = bv ? txg[2ll * Ex * Q * P + (long long)exm * Q + k] : 0.0;
        mbN[k] = bv ? (float)(w * txg[((long long)exm * Q + k) * P + mj]) : 0.f;
        mbD[k] = bv ? (float)(w * txg[((long long)(Ex + exm) * Q + k) * P + mj]) : 0.f;
      }
    }
    if constexpr (!MF) {
      const gmem<double>* txg = gview(J.tab[0]);
#pragma unroll
      for (int g = 0; g < Q; ++g) {
        const double w = exv ? txg[2ll * Ex * Q * P + (long long)ex * Q + g] : 0.0;
        if constexpr (!kFoldX) xW[g] = (T)w;
#pragma unroll
        for (int a = 0; a < P; ++a) {
          const double n = exv ? txg[((long long)ex * Q + g) * P + a] : 0.0;
          const double d = exv ? txg[((long long)(Ex + ex) * Q + g) * P + a] : 0.0;
          xN[g][a] = (T)n;
          xD[g][a] = (T)d;
          if constexpr (kFoldX) {
            xNw[g][a] = (T)(w * n);
            xDw[g][a] = (T)(w * d);
          }
        }
      }
    }
    // Without a wave-speed field nothing pointwise sits between the x-forward
    // and the x-backward contraction of a channel, so the pair is one 3x3
    // (PxP) element matrix: the x-stiffness Kx = sum_g w_g D_g D_g^T for the
    // x-derivative channel and the x-mass Mx = sum_g w_g N_g N_g^T for the
    // others; formed in FP64 per lane.  Kx annihilates constants (the
    // derivative tables sum to zero), so it acts on the differences
    // d_b = c_b - c_0 and only its columns 1.. are kept: Kx[a][b-1].
    T Kx[P][P - 1], Mx[P][P];
    if constexpr (!CF) {
      const gmem<double>* txg = gview(J.tab[0]);
      double k[P][P - 1] = {}, mm[P][P] = {};
#pragma unroll
      for (int g = 0; g < Q; ++g) {
        const double w = exv ? txg[2ll * Ex * Q * P + (long long)ex * Q + g] : 0.0;
        double n[P], d[P];
#pragma unroll
        for (int a = 0; a < P; ++a) {
          n[a] = exv ? txg[((long long)ex * Q + g) * P + a] : 0.0;
          d[a] = exv ? txg[((long long)(Ex + ex) * Q + g) * P + a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int b = 0; b < P; ++b) {
            mm[a][b] = fma(w * n[a], n[b], mm[a][b]);
            if (b > 0) k[a][b - 1] = fma(w * d[a], d[b], k[a][b - 1]);
          }
      }
#pragma unroll
      for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) {
          Mx[a][b] = (T)mm[a][b];
          if (b > 0) Kx[a][b - 1] = (T)k[a][b - 1];
        }
    }
    // backward x table entries at Gauss point gx
    auto bxN = [&](int gx, int a) -> T { if constexpr (kFoldX) return xNw[gx][a]; else return xN[gx][a]; };
    auto bxD = [&](int gx, int a) -> T { if constexpr (kFoldX) return xDw[gx][a]; else return xD[gx][a]; };
    double ampv = 0.0;
    if (J.load != nullptr && J.amp != nullptr) {
      long long ai = (long long)(*gview(J.counter)) + J.amp_shift;
      ampv = (ai >= 0 && ai < J.namp) ? gview(J.amp)[ai] : 0.0;
    }

    // predictor loads: ring position k = tid + i*NT, global row offset per tile
    long long prow[NF];
    bool pval[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int k = tid + i * NT;
      const int cyl = k / TXH, cxl = k - cyl * TXH;
      const int cy = Y0 - p + cyl, cx = X0 - p + cxl;
      pval[i] = k < NC && cy >= oy && cy < oy + nfy && cx >= ox && cx < ox + nfx;
      prow[i] = (long long)(cy - oy) * nfx + (cx - ox);
    }
    // (positions outside the mesh load offset 0 and are zeroed: no branch
    // around the loads)
    double pf[NF];
    auto prefetch_layer = [&](int cz) {
      const bool zv = cz >= oz && cz < oz + nfz;
      const long long zo = (long long)(cz - oz) * sxy;
      long long gi[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) gi[i] = (zv && pval[i]) ? zo + prow[i] : 0;
#pragma unroll
      for (int i = 0; i < NF; ++i) pf[i] = cu * U[gi[i]];
      if (V != nullptr) {
#pragma unroll
        for (int i = 0; i < NF; ++i) pf[i] = fma(cv, V[gi[i]], pf[i]);
      }
      if (A != nullptr) {
#pragma unroll
        for (int i = 0; i < NF; ++i) pf[i] = fma(ca, A[gi[i]], pf[i]);
      }
#pragma unroll
      for (int i = 0; i < NF; ++i) pf[i] = (zv && pval[i]) ? pf[i] : 0.0;
    };
    // BF16 input split (wsplit 1 / 2): hi = w rounded to BF16 (through
    // FP32, to nearest even), lo = w - hi in FP64 (exact: hi is within a
    // factor 2 of w); the two passes together contract w
    const int wsplit = J.wsplit;
    auto commit_layer = [&](int cz) {
      T* dst = ring + (cz % P) * NC;
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const int k = tid + i * NT;
        double w = pf[i];
        if (wsplit != 0) {
          const double hi = (double)bf16_round((float)w);
          w = wsplit == 1 ? hi : w - hi;
        }
        if (k < NC) dst[k] = (T)w;
      }
    };
    const long long obase = (long long)(Y0 + cyo - oy) * nfx + (X0 + cxo - ox);
    const bool ocol = own && Y0 + cyo < oy + nfy && X0 + cxo < ox + nfx;
    auto store_out = [&](int cz, double accv) {
      if (ocol && cz >= Z0 && cz < Zend) {
        const long long gi = (long long)(cz - oz) * sxy + obase;
        const double f = (LD != nullptr) ? ampv * LD[gi] : 0.0;
        const double r = rscale * (f - accv);
        R[gi] = accumulate ? R[gi] + r : r;
      }
    };

    double acc[P];
#pragma unroll
    for (int a = 0; a < P; ++a) acc[a] = 0.0;

    const int ez0 = max(0, Z0 - p);
    const int ez1 = min(Ez - 1, Zend - 1);
    for (int cz = ez0; cz <= ez0 + p; ++cz) {
      prefetch_layer(cz);
      commit_layer(cz);
    }
    __syncthreads();

    // z tables at wave-uniform addresses: scalar loads, which do not wait
    // behind the predictor prefetch in flight
    const cmem<double>* tzg = cview(J.tab[2]);
    int buf = 0;
    for (int ez = ez0; ez <= ez1; ++ez) {
      if (ez < ez1) prefetch_layer(ez + P);
      // (Z) z-contraction of this wave's coefficient rows at every z Gauss
      // point (value, z-derivative)
      {
        T nz[Q][P], dz[Q][P];
        // without a field: the layer's element matrices (after the tables:
        // M_e, then K_e, [E][P][P]); the z-forward and z-backward
        // contractions collapse to them, and the loop over z Gauss points
        // below runs over the element's local z-slots instead
        T mz[P][P], kz[P][P - 1];
        if constexpr (CF) {
#pragma unroll
        for (int g = 0; g < Q; ++g)
#pragma unroll
          for (int a = 0; a < P; ++a) {
            nz[g][a] = (T)tzg[((long long)ez * Q + g) * P + a];
            dz[g][a] = (T)tzg[((long long)(Ez + ez) * Q + g) * P + a];
          }
        } else {
          const cmem<double>* tme = tzg + (4ll * Ez * Q * P + (long long)Ez * Q) + (long long)ez * P * P;
          const cmem<double>* tke = tme + (long long)Ez * P * P;
#pragma unroll
          for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
              mz[a][b] = (T)tme[a * P + b];
              if (b > 0) kz[a][b - 1] = (T)tke[a * P + b];
            }
        }
        const T* rs[P];
#pragma unroll
        for (int a = 0; a < P; ++a) rs[a] = ring + ((ez + a) % P) * NC + wv * WE * TXH;
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          const int k = lane + 64 * i;
          if (k < NZW) {
            T r[P];
#pragma unroll
            for (int a = 0; a < P; ++a) r[a] = rs[a][k];
            T dr[P];
#pragma unroll
            for (int a = 1; a < P; ++a) dr[a] = r[a] - r[0];
            if constexpr (CF) {
#pragma unroll
            for (int g = 0; g < Q; ++g) {
              T v = nz[g][0] * r[0], d = dz[g][1] * dr[1];
#pragma unroll
              for (int a = 1; a < P; ++a) v = fma(nz[g][a], r[a], v);
#pragma unroll
              for (int a = 2; a < P; ++a) d = fma(dz[g][a], dr[a], d);
              zc[(2 * g) * NZW + k] = v;
              zc[(2 * g + 1) * NZW + k] = d;
            }
            } else {
              // element matrices of the layer: slot s holds Mz r and Kz r
              // (Kz annihilates constants: columns 1.. on the differences)
#pragma unroll
              for (int s2 = 0; s2 < P; ++s2) {
                T v = mz[s2][0] * r[0], d = kz[s2][0] * dr[1];
#pragma unroll
                for (int a = 1; a < P; ++a) v = fma(mz[s2][a], r[a], v);
#pragma unroll
                for (int a = 2; a < P; ++a) d = fma(kz[s2][a - 1], dr[a], d);
                zc[(2 * s2) * NZW + k] = v;
                zc[(2 * s2 + 1) * NZW + k] = d;
              }
            }
          }
        }
      }
      wave_sync();
#pragma unroll 1
      for (int gz = 0; gz < Q; ++gz) {
        T* sbb = sb + buf * Gm::NCH * SBC;
        // wave-speed field of this lane's x-element at the Gauss rows of its
        // x-stage (lane mapping of the VALU or of the MFMA form), loaded
        // here, before the y-stage, and used raw (no select or conversion
        // before the x-stage, which would wait for the loads at once); rows
        // outside the mesh load the first entry and are zeroed at use
        double cqr[CF ? NRW : 1][Q];
        bool cqok[CF ? NRW : 1];
        if constexpr (CF) {
          const int xr = MF ? mj : grp, xe = MF ? exm : ex;
          const bool xv = MF ? exvm : exv;
#pragma unroll
          for (int i = 0; i < NRW; ++i) {
            const int r = wv * WE * Q + 4 * i + xr;
            const int ey = Y0 - p + r / Q, gy = r - (r / Q) * Q;
            cqok[i] = xv && ey >= 0 && ey < Ey;
            const long long o = (((long long)ez * Q + gz) * ((long long)Ey * Q) + (long long)ey * Q + gy) *
                                    ((long long)Ex * Q) + (long long)xe * Q;
            const gmem<double>* cp = C + (cqok[i] ? o : 0ll);
#pragma unroll
            for (int gx = 0; gx < Q; ++gx) cqr[i][gx] = cp[gx];
          }
        }
        // (Y) y-contraction of this wave's y-elements: value, y-derivative,
        // z-derivative per y Gauss row
        {
          const T* z0 = zc + (2 * gz) * NZW + yzc;
          const T* z1 = z0 + NZW;
          T av[P], bv[P];
#pragma unroll
          for (int b = 0; b < P; ++b) {
            av[b] = z0[b * TXH];
            bv[b] = z1[b * TXH];
          }
          T da[P];
#pragma unroll
          for (int b = 1; b < P; ++b) da[b] = av[b] - av[0];
          if constexpr (CF) {
          const T* tN = tyl + yty;
          const T* tD = tN + Q * P;
#pragma unroll
          for (int gy = 0; gy < Q; ++gy) {
            T c = tN[gy * P] * av[0], dzv = tN[gy * P] * bv[0], dyv = tD[gy * P + 1] * da[1];
#pragma unroll
            for (int b = 1; b < P; ++b) {
              c = fma(tN[gy * P + b], av[b], c);
              dzv = fma(tN[gy * P + b], bv[b], dzv);
            }
#pragma unroll
            for (int b = 2; b < P; ++b) dyv = fma(tD[gy * P + b], da[b], dyv);
            T* o = sbb + rowstep(ysb, ypar, gy);
            o[0] = c;
            o[SBC] = dyv;
            o[2 * SBC] = dzv;
          }
          } else {
            // element matrices: row a (local y-slot) holds My av and, with z
            // collapsed too (every channel ends in the same sum), the y- and
            // z-derivative channels that the x-mass matrix takes, added:
            // Ky da + My bv
            const T* tM = tyl + yty;
            const T* tK = tM + P * P;
#pragma unroll
            for (int a = 0; a < P; ++a) {
              T c = tM[a * P] * av[0], d = tM[a * P] * bv[0];
#pragma unroll
              for (int b = 1; b < P; ++b) {
                c = fma(tM[a * P + b], av[b], c);
                d = fma(tM[a * P + b], bv[b], d);
              }
#pragma unroll
              for (int b = 1; b < P; ++b) d = fma(tK[a * (P - 1) + b - 1], da[b], d);
              T* o = sbb + rowstep(ysb, ypar, a);
              o[0] = c;
              o[SBC] = d;
            }
          }
        }
        if (xok) {
          const T* z0 = zc + (2 * gz) * NZW + xzc;
          const T* z1 = z0 + NZW;
          T av[P], bv[P];
#pragma unroll
          for (int b = 0; b < P; ++b) {
            av[b] = z0[b * TXH];
            bv[b] = z1[b * TXH];
          }
          T c, dzv, dyv;
          if constexpr (CF) {
            const T* tN = tyl + xty;
            const T* tD = tN + Q * P;
            c = tN[0] * av[0];
            dzv = tN[0] * bv[0];
            dyv = tD[1] * (av[1] - av[0]);
#pragma unroll
            for (int b = 1; b < P; ++b) {
              c = fma(tN[b], av[b], c);
              dzv = fma(tN[b], bv[b], dzv);
            }
#pragma unroll
            for (int b = 2; b < P; ++b) dyv = fma(tD[b], av[b] - av[0], dyv);
          } else {
            // local y-slot xa of the element (as in the full pass)
            const T* tM = tyl + (xty - xa * P);
            const T* tK = tM + P * P;
            T da[P];
#pragma unroll
            for (int b = 1; b < P; ++b) da[b] = av[b] - av[0];
            c = tM[xa * P] * av[0];
            dzv = tM[xa * P] * bv[0];
#pragma unroll
            for (int b = 1; b < P; ++b) {
              c = fma(tM[xa * P + b], av[b], c);
              dzv = fma(tM[xa * P + b], bv[b], dzv);
            }
#pragma unroll
            for (int b = 1; b < P; ++b) dzv = fma(tK[xa * (P - 1) + b - 1], da[b], dzv);
            dyv = T(0);
          }
          T* o = sbb + xsb;
          o[0] = c;
          if constexpr (CF) {
            o[SBC] = dyv;
            o[2 * SBC] = dzv;
          } else {
            o[SBC] = dyv + dzv;
          }
        }
        wave_sync();
        // (X) x-forward, x-weights, x-backward on this wave's rows; lanes
        // are x-elements
#pragma unroll
        for (int i = 0; i < NRW; ++i) {
          if constexpr (MF) {
            // rows 4i + mj of the three channels, column of x-element mb
            T* rm = sbb + xrowm0 + 2 * i * RP;
            float cq[4];
#pragma unroll
            for (int gx = 0; gx < 4; ++gx) cq[gx] = (gx < Q && cqok[i]) ? (float)cqr[i][gx < Q ? gx : 0] : 0.f;
            // forward: x-derivative of channel 0 (on differences: the
            // derivative tables annihilate constants), values of channels
            // 1 and 2, at the element's Gauss points (register = point)
            f4 gX = {0.f, 0.f, 0.f, 0.f}, gY = gX, gZ = gX;
            const float base = rm[0];
#pragma unroll
            for (int k = 1; k < P; ++k) gX = mfma4(mfD[k], rm[k] - base, gX);
#pragma unroll
            for (int k = 0; k < P; ++k) {
              gY = mfma4(mfN[k], rm[SBC + k], gY);
              gZ = mfma4(mfN[k], rm[2 * SBC + k], gZ);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              gX[g] *= cq[g];
              gY[g] *= cq[g];
              gZ[g] *= cq[g];
            }
            // backward: point values in registers are the B operand of the
            // K-steps (register k = Gauss point k); register = slot
            f4 oX = {0.f, 0.f, 0.f, 0.f}, oY = oX, oZ = oX;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
              oX = mfma4(mbD[k], gX[k], oX);
              oY = mfma4(mbN[k], gY[k], oY);
              oZ = mfma4(mbN[k], gZ[k], oZ);
            }
            // coefficient of slot mb - p collects slot a of element mb - a
            // (the block 4a lanes down)
            float tX = oX[P - 1], tY = oY[P - 1], tZ = oZ[P - 1];
#pragma unroll
            for (int a = P - 2; a >= 0; --a) {
              tX = oX[a] + lane_sub4(tX, lane);
              tY = oY[a] + lane_sub4(tY, lane);
              tZ = oZ[a] + lane_sub4(tZ, lane);
            }
            if (mb >= p) {
              rm[-p] = tX;
              rm[SBC - p] = tY;
              rm[2 * SBC - p] = tZ;
            }
            continue;
          }
          T* row = sbb + xrow0 + 2 * i * RP;
          // wave-speed field: the lane's q points of this Gauss row (0 outside the mesh)
          T cq[Q];
          if constexpr (CF) {
#pragma unroll
            for (int gx = 0; gx < Q; ++gx) cq[gx] = cqok[i] ? (T)cqr[i][gx] : T(0);
          }
          T c0[P], c1[P], c2[P];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            c0[a] = row[j + a];
            c1[a] = row[SBC + j + a];
            if constexpr (CF) c2[a] = row[2 * SBC + j + a];
          }
          T d0[P];
#pragma unroll
          for (int a = 1; a < P; ++a) d0[a] = c0[a] - c0[0];
          T o0[P], o1[P], o2[P];
          if constexpr (!CF) {
            // element matrices (see Kx, Mx): o0 = Mx c1 + Kx d0 (c1: the y-
            // and z-derivative channels summed by the y-stage), one chain
#pragma unroll
            for (int a = 0; a < P; ++a) {
              T s1 = Mx[a][0] * c1[0];
#pragma unroll
              for (int b = 1; b < P; ++b) s1 = fma(Mx[a][b], c1[b], s1);
#pragma unroll
              for (int b = 1; b < P; ++b) s1 = fma(Kx[a][b - 1], d0[b], s1);
              o0[a] = s1;
            }
          } else {
#pragma unroll
          for (int gx = 0; gx < Q; ++gx) {
            T gX = xD[gx][1] * d0[1], gY = xN[gx][0] * c1[0], gZ = xN[gx][0] * c2[0];
#pragma unroll
            for (int a = 2; a < P; ++a) gX = fma(xD[gx][a], d0[a], gX);
#pragma unroll
            for (int a = 1; a < P; ++a) {
              gY = fma(xN[gx][a], c1[a], gY);
              gZ = fma(xN[gx][a], c2[a], gZ);
            }
            if constexpr (!kFoldX) {
              gX *= xW[gx];
              gY *= xW[gx];
              gZ *= xW[gx];
            }
            if constexpr (CF) {
              gX *= cq[gx];
              gY *= cq[gx];
              gZ *= cq[gx];
            }
            if (gx == 0) {
#pragma unroll
              for (int a = 0; a < P; ++a) {
                o0[a] = bxD(0, a) * gX;
                o1[a] = bxN(0, a) * gY;
                o2[a] = bxN(0, a) * gZ;
              }
            } else {
#pragma unroll
              for (int a = 1; a < P; ++a) o0[a] = fma(bxD(gx, a), gX, o0[a]);
#pragma unroll
              for (int a = 0; a < P; ++a) {
                o1[a] = fma(bxN(gx, a), gY, o1[a]);
                o2[a] = fma(bxN(gx, a), gZ, o2[a]);
              }
            }
          }
          }
          // coefficient c = ex collects slot a of element ex - a (lane j - a)
          if constexpr (CF) {
            // backward derivative tables sum to zero: slot 0 from the others
            {
              T s = o0[1];
#pragma unroll
              for (int a = 2; a < P; ++a) s += o0[a];
              o0[0] = -s;
            }
            const T r0v = horner_shift<P, T>(o0);
            const T r1v = horner_shift<P, T>(o1);
            const T r2v = horner_shift<P, T>(o2);
            if (j >= p) {
              row[j - p] = r0v;
              row[SBC + j - p] = r1v;
              row[2 * SBC + j - p] = r2v;
            }
          } else {
            // all channels end in one sum: assembled once, one value per row.
            // Lanes j < p own no coefficient: they write to the spare columns
            // TX + p + j of the row, which nothing reads afterwards, so that
            // the rows of a slot form one block the scheduler can interleave
            const T r01 = horner_shift<P, T>(o0);
            row[j >= p ? j - p : TX + p + j] = r01;
          }
        }
        // refill the ring slot of layer ez (its z stage is done in every
        // wave: they all passed the barrier of an earlier Gauss point)
        if (gz == Q - 1 && ez < ez1) commit_layer(ez + P);
        __syncthreads();
        // (B) y-backward and z-backward into the owned column's accumulators
        if (own) {
          // backward z tables at this Gauss point (weighted tables W*N, W*D)
          const cmem<double>* tw = tzg + (2ll * Ez * Q * P + (long long)Ez * Q) + ((long long)ez * Q + gz) * P;
          double nzw[P], dzw[P];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            nzw[a] = tw[a];
            dzw[a] = tw[(long long)Ez * Q * P + a];
          }
          T Ap = T(0), Bp = T(0);
          if constexpr (CF) {
#pragma unroll
          for (int b = 0; b < P; ++b) {
#pragma unroll
            for (int gy = 0; gy < Q; ++gy) {
              const T* e = sbb + rowstep(brow0, bpar, (p - b) * Q + gy);
              Ap = fma(bN[b][gy], e[0], Ap);
              Ap = fma(bD[b][gy], e[SBC], Ap);
              Bp = fma(bN[b][gy], e[2 * SBC], Bp);
            }
          }
          } else {
            // the column collects local slot b of y-element cyo + p - b
            // (all channels already summed)
#pragma unroll
            for (int b = 0; b < P; ++b) Ap += sbb[rowstep(brow0, bpar, (p - b) * Q + b)];
          }
          if constexpr (CF) {
#pragma unroll
            for (int a = 0; a < P; ++a) acc[a] = fma(nzw[a], (double)Ap, fma(dzw[a], (double)Bp, acc[a]));
          } else {
            // local z-slot gz of the layer's element: coefficient ez + gz
            const double v = (double)Ap + (double)Bp;
#pragma unroll
            for (int a = 0; a < P; ++a) acc[a] += a == gz ? v : 0.0;
          }
        }
        buf ^= 1;
      }
      store_out(ez, acc[0]);
#pragma unroll
      for (int a = 0; a < P - 1; ++a) acc[a] = acc[a + 1];
      acc[P - 1] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < P - 1; ++a) store_out(ez1 + 1 + a, acc[a]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// variants (tile height, workgroup size) per degree and arithmetic; variant
// 0 is the same for both arithmetics.  The autotuner in api.cpp times them
// on the real mesh.
struct RhsVariant {
  int TY, NT;
};
static const RhsVariant kVarP2F[] = {{14, 256}, {26, 448}, {10, 192}};
static const RhsVariant kVarP2D[] = {{14, 256}, {30, 512}, {22, 384}};
static const RhsVariant kVarP3F[] = {{13, 256}, {29, 512}, {21, 384}};
static const RhsVariant kVarP3D[] = {{13, 256}, {21, 384}, {9, 192}};

// variant 3: the Kronecker (assembled band) form of k_rhs_band.hip, for
// jobs without a wave-speed field; variant 4: the MFMA x-stage (FP32 with a
// field), at one tile shape per degree
static constexpr RhsVariant kVarMX[] = {{10, 192}, {13, 256}};
bool rhs_variant_exists(int p, int mixed, int var, int coef) {
  const bool quad = p == 2 || p == 3;
  if (var == 3) return !coef;
  if (var == 4) return quad && coef && mixed;
  return quad && var >= 0 && var <= 2;
}
int rhs_tile_x(int p, int var) { return var == 3 ? rhs_band_tile_x() : 16 - p; }
int rhs_tile_y(int p, int mixed, int var) {
  if (var == 3) return rhs_band_tile_y();
  if (var == 4) return kVarMX[p <= 2 ? 0 : 1].TY;
  if (var < 0 || var > 2) var = 0;
  if (p <= 2) return mixed ? kVarP2F[var].TY : kVarP2D[var].TY;
  return mixed ? kVarP3F[var].TY : kVarP3D[var].TY;
}

// op 0: launch; op 1: *out = resident workgroups per CU (persistent grids)
template <typename T, int P, int TY, int NT, bool CF, bool MX = false>
static hipError_t launch_one(const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  using Gm = RhsGeom<T, P, P, TY, NT, CF>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)rhs_pwave_kernel<T, P, P, TY, NT, CF, MX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm::lds_bytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (op == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, (const void*)rhs_pwave_kernel<T, P, P, TY, NT, CF, MX>,
                                                        NT, Gm::lds_bytes);
  hipLaunchKernelGGL((rhs_pwave_kernel<T, P, P, TY, NT, CF, MX>), dim3(grid), dim3(NT), Gm::lds_bytes, s, d_hdr);
  return hipGetLastError();
}

// variant 4 (mixed mode with a field only)
static hipError_t launch_mx(int p, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  static_assert(kVarMX[0].TY == 10 && kVarMX[0].NT == 192 && kVarMX[1].TY == 13 && kVarMX[1].NT == 256,
                "variant 4 instantiations");
  if (p == 2) return launch_one<float, 3, 10, 192, true, true>(d_hdr, grid, s, op, out);
  return launch_one<float, 4, 13, 256, true, true>(d_hdr, grid, s, op, out);
}

template <bool CF>
static hipError_t launch_f(int p, int var, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  if (p == 2) {
    switch (var) {
      case 0: return launch_one<float, 3, 14, 256, CF>(d_hdr, grid, s, op, out);
      case 1: return launch_one<float, 3, 26, 448, CF>(d_hdr, grid, s, op, out);
      default: return launch_one<float, 3, 10, 192, CF>(d_hdr, grid, s, op, out);
    }
  }
  switch (var) {
    case 0: return launch_one<float, 4, 13, 256, CF>(d_hdr, grid, s, op, out);
    case 1: return launch_one<float, 4, 29, 512, CF>(d_hdr, grid, s, op, out);
    default: return launch_one<float, 4, 21, 384, CF>(d_hdr, grid, s, op, out);
  }
}

template <bool CF>
static hipError_t launch_d(int p, int var, const LaunchHdr* d_hdr, int grid, hipStream_t s, int op, int* out) {
  if (p == 2) {
    switch (var) {
      case 0: return launch_one<double, 3, 14, 256, CF>(d_hdr, grid, s, op, out);
      case 1: return launch_one<double, 3, 30, 512, CF>(d_hdr, grid, s, op, out);
      default: return launch_one<double, 3, 22, 384, CF>(d_hdr, grid, s, op, out);
    }
  }
  switch (var) {
    case 0: return launch_one<double, 4, 13, 256, CF>(d_hdr, grid, s, op, out);
    case 1: return launch_one<double, 4, 21, 384, CF>(d_hdr, grid, s, op, out);
    default: return launch_one<double, 4, 9, 192, CF>(d_hdr, grid, s, op, out);
  }
}

static hipError_t dispatch(int p, int mixed, int var, int coef, const LaunchHdr* d_hdr, int grid, hipStream_t s,
                           int op, int* out) {
  if (mixed) return coef ? launch_f<true>(p, var, d_hdr, grid, s, op, out) : launch_f<false>(p, var, d_hdr, grid, s, op, out);
  return coef ? launch_d<true>(p, var, d_hdr, grid, s, op, out) : launch_d<false>(p, var, d_hdr, grid, s, op, out);
}

hipError_t launch_rhs_pwave(int p, int mixed, int var, int coef, const LaunchHdr* d_hdr, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (var == 3) return coef ? hipErrorInvalidValue : launch_rhs_band(p, mixed, d_hdr, grid, s);
  if (p != 2 && p != 3) return hipErrorInvalidValue;   // the quadrature is instantiated for p = 2, 3
  if (var == 4) return (coef && mixed) ? launch_mx(p, d_hdr, grid, s, 0, nullptr) : hipErrorInvalidValue;
  if (var < 0 || var > 2) var = 0;
  return dispatch(p, mixed, var, coef, d_hdr, grid, s, 0, nullptr);
}

int rhs_blocks_per_cu(int p, int mixed, int var, int coef) {
  if (var == 3 && !coef) return rhs_band_blocks_per_cu(p, mixed);
  if (p != 2 && p != 3) return 1;
  int n = 1;
  if (var == 4 && coef && mixed) {
    (void)launch_mx(p, nullptr, 0, nullptr, 1, &n);
    return n < 1 ? 1 : n;
  }
  if (var < 0 || var > 2) var = 0;
  (void)dispatch(p, mixed, var, coef, nullptr, 0, nullptr, 1, &n);
  return n < 1 ? 1 : n;
}

}  // namespace ads
