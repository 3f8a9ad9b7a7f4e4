// C-ABI implementation: simulation object, workspace planner, per-step
// launch lists.  See include/ads.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ads.h"
#include "common.hpp"
#include "host_math.hpp"
#include "launch.hpp"

using namespace ads;

// Staging memory of ads_project_static: a file-scope device array, so that
// that entry point allocates nothing.  Each device holds its own copy; host
// code uses the address hipGetSymbolAddress returns for the current device
// (static_scratch_address below), never the array's name, which on the host
// is not a device address.  Every call on a device shares its copy.
static __device__ __align__(256) char scratch[(size_t)ADS_PROJECT_STATIC_BYTES];

namespace {

thread_local std::string g_err = "no error";
thread_local int g_force_var = -1;   // right-hand-side tile variant imposed by a pool

ads_status fail(ads_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHECK(expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ADS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

// Kernel attributes (dynamic LDS above the default) are set once per
// process; the static's initialization is thread-safe.
hipError_t set_attributes_once() {
  static const hipError_t e = [] {
    const hipError_t a = sweep_set_attributes();
    return a != hipSuccess ? a : kron_set_attributes();
  }();
  return e;
}

constexpr size_t kStaticScratchBytes = (size_t)ADS_PROJECT_STATIC_BYTES;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
ads_status static_scratch_address(void** out) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ADS_EDEVICE, "device index beyond the static-buffer table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ADS_EDEVICE, "hipGetSymbolAddress returned NULL for the static buffer");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return ADS_OK;
}

constexpr int kAmpCap = 4096;
constexpr size_t kAlign = 256;
constexpr size_t kJobArena = 96 * 1024;

// Bump allocator over the caller's workspace; with base == nullptr it only
// counts bytes (the same walk sizes and carves the workspace).
struct Carver {
  char* base;
  size_t used = 0;
  void* take(size_t bytes) {
    used = (used + kAlign - 1) / kAlign * kAlign;
    void* p = base ? base + used : nullptr;
    used += bytes;
    return p;
  }
  double* dbl(size_t n) { return (double*)take(n * sizeof(double)); }
};

// One kernel launch of a step (or of setup), with its device job table
// (LaunchHdr + jobs) and a host copy of the jobs (for batching).
struct Launch {
  enum Kind { RHS_P, RHS_E, SWEEP, KRON, PLANE } kind;
  const LaunchHdr* d_hdr;
  int njobs, total_tiles, max_m, p;
  int dir = -1;   // sweeps: direction
  int var = 0;    // right-hand side: tile variant
  int mixed = 0;  // right-hand side: FP32 contractions
  std::vector<char> host_jobs;
  int w = 4;      // sweeps: lines per wave tile
  int coef = 0;   // P-wave right-hand side: jobs carry a wave-speed field
  size_t lds = 0; // in-plane sweeps: dynamic LDS bytes
  bool coupled = false;  // in-plane sweeps: jobs carry coupling terms
};

struct DevFactor {
  double *L, *U, *rd;
  int m;
};

// Host-side mirror of the job arena: jobs are appended here, then uploaded.
struct JobArena {
  char* d_base = nullptr;
  std::vector<char> host;
  size_t cap = 0;
  // Appends a header + job table (tile0 set to prefix sums); returns the
  // device address of the header, or nullptr when the arena is full.
  template <class T>
  const LaunchHdr* add(std::vector<T> jobs, std::string& err, int* total = nullptr) {
    size_t off = (host.size() + kAlign - 1) / kAlign * kAlign;
    size_t bytes = sizeof(LaunchHdr) + jobs.size() * sizeof(T);
    if (off + bytes > cap) {
      err = "job arena full";
      return nullptr;
    }
    int t = 0;
    for (T& j : jobs) {
      j.tile0 = t;
      t += j.ntiles;
    }
    LaunchHdr h{};
    h.njobs = (int)jobs.size();
    h.total_tiles = t;
    host.resize(off + bytes);
    std::memcpy(host.data() + off, &h, sizeof(h));
    std::memcpy(host.data() + off + sizeof(LaunchHdr), jobs.data(), jobs.size() * sizeof(T));
    if (total) *total = t;
    return (const LaunchHdr*)(d_base + off);
  }
};

template <class T>
std::vector<char> as_bytes(const T& j) {
  std::vector<char> b(sizeof(T));
  std::memcpy(b.data(), &j, sizeof(T));
  return b;
}

}  // namespace

struct ads_sim {
  ads_params prm;
  hipStream_t stream = nullptr;
  int E[3], n[3], nf[3], off[3];
  int p, q, P, ncomp;
  long long nfree;
  bool elastic;
  Tables1D tab[3];
  Band Mf[3], Kf[3], Gf[3];   // free-block bands
  // device
  double* d_tab[3];
  double* d_bandM[3];
  double* d_bandG[3];
  double* d_bandGT[3];
  double* d_bandA[3];   // split bands (energy diagnostic): P-wave M_d + tau^2/4 K_d,
  double* d_bandA2[3];  // elasticity M_d + tau^2 c K_d/(4 rho), c = mu (A) and 2 mu + lambda (A2)
  double* red;          // dot-product partial sums + 3 results
  DevFactor fS[3], fS2[3], fM[3];  // P-wave: fS = M + eta K; elastic: fS = mu, fS2 = 2mu+lam
  double *u, *v, *a, *R, *X, *T, *Y, *Z, *load, *amp;
  // P-wave: the time step advances (w, b, a), w = u + tau v + eta a the
  // predictor of the next step and b = v + tau/2 a the half-step velocity
  // (printed coefficient set: (w, v, a), w = u + tau v), so that its
  // right-hand side reads one field and its update two; u and v are formed
  // from them when read (w_stale: w and b must be formed from u, v, a,
  // after the state was set; u_stale: u and v must be formed from w, b, a,
  // after time steps)
  double* w = nullptr;
  double* b = nullptr;
  bool w_stale = true, u_stale = false;
  unsigned long long* counter;
  unsigned long long* flag;
  JobArena arena;
  std::vector<Launch> step_l, start_l, projM_l, energy_l;
  bool factored = false, need_start = true, have_load = false;
  int namp = 0;
  int tz = 0;           // right-hand side: owned z-layers per tile (0: chosen from the occupancy)
  int sweep_w[3] = {0, 0, 0};   // sweeps per direction: lines per wave tile (0: default)
  // elasticity couplings: true = applied in the input stage of the in-plane
  // sweep that consumes them where the plane fits, false = separate launches
  // (the default; ads_tune times both)
  bool couple_fused = false;
  int ncu = 0;          // compute units of the device (tiling of the right-hand side)
  // P-wave right-hand side: 3 = the Kronecker form (jobs with a wave-speed
  // field take the quadrature kernel's variant 0); ads_tune may choose another
  int rhs_var = 3;
  bool mixed = false;   // FP32 contractions in the right-hand side
  bool bf16 = false;    // ... on BF16 inputs, plus a correction pass on the remainder
  bool literal = false; // P-wave: the printed coefficient set (diagnostic)
  bool pooled = false;  // owned by a pool: its launch shapes are the pool's
  bool* pool_dirty = nullptr;   // the owning pool's flag: its tables copy this sim's jobs
  const double* coef = nullptr;   // P-wave: caller's c^2 at the Gauss points, or null
  double c2ref = 1.0;             // P-wave: c^2 of the split left-hand side
  // kernel timing (measurement support)
  bool prof = false;
  std::vector<hipEvent_t> ev;     // (launches + 1) events per recorded step
  int prof_steps = 0;
  ~ads_sim() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

namespace {

// Free coefficients of direction d: all n = nelem + p of them with natural
// conditions, the n - 2 interior ones with zero Dirichlet conditions.
// nelem[2] = 0: a two-dimensional problem (x, y); the z-direction is one
// constant function (one free coefficient).  Elasticity there is plane
// strain in (u_x, u_y), its blocks with z-derivatives vanishing, beside the
// decoupled antiplane component u_z.
bool flat_z(const ads_params& P) { return P.nelem[2] == 0; }
int free_count(const ads_params& P, int d) {
  if (d == 2 && flat_z(P)) return 1;
  return P.nelem[d] + P.p - (P.bc == ADS_BC_NATURAL ? 0 : 2);
}
Tables1D tables_of(const ads_params& P, int d) {
  const int q = P.nquad > 0 ? P.nquad : P.p + 1;
  return (d == 2 && flat_z(P)) ? make_tables_flat(P.p, q) : make_tables(P.nelem[d], P.p, q);
}

bool valid_params(const ads_params* prm, std::string& why) {
  if (!prm) {
    why = "params is NULL";
    return false;
  }
  if (prm->problem != ADS_PWAVE && prm->problem != ADS_ELASTIC) {
    why = "problem must be ADS_PWAVE or ADS_ELASTIC";
    return false;
  }
  for (int d = 0; d < 3; ++d) {
    if (d == 2 && prm->nelem[2] == 0) continue;   // two-dimensional
    if (prm->nelem[d] < 1 || prm->nelem[d] > 4096) {
      why = "nelem must be in [1, 4096] (nelem[2] = 0: two-dimensional)";
      return false;
    }
  }
  if (prm->p < 1 || prm->p > 5) {
    why = "spline degree p must be in [1, 5]";
    return false;
  }
  if (prm->nquad != 0 && (prm->nquad < prm->p + 1 || prm->nquad > prm->p + 3)) {
    why = "nquad must be 0 (p+1) or in [p+1, p+3]";
    return false;
  }
  if (prm->bc != ADS_BC_DIRICHLET0 && prm->bc != ADS_BC_NATURAL) {
    why = "bc must be ADS_BC_DIRICHLET0 or ADS_BC_NATURAL";
    return false;
  }
  if (!(prm->tau > 0.0) || !std::isfinite(prm->tau)) {
    why = "tau must be positive and finite";
    return false;
  }
  if (prm->precision != ADS_FP64 && prm->precision != ADS_MIXED_FP32 && prm->precision != ADS_MIXED_BF16) {
    why = "precision must be ADS_FP64, ADS_MIXED_FP32 or ADS_MIXED_BF16";
    return false;
  }
  if (prm->precision == ADS_MIXED_BF16 && prm->problem != ADS_PWAVE) {
    why = "the BF16-input mode is implemented for the P-wave only (elasticity: ADS_FP64 or ADS_MIXED_FP32)";
    return false;
  }
  if (prm->problem == ADS_ELASTIC) {
    if (!(prm->rho > 0.0) || !(prm->mu > 0.0) || !(prm->lambda + 2.0 * prm->mu / 3.0 > 0.0)) {
      why = "elasticity needs rho > 0, mu > 0, lambda + 2 mu / 3 > 0";
      return false;
    }
  }
  for (int d = 0; d < 3; ++d)
    if (free_count(*prm, d) > 512) {
      why = "at most 512 free coefficients per direction";
      return false;
    }
  return true;
}

void geometry(ads_sim* s) {
  const ads_params& P = s->prm;
  s->p = P.p;
  s->q = P.nquad > 0 ? P.nquad : P.p + 1;
  s->P = P.p + 1;
  s->elastic = P.problem == ADS_ELASTIC;
  s->ncomp = s->elastic ? 3 : 1;
  for (int d = 0; d < 3; ++d) {
    const bool flat = d == 2 && flat_z(P);
    s->E[d] = flat ? 1 : P.nelem[d];
    s->n[d] = flat ? 1 : P.nelem[d] + P.p;
    s->nf[d] = free_count(P, d);
    s->off[d] = (flat || P.bc == ADS_BC_NATURAL) ? 0 : 1;
  }
  s->nfree = (long long)s->nf[0] * s->nf[1] * s->nf[2];
  s->mixed = P.precision == ADS_MIXED_FP32 || P.precision == ADS_MIXED_BF16;
  s->bf16 = P.precision == ADS_MIXED_BF16;
}

// Walks every device allocation of a simulation (sizing and carving).
void carve(ads_sim* s, Carver& c) {
  const long long nfr = s->nfree;
  const int P = s->P, q = s->q, p = s->p;
  // per direction: N, D [E][q][P], W [E][q], W*N, W*D [E][q][P], then the
  // element mass and stiffness matrices sum_g W N N^T, sum_g W D D^T [E][P][P],
  // then the assembled matrices M, K of the free coefficients [nf][2p+1]
  // (elasticity: then G and G^T of the free coefficients [nf][2p+1])
  for (int d = 0; d < 3; ++d)
    s->d_tab[d] = c.dbl((size_t)4 * s->E[d] * q * P + (size_t)s->E[d] * q + (size_t)2 * s->E[d] * P * P +
                        (size_t)(s->elastic ? 4 : 2) * s->nf[d] * (2 * p + 1));
  auto fac = [&](DevFactor& f, int d) {
    f.m = s->nf[d];
    f.L = c.dbl((size_t)f.m * p);
    f.U = c.dbl((size_t)f.m * p);
    f.rd = c.dbl(f.m);
  };
  for (int d = 0; d < 3; ++d) {
    fac(s->fS[d], d);
    fac(s->fM[d], d);
    if (s->elastic) fac(s->fS2[d], d);
    else s->fS2[d] = DevFactor{nullptr, nullptr, nullptr, 0};
  }
  const int nc = s->ncomp;
  s->u = c.dbl(nfr * nc);
  s->v = c.dbl(nfr * nc);
  s->R = c.dbl(nfr * nc);
  s->X = c.dbl(nfr);
  s->load = c.dbl(nfr * nc);
  s->amp = c.dbl(kAmpCap);
  if (s->elastic) {
    s->a = nullptr;
    s->T = c.dbl(nfr);
    s->Y = c.dbl(nfr * 3);
    s->Z = c.dbl(nfr * 3);
    for (int d = 0; d < 3; ++d) {
      size_t bw = (size_t)s->nf[d] * (2 * p + 1);
      s->d_bandM[d] = c.dbl(bw);
      s->d_bandG[d] = c.dbl(bw);
      s->d_bandGT[d] = c.dbl(bw);
      s->d_bandA[d] = c.dbl(bw);
      s->d_bandA2[d] = c.dbl(bw);
    }
  } else {
    s->a = c.dbl(nfr);
    s->w = c.dbl(nfr);
    s->b = c.dbl(nfr);
    s->T = s->Y = s->Z = nullptr;
    for (int d = 0; d < 3; ++d) s->d_bandA[d] = c.dbl((size_t)s->nf[d] * (2 * p + 1));
  }
  s->red = c.dbl(dot_scratch_doubles() + 4);
  s->counter = (unsigned long long*)c.take(64);
  s->flag = (unsigned long long*)c.take(64);
  s->arena.d_base = (char*)c.take(kJobArena);
  s->arena.cap = kJobArena;
}

// --- job builders ------------------------------------------------------------

int max_m(const ads_sim* s) { return std::max(s->nf[0], std::max(s->nf[1], s->nf[2])); }

// Tile width of a sweep launch of direction dir: the one set by
// ads_set_launch_shape where it fits, else the default.
int sim_sweep_width(const ads_sim* s, int dir, long long lines) {
  const int w = s->sweep_w[dir];
  if (w > 0 && sweep_width_fits(w, max_m(s), s->p)) return w;
  return sweep_width_for(lines, max_m(s), s->ncu, s->p);
}

SweepJob sweep_job(const ads_sim* s, int dir, const DevFactor& f, const double* in, double* out, double scale) {
  SweepJob J{};
  J.in = in;
  J.out = out;
  J.f = Factor1D{f.L, f.U, f.rd, f.m};
  J.dir = dir;
  J.p = s->p;
  J.nx = s->nf[0];
  J.ny = s->nf[1];
  J.nz = s->nf[2];
  J.nlines = (int)(s->nfree / s->nf[dir]);
  J.ntiles = sweep_groups(J.nlines, sim_sweep_width(s, dir, J.nlines));
  J.tile0 = 0;
  J.epi = EPI_STORE;
  J.scale = scale;
  return J;
}

// Three sweeps x (in -> X), y (X -> tmp), z (tmp -> out/epilogue) with one
// factor per direction; when a z-plane fits in LDS the x- and y-sweeps are
// one in-plane launch (in -> tmp).  With coupling terms (the caller has
// checked plane_couple_fits) the in-plane launch adds them to `in` (which
// may then be null).
bool add_ads_solve(ads_sim* s, std::vector<Launch>& L, const DevFactor f[3], const double* in, double* tmp,
                   double* out, double scale, SweepJob zlast, std::string& err, const KronTerm* terms = nullptr,
                   int nterm = 0) {
  const bool fused = nterm > 0 || plane_fits(s->nf[0], s->nf[1], s->p);
  if (nterm > kPlaneMaxTerms || (nterm > 0 && !plane_couple_fits(s->nf[0], s->nf[1], s->p))) {
    err = "coupling terms do not fit the in-plane sweep";
    return false;
  }
  if (fused) {
    PlaneJob jp{};
    jp.nterm = nterm;
    for (int t = 0; t < nterm; ++t) jp.term[t] = terms[t];
    jp.in = in;
    jp.out = tmp;
    jp.fx = Factor1D{f[0].L, f[0].U, f[0].rd, f[0].m};
    jp.fy = Factor1D{f[1].L, f[1].U, f[1].rd, f[1].m};
    jp.p = s->p;
    jp.nx = s->nf[0];
    jp.ny = s->nf[1];
    jp.nz = s->nf[2];
    jp.scale = scale;
    jp.tile0 = 0;
    jp.ntiles = s->nf[2];
    const LaunchHdr* d = s->arena.add(std::vector<PlaneJob>{jp}, err);
    if (!d) return false;
    L.push_back(Launch{Launch::PLANE, d, 1, jp.ntiles, max_m(s), s->p, -1, 0, 0, as_bytes(jp)});
    L.back().lds = plane_lds_bytes(jp.nx, jp.ny, jp.p, nterm > 0);
    L.back().coupled = nterm > 0;
  }
  SweepJob jx = sweep_job(s, 0, f[0], in, s->X, scale);
  SweepJob jy = sweep_job(s, 1, f[1], s->X, tmp, 1.0);
  SweepJob jz = zlast;
  const SweepJob base = sweep_job(s, 2, f[2], tmp, out, 1.0);
  jz.in = base.in;
  jz.out = out;
  jz.f = base.f;
  jz.dir = 2;
  jz.p = base.p;
  jz.nx = base.nx;
  jz.ny = base.ny;
  jz.nz = base.nz;
  jz.nlines = base.nlines;
  jz.ntiles = base.ntiles;
  jz.tile0 = 0;
  jz.scale = 1.0;
  std::vector<SweepJob*> js{&jx, &jy, &jz};
  if (fused) js = {&jz};
  for (SweepJob* j : js) {
    const LaunchHdr* d = s->arena.add(std::vector<SweepJob>{*j}, err);
    if (!d) return false;
    L.push_back(Launch{Launch::SWEEP, d, 1, j->ntiles, max_m(s), s->p, j->dir, 0, 0, as_bytes(*j)});
    L.back().w = sim_sweep_width(s, j->dir, j->nlines);
  }
  return true;
}

SweepJob plain_epi() {
  SweepJob z{};
  z.epi = EPI_STORE;
  return z;
}

void fill_tables(const ads_sim* s, RhsJob& J) {
  for (int d = 0; d < 3; ++d) {
    J.tab[d] = s->d_tab[d];
    J.band[d] = s->d_tab[d] + (4ll * s->E[d] * s->q * s->P + (long long)s->E[d] * s->q + 2ll * s->E[d] * s->P * s->P);
    J.E[d] = s->E[d];
    J.nf[d] = s->nf[d];
    J.off[d] = s->off[d];
  }
}

// Number of z-chunks k for right-hand-side jobs sharing one launch: a tile
// of job j marches over ceil(nfz_j / k) + p element layers, and `resident`
// workgroups take the sum_j xy_j * k tiles in rounds, so the launch lasts
// about rounds(k) * max_j (ceil(nfz_j / k) + p) layer-steps; k minimizes it
// (the fewest chunks among equals, i.e. the least z-halo work).
int best_zchunks(const std::vector<std::pair<long long, int>>& xy_nfz, int p, long long resident) {
  long long xy = 0;
  int nfz = 1;
  for (const auto& e : xy_nfz) {
    xy += e.first;
    nfz = std::max(nfz, e.second);
  }
  resident = std::max(1ll, resident);
  int best = 1;
  long long best_cost = -1;
  for (int k = 1; k <= nfz; ++k) {
    int layers = 0;
    for (const auto& e : xy_nfz) layers = std::max(layers, (e.second + k - 1) / k + p);
    const long long rounds = (xy * k + resident - 1) / resident;
    const long long cost = rounds * layers;
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = k;
    }
  }
  return best;
}

void set_zchunks(RhsJob& J, int nfz, int k) {
  const int TZ = (nfz + k - 1) / k;
  J.TZ = TZ;
  J.tiles[2] = (nfz + TZ - 1) / TZ;
  J.ntiles = J.tiles[0] * J.tiles[1] * J.tiles[2];
}

void set_kron_zchunks(KronJob& K, int k) {
  K.TZ = (K.nz + k - 1) / k;
  K.tiles[2] = (K.nz + K.TZ - 1) / K.TZ;
  K.ntiles = K.tiles[0] * K.tiles[1] * K.tiles[2];
}

// Tiling of one right-hand-side job.  resident > 0: z-chunks chosen for that
// many resident workgroups; otherwise enough tiles to cover the chip twice.
// halo: source layers a tile reads beyond its outputs (p, or 2p for the
// Kronecker form).
void rhs_tiles(const ads_sim* s, RhsJob& J, int TX, int TY, long long resident = 0, int halo = -1) {
  J.tiles[0] = (s->nf[0] + TX - 1) / TX;
  J.tiles[1] = (s->nf[1] + TY - 1) / TY;
  const int xy = J.tiles[0] * J.tiles[1];
  J.tile0 = 0;
  if (s->tz > 0) {   // fixed z-tile depth
    J.TZ = s->tz;
    J.tiles[2] = (s->nf[2] + s->tz - 1) / s->tz;
    J.ntiles = xy * J.tiles[2];
    return;
  }
  if (resident > 0) {
    set_zchunks(J, s->nf[2], best_zchunks({{xy, s->nf[2]}}, halo < 0 ? s->p : halo, resident));
    return;
  }
  const int want = std::max(1, (1024 + xy - 1) / xy);
  const int chunks = std::min(want, std::max(1, s->nf[2] / 8));
  set_zchunks(J, s->nf[2], chunks);
}

// Variant actually run: the Kronecker form (3) has no wave-speed field, so
// jobs with one take the quadrature kernel's variant 0 instead; the MFMA
// x-stage (4) exists only in mixed mode with a field, other jobs take
// variant 0 too.
int rhs_form_var(int var, bool coef, bool mixed) {
  if (coef && var == 3) return 0;
  if (var == 4 && !(coef && mixed)) return 0;
  return var;
}

// The quadrature kernels (P-wave tile variants 0-2, elasticity variant 0)
// are instantiated for p = 2 and 3 with q = p+1 Gauss points; every degree
// and Gauss rule has the Kronecker form (its band matrices are assembled on
// the host with the simulation's rule).
bool quadrature_ok(int p) { return p == 2 || p == 3; }
bool quadrature_ok(const ads_sim* s) { return quadrature_ok(s->p) && s->q == s->p + 1; }
// Variant of an FP64 right-hand side used by the start and the energy
// diagnostic: the quadrature's variant 0 where it exists, else the
// Kronecker form.
int fp64_aux_var(const ads_sim* s) { return quadrature_ok(s) ? 0 : 3; }

// P-wave right-hand side R = F(t) - K src of one field (the time step's
// predictor field, the state for the start and the energy diagnostic).
RhsJob rhs_pwave_job(const ads_sim* s, const double* src, int amp_shift, int mixed, int var) {
  RhsJob J{};
  J.u = src;
  J.cu = 1.0;
  J.R = s->R;
  J.load = s->have_load ? s->load : nullptr;
  J.amp = s->amp;
  J.namp = s->namp;
  J.amp_shift = amp_shift;
  J.counter = s->counter;
  J.rscale = 1.0;
  J.coef = s->coef;
  fill_tables(s, J);
  var = rhs_form_var(var, s->coef != nullptr, mixed != 0);
  rhs_tiles(s, J, rhs_tile_x(s->p, var), rhs_tile_y(s->p, mixed, var),
            (long long)rhs_blocks_per_cu(s->p, mixed, var, s->coef != nullptr) * s->ncu,
            var == 3 ? 2 * s->p : s->p);
  return J;
}

// Elasticity right-hand side: variant 3 is the Kronecker form (band passes,
// FP64 or mixed), variant 0 the sum-factorized quadrature (FP64).
RhsJob rhs_elastic_job(const ads_sim* s, int var, int mixed) {
  RhsJob J{};
  J.u = s->u;
  J.cu = 1.0;
  J.R = s->R;
  J.load = s->have_load ? s->load : nullptr;
  J.amp = s->amp;
  J.namp = s->namp;
  J.amp_shift = 0;
  J.counter = s->counter;
  const double tau = s->prm.tau;
  J.rscale = tau * tau;
  J.lam = s->prm.lambda;
  J.mu = s->prm.mu;
  fill_tables(s, J);
  if (var == 3)
    rhs_tiles(s, J, rhs_el_band_tile_x(), rhs_el_band_tile_y(s->p),
              (long long)rhs_el_band_blocks_per_cu(s->p, mixed) * s->ncu, 2 * s->p);
  else
    rhs_tiles(s, J, rhs_el_tile_x(s->p), rhs_el_tile_y(s->p));
  return J;
}

KronJob kron_base(const ads_sim* s, double* out, const double* base, double alpha) {
  KronJob K{};
  K.out = out;
  K.base = base;
  K.alpha = alpha;
  K.p = s->p;
  K.nx = s->nf[0];
  K.ny = s->nf[1];
  K.nz = s->nf[2];
  K.nterm = 0;
  K.tile0 = 0;
  K.tiles[0] = (K.nx + kron_tile_x() - 1) / kron_tile_x();
  K.tiles[1] = (K.ny + kron_tile_y() - 1) / kron_tile_y();
  // a tile walks TZ + 2p source layers
  set_kron_zchunks(K, best_zchunks({{(long long)K.tiles[0] * K.tiles[1], K.nz}}, 2 * K.p,
                                   (long long)kron_blocks_per_cu(s->p) * s->ncu));
  return K;
}

// Upsilon_ik (i != k) as two tensor-product terms acting on src.
void kron_add_upsilon(const ads_sim* s, KronJob& K, int i, int k, const double* src, double coef) {
  const int j = 3 - i - k;
  KronTerm tm{}, tl{};
  tm.src = tl.src = src;
  tm.T[i] = s->d_bandG[i];
  tm.T[k] = s->d_bandGT[k];
  tm.T[j] = s->d_bandM[j];
  tm.coef = coef * s->prm.mu;
  tl.T[i] = s->d_bandGT[i];
  tl.T[k] = s->d_bandG[k];
  tl.T[j] = s->d_bandM[j];
  tl.coef = coef * s->prm.lambda;
  K.term[K.nterm++] = tm;
  K.term[K.nterm++] = tl;
}

void kron_add_mass(const ads_sim* s, KronJob& K, const double* src, double coef) {
  KronTerm t{};
  t.src = src;
  for (int d = 0; d < 3; ++d) t.T[d] = s->d_bandM[d];
  t.coef = coef;
  K.term[K.nterm++] = t;
}

bool push_kron(ads_sim* s, std::vector<Launch>& L, const KronJob& K, std::string& err) {
  const LaunchHdr* d = s->arena.add(std::vector<KronJob>{K}, err);
  if (!d) return false;
  L.push_back(Launch{Launch::KRON, d, 1, K.ntiles, 0, s->p, -1, 0, 0, as_bytes(K)});
  return true;
}

// The coupling of a stage goes into the in-plane sweep of the solve that
// consumes it when the plane takes it; its launch slot then stays, empty
// (no tiles, nothing launched), so that every elasticity step has the same
// launch sequence (the pool's stages).
bool couple_in_plane(const ads_sim* s) { return s->couple_fused && plane_couple_fits(s->nf[0], s->nf[1], s->p); }
void push_empty_kron(ads_sim* s, std::vector<Launch>& L) {
  L.push_back(Launch{Launch::KRON, nullptr, 0, 0, 0, s->p, -1, 0, 0, {}});
}

// Alternating-triangular solve Z = D^{-1} R (three-level form of eq. pre /
// eq. corr with the split diagonal blocks of eq. spill); with `update` the
// last sweep of every component also performs U^{n+1} = 2U^n - U^{n-1} + Z.
bool add_at_solve(ads_sim* s, std::vector<Launch>& L, bool update, bool count, std::string& err) {
  const long long nf = s->nfree;
  const double tau = s->prm.tau, rho = s->prm.rho, h = 0.5 * tau * tau;
  auto facs = [&](int i, DevFactor out[3]) {
    for (int d = 0; d < 3; ++d) out[d] = (d == i) ? s->fS2[d] : s->fS[d];
  };
  const bool in_plane = couple_in_plane(s);
  // stage 1 (block lower): components x, y, z
  for (int i = 0; i < 3; ++i) {
    const double* rhs = s->R + i * nf;
    KronJob K = kron_base(s, s->T, s->R + i * nf, 1.0);
    if (i > 0) {
      for (int jj = 0; jj < i; ++jj) kron_add_upsilon(s, K, i, jj, s->Y + jj * nf, -h);
      if (in_plane) {
        push_empty_kron(s, L);
      } else {
        if (!push_kron(s, L, K, err)) return false;
        rhs = s->T;
      }
    }
    DevFactor f[3];
    facs(i, f);
    const int nt = (i > 0 && in_plane) ? K.nterm : 0;
    if (!add_ads_solve(s, L, f, rhs, s->Z + i * nf /*tmp*/, s->Y + i * nf, 1.0 / rho, plain_epi(), err, K.term, nt))
      return false;
  }
  // stage 2 (block upper): components z, y, x
  for (int i = 2; i >= 0; --i) {
    KronJob K = kron_base(s, s->T, nullptr, 0.0);
    kron_add_mass(s, K, s->Y + i * nf, rho);
    for (int jj = i + 1; jj < 3; ++jj) kron_add_upsilon(s, K, i, jj, s->Z + jj * nf, -h);
    if (in_plane) push_empty_kron(s, L);
    else if (!push_kron(s, L, K, err)) return false;
    DevFactor f[3];
    facs(i, f);
    SweepJob z{};
    if (update) {
      z.epi = EPI_THREELEVEL;
      z.e0 = s->u + i * nf;
      z.e1 = s->v + i * nf;
    } else {
      z.epi = EPI_STORE;
    }
    if (count && i == 0) z.counter = s->counter;
    // tmp for the y-sweep: R_i is no longer needed in stage 2
    if (in_plane) {
      if (!add_ads_solve(s, L, f, nullptr, s->R + i * nf, s->Z + i * nf, 1.0 / rho, z, err, K.term, K.nterm))
        return false;
    } else if (!add_ads_solve(s, L, f, s->T, s->R + i * nf, s->Z + i * nf, 1.0 / rho, z, err)) {
      return false;
    }
  }
  return true;
}

int grid_of(const Launch& l, int cap) { return (cap > 0 && l.total_tiles > cap) ? cap : l.total_tiles; }

ads_status enqueue(ads_sim* s, const std::vector<Launch>& L, int grid_cap = 0, hipEvent_t* evs = nullptr) {
  if (evs) HIPCHECK(hipEventRecord(evs[0], s->stream));
  for (size_t li = 0; li < L.size(); ++li) {
    const Launch& l = L[li];
    hipError_t e = hipSuccess;
    switch (l.kind) {
      case Launch::RHS_P:
        e = launch_rhs_pwave(l.p, l.mixed, l.var, l.coef, l.d_hdr, grid_of(l, grid_cap), s->stream);
        break;
      case Launch::RHS_E:
        e = l.var == 3 ? launch_rhs_elastic_band(l.p, l.mixed, l.d_hdr, grid_of(l, grid_cap), s->stream)
                       : launch_rhs_elastic(l.p, l.d_hdr, grid_of(l, grid_cap), s->stream);
        break;
      case Launch::SWEEP:
        e = launch_sweeps(l.d_hdr, grid_of(l, grid_cap), l.w, l.max_m, l.p, s->stream);
        break;
      case Launch::KRON:
        e = launch_kron(l.d_hdr, grid_of(l, grid_cap), l.p, s->stream);
        break;
      case Launch::PLANE:
        e = launch_planes(l.d_hdr, grid_of(l, grid_cap), l.lds, l.p, l.coupled, s->stream);
        break;
    }
    if (e != hipSuccess) return fail(ADS_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    if (evs) HIPCHECK(hipEventRecord(evs[li + 1], s->stream));
  }
  return ADS_OK;
}

// 0 right-hand side, 1/2/3 x/y/z sweep, 4 coupling, 6 in-plane (x and y) sweeps
int launch_kind_code(const Launch& l) {
  if (l.kind == Launch::RHS_P || l.kind == Launch::RHS_E) return 0;
  if (l.kind == Launch::KRON) return 4;
  if (l.kind == Launch::PLANE) return 6;
  return 1 + l.dir;
}

ads_status upload(ads_sim* s, void* dst, const void* src, size_t bytes) {
  HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream));
  return ADS_OK;
}

ads_status upload_factor(ads_sim* s, const DevFactor& f, const Band& A) {
  BandLU lu;
  if (!band_lu(A, lu)) return fail(ADS_ENUMERIC, "banded LU met a non-positive pivot");
  ads_status st;
  if ((st = upload(s, f.L, lu.L.data(), lu.L.size() * 8)) != ADS_OK) return st;
  if ((st = upload(s, f.U, lu.U.data(), lu.U.size() * 8)) != ADS_OK) return st;
  return upload(s, f.rd, lu.rd.data(), lu.rd.size() * 8);
}

// P-wave: the stepping state (w, b) from u, v, a (after the state was set or
// started), and u, v back from w, b, a (after time steps), on the stream.
// The printed coefficient set steps (w, v, a): only w and u convert.
ads_status sync_predictor(ads_sim* s) {
  if (s->elastic || !s->w_stale) return ADS_OK;
  const double tau = s->prm.tau;
  HIPCHECK(launch_lin3(s->w, s->u, s->v, s->literal ? nullptr : s->a, tau, 0.25 * tau * tau, s->nfree, s->stream));
  if (!s->literal) HIPCHECK(launch_lin3(s->b, s->v, s->a, nullptr, 0.5 * tau, 0.0, s->nfree, s->stream));
  s->w_stale = false;
  return ADS_OK;
}
ads_status materialize_u(ads_sim* s) {
  if (s->elastic || !s->u_stale) return ADS_OK;
  const double tau = s->prm.tau;
  if (!s->literal) HIPCHECK(launch_lin3(s->v, s->b, s->a, nullptr, -0.5 * tau, 0.0, s->nfree, s->stream));
  HIPCHECK(launch_lin3(s->u, s->w, s->v, s->literal ? nullptr : s->a, -tau, -0.25 * tau * tau, s->nfree, s->stream));
  s->u_stale = false;
  return ADS_OK;
}
// the stepping state's second field: b (Newmark) or v (printed set)
double* step_field1(const ads_sim* s) { return s->literal ? s->v : s->b; }

// (Re)build every job table and launch list; uploads the arena.
ads_status build_launches(ads_sim* s) {
  std::string err;
  s->arena.host.clear();
  s->step_l.clear();
  s->start_l.clear();
  s->projM_l.clear();
  s->energy_l.clear();
  const double tau = s->prm.tau;
  if (!s->elastic) {
    // step: RHS with the Newmark predictor, sweeps, z-sweep fused with the update
    // (the printed coefficient set drops the u'' term of the predictor)
    RhsJob rj = rhs_pwave_job(s, s->w, 1, s->mixed ? 1 : 0, s->rhs_var);
    // BF16 inputs: the predictor rounded to BF16, then a second pass on the
    // remainder accumulated into R (the one-step correction)
    std::vector<RhsJob> passes{rj};
    if (s->bf16) {
      passes[0].wsplit = 1;
      RhsJob lo = rj;
      lo.wsplit = 2;
      lo.accumulate = 1;
      lo.load = nullptr;
      passes.push_back(lo);
    }
    const LaunchHdr* d = nullptr;
    for (const RhsJob& pj : passes) {
      d = s->arena.add(std::vector<RhsJob>{pj}, err);
      if (!d) return fail(ADS_ENOMEM, err);
      s->step_l.push_back(
          Launch{Launch::RHS_P, d, 1, pj.ntiles, 0, s->p, -1, rhs_form_var(s->rhs_var, s->coef != nullptr, s->mixed),
                 s->mixed ? 1 : 0, as_bytes(pj)});
      s->step_l.back().coef = s->coef != nullptr;
    }
    SweepJob z{};
    z.epi = s->literal ? EPI_NEWMARK_LITERAL : EPI_NEWMARK;
    z.c0 = tau;
    z.c1 = tau * tau;
    z.e0 = s->w;
    z.e1 = step_field1(s);
    z.e2 = s->a;
    z.counter = s->counter;
    if (!add_ads_solve(s, s->step_l, s->fS, s->R, s->R, nullptr, 1.0, z, err)) return fail(ADS_ENOMEM, err);
    // start: u''_0 = G^{-1}(F_0 - K u_0)
    // the start is computed in FP64 in every precision mode
    const int av = rhs_form_var(fp64_aux_var(s), s->coef != nullptr, false);
    RhsJob r0 = rhs_pwave_job(s, s->u, 0, 0, av);
    d = s->arena.add(std::vector<RhsJob>{r0}, err);
    if (!d) return fail(ADS_ENOMEM, err);
    s->start_l.push_back(Launch{Launch::RHS_P, d, 1, r0.ntiles, 0, s->p, -1, av, 0, as_bytes(r0)});
    s->start_l.back().coef = s->coef != nullptr;
    // energy diagnostic: R = K u, R = K v (FP64 quadrature), R = G v (split operator)
    for (double* src : {s->u, s->v}) {
      RhsJob ke = rhs_pwave_job(s, src, 0, 0, av);
      ke.load = nullptr;
      ke.amp = nullptr;
      ke.rscale = -1.0;
      d = s->arena.add(std::vector<RhsJob>{ke}, err);
      if (!d) return fail(ADS_ENOMEM, err);
      s->energy_l.push_back(Launch{Launch::RHS_P, d, 1, ke.ntiles, 0, s->p, -1, av, 0, as_bytes(ke)});
      s->energy_l.back().coef = s->coef != nullptr;
    }
    {
      KronJob G = kron_base(s, s->R, nullptr, 0.0);
      KronTerm t{};
      t.src = s->v;
      for (int dd = 0; dd < 3; ++dd) t.T[dd] = s->d_bandA[dd];
      t.coef = 1.0;
      G.term[G.nterm++] = t;
      if (!push_kron(s, s->energy_l, G, err)) return fail(ADS_ENOMEM, err);
    }
    if (!add_ads_solve(s, s->start_l, s->fS, s->R, s->R, s->a, 1.0, plain_epi(), err))
      return fail(ADS_ENOMEM, err);
  } else {
    // step: the chosen variant and precision; start and energy in FP64
    const int mx = (s->mixed && s->rhs_var == 3) ? 1 : 0;
    RhsJob rj = rhs_elastic_job(s, s->rhs_var, mx);
    const LaunchHdr* d = s->arena.add(std::vector<RhsJob>{rj}, err);
    if (!d) return fail(ADS_ENOMEM, err);
    s->step_l.push_back(Launch{Launch::RHS_E, d, 1, rj.ntiles, 0, s->p, -1, s->rhs_var, mx, as_bytes(rj)});
    if (!add_at_solve(s, s->step_l, true, true, err)) return fail(ADS_ENOMEM, err);
    RhsJob r0 = rhs_elastic_job(s, s->rhs_var, 0);
    d = s->arena.add(std::vector<RhsJob>{r0}, err);
    if (!d) return fail(ADS_ENOMEM, err);
    s->start_l.push_back(Launch{Launch::RHS_E, d, 1, r0.ntiles, 0, s->p, -1, s->rhs_var, 0, as_bytes(r0)});
    if (!add_at_solve(s, s->start_l, false, false, err)) return fail(ADS_ENOMEM, err);
    // energy diagnostic (V = (U^{n+1} - U^n)/tau in Y, W = (U^{n+1} + U^n)/2 in Z):
    // R = Upsilon W, R = Upsilon V (quadrature), R = L^T V (split diagonal and
    // upper couplings), Z = (rho M)^{-1} R per component
    const long long nf = s->nfree;
    const double tau = s->prm.tau, rho = s->prm.rho, h = 0.5 * tau * tau;
    for (double* src : {s->Z, s->Y}) {
      RhsJob ke = rhs_elastic_job(s, s->rhs_var, 0);
      ke.u = src;
      ke.load = nullptr;
      ke.amp = nullptr;
      ke.rscale = -1.0;
      d = s->arena.add(std::vector<RhsJob>{ke}, err);
      if (!d) return fail(ADS_ENOMEM, err);
      s->energy_l.push_back(Launch{Launch::RHS_E, d, 1, ke.ntiles, 0, s->p, -1, s->rhs_var, 0, as_bytes(ke)});
    }
    for (int i = 0; i < 3; ++i) {
      KronJob K = kron_base(s, s->R + i * nf, nullptr, 0.0);
      KronTerm t{};
      t.src = s->Y + i * nf;
      for (int dd = 0; dd < 3; ++dd) t.T[dd] = dd == i ? s->d_bandA2[dd] : s->d_bandA[dd];
      t.coef = rho;
      K.term[K.nterm++] = t;
      for (int jj = i + 1; jj < 3; ++jj) kron_add_upsilon(s, K, i, jj, s->Y + jj * nf, h);
      if (!push_kron(s, s->energy_l, K, err)) return fail(ADS_ENOMEM, err);
    }
    for (int i = 0; i < 3; ++i)
      if (!add_ads_solve(s, s->energy_l, s->fM, s->R + i * nf, s->T, s->Z + i * nf, 1.0 / rho, plain_epi(), err))
        return fail(ADS_ENOMEM, err);
  }
  // mass solve used by the projection: R -> R (per component, offset applied at launch)
  if (!add_ads_solve(s, s->projM_l, s->fM, s->R, s->R, s->R, 1.0, plain_epi(), err))
    return fail(ADS_ENOMEM, err);
  // a pool holds copies of the step's jobs: they are gathered again
  if (s->pool_dirty) *s->pool_dirty = true;
  return upload(s, s->arena.d_base, s->arena.host.data(), s->arena.host.size());
}

}  // namespace

namespace {
ads_status project_impl(ads_sim* s, const double* vals, double* coef, void* scratch);
}  // namespace

// ============================================================================
extern "C" {

const char* ads_last_error(void) { return g_err.c_str(); }

ads_status ads_workspace_bytes(const ads_params* prm, size_t* bytes) {
  std::string why;
  if (!valid_params(prm, why)) return fail(ADS_EINVAL, why);
  if (!bytes) return fail(ADS_EINVAL, "bytes is NULL");
  ads_sim s;
  s.prm = *prm;
  geometry(&s);
  Carver c{nullptr};
  carve(&s, c);
  *bytes = c.used;
  return ADS_OK;
}

ads_status ads_quad_points(const ads_params* prm, int32_t d, double* host_out) {
  std::string why;
  if (!valid_params(prm, why)) return fail(ADS_EINVAL, why);
  if (d < 0 || d > 2 || !host_out) return fail(ADS_EINVAL, "bad direction or NULL output");
  Tables1D t = tables_of(*prm, d);
  std::memcpy(host_out, t.X.data(), t.X.size() * sizeof(double));
  return ADS_OK;
}

ads_status ads_project_scratch_bytes(const ads_params* prm, size_t* bytes) {
  std::string why;
  if (!valid_params(prm, why)) return fail(ADS_EINVAL, why);
  if (!bytes) return fail(ADS_EINVAL, "bytes is NULL");
  const long long q = prm->nquad > 0 ? prm->nquad : prm->p + 1;
  const long long gz = (flat_z(*prm) ? 1 : prm->nelem[2]) * q, gy = prm->nelem[1] * q;
  const long long fx = free_count(*prm, 0), fy = free_count(*prm, 1);
  *bytes = (size_t)(gz * gy * fx + gz * fy * fx) * sizeof(double) + 2 * kAlign;
  return ADS_OK;
}

ads_status ads_create(const ads_params* prm, void* ws, size_t bytes, void* stream, const double* u0,
                      const double* v0, ads_sim** out) {
  std::string why;
  if (!valid_params(prm, why)) return fail(ADS_EINVAL, why);
  if (!out) return fail(ADS_EINVAL, "out is NULL");
  if (!ws) return fail(ADS_EINVAL, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign) return fail(ADS_EINVAL, "workspace must be 256-byte aligned");
  size_t need = 0;
  ads_workspace_bytes(prm, &need);
  if (bytes < need) return fail(ADS_ENOMEM, "workspace smaller than ads_workspace_bytes");
  HIPCHECK(set_attributes_once());
  int dev = 0, ncu = 0;
  HIPCHECK(hipGetDevice(&dev));
  HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  ads_sim* s = new ads_sim();
  std::unique_ptr<ads_sim> owner(s);   // frees the handle on every error return
  s->prm = *prm;
  s->stream = (hipStream_t)stream;
  geometry(s);
  s->ncu = ncu;
  if (g_force_var >= 0) s->rhs_var = g_force_var;   // simulations created by a pool
  if (s->elastic && s->rhs_var != 3) s->rhs_var = 0;  // elasticity: quadrature (0) or Kronecker form (3)
  if (!quadrature_ok(s)) s->rhs_var = 3;               // degrees and rules without a quadrature kernel
  Carver c{(char*)ws};
  carve(s, c);
  // host tables and matrices
  for (int d = 0; d < 3; ++d) {
    s->tab[d] = tables_of(s->prm, d);
    Band M = assemble(s->tab[d], MAT_MASS), K = assemble(s->tab[d], MAT_STIFF), G = assemble(s->tab[d], MAT_MIXED);
    s->Mf[d] = restrict_band(M, s->off[d], s->nf[d]);
    s->Kf[d] = restrict_band(K, s->off[d], s->nf[d]);
    s->Gf[d] = restrict_band(G, s->off[d], s->nf[d]);
  }
  ads_status st;
  for (int d = 0; d < 3; ++d) {
    const Tables1D& t = s->tab[d];
    std::vector<double> buf;
    buf.insert(buf.end(), t.N.begin(), t.N.end());
    buf.insert(buf.end(), t.D.begin(), t.D.end());
    buf.insert(buf.end(), t.W.begin(), t.W.end());
    for (const std::vector<double>* v : {&t.N, &t.D})
      for (size_t k = 0; k < v->size(); ++k) buf.push_back(t.W[k / s->P] * (*v)[k]);
    for (const std::vector<double>* v : {&t.N, &t.D})
      for (int e = 0; e < s->E[d]; ++e)
        for (int a = 0; a < s->P; ++a)
          for (int b = 0; b < s->P; ++b) {
            double m = 0.0;
            for (int g = 0; g < s->q; ++g) {
              const size_t r = ((size_t)e * s->q + g) * s->P;
              m += t.W[(size_t)e * s->q + g] * (*v)[r + a] * (*v)[r + b];
            }
            buf.push_back(m);
          }
    // band matrices of the Kronecker form: M, then K (elasticity: then G
    // and G^T); in x and y the diagonal slot of K, G and G^T holds the row
    // sum (the x- and y-passes apply them to differences to the diagonal,
    // so that FP32-rounded entries still annihilate constants); z keeps the
    // matrices themselves (its pass is FP64)
    buf.insert(buf.end(), s->Mf[d].a.begin(), s->Mf[d].a.end());
    auto push_diff_band = [&](const Band& K) {
      const int B = 2 * K.p + 1;
      for (int i = 0; i < K.n; ++i) {
        double rs = 0.0;
        for (int k = 0; k < B; ++k) rs += K.a[(size_t)i * B + k];
        for (int k = 0; k < B; ++k) buf.push_back(k == K.p && d < 2 ? rs : K.a[(size_t)i * B + k]);
      }
    };
    push_diff_band(s->Kf[d]);
    if (s->elastic) {
      Band GT = s->Gf[d];
      for (int i = 0; i < GT.n; ++i)
        for (int j = std::max(0, i - GT.p); j <= std::min(GT.n - 1, i + GT.p); ++j) GT.at(i, j) = s->Gf[d].at(j, i);
      push_diff_band(s->Gf[d]);
      push_diff_band(GT);
    }
    if ((st = upload(s, s->d_tab[d], buf.data(), buf.size() * 8)) != ADS_OK) return st;
    if ((st = upload_factor(s, s->fM[d], s->Mf[d])) != ADS_OK) return st;
    if (s->elastic) {
      Band GT = s->Gf[d];
      for (int i = 0; i < GT.n; ++i)
        for (int j = std::max(0, i - GT.p); j <= std::min(GT.n - 1, i + GT.p); ++j) GT.at(i, j) = s->Gf[d].at(j, i);
      if ((st = upload(s, s->d_bandM[d], s->Mf[d].a.data(), s->Mf[d].a.size() * 8)) != ADS_OK) return st;
      if ((st = upload(s, s->d_bandG[d], s->Gf[d].a.data(), s->Gf[d].a.size() * 8)) != ADS_OK) return st;
      if ((st = upload(s, s->d_bandGT[d], GT.a.data(), GT.a.size() * 8)) != ADS_OK) return st;
    }
  }
  const int nc = s->ncomp;
  const long long nfr = s->nfree;
  // state: u (U^n), v (u' for the P-wave; V^0 then U^{n-1} for elasticity), a
  if (launch_full_to_free(u0, s->u, s->n, s->nf, s->off, nc, s->stream) != hipSuccess ||
      launch_full_to_free(v0, s->v, s->n, s->nf, s->off, nc, s->stream) != hipSuccess)
    return fail(ADS_EDEVICE, "layout copy failed");
  if (s->a) HIPCHECK(launch_fill(s->a, nfr, 0.0, s->stream));
  HIPCHECK(launch_fill(s->load, nfr * nc, 0.0, s->stream));
  HIPCHECK(launch_fill(s->amp, kAmpCap, 0.0, s->stream));
  HIPCHECK(launch_set_u64(s->counter, 0ull, s->stream));
  if ((st = build_launches(s)) != ADS_OK) return st;
  HIPCHECK(hipStreamSynchronize(s->stream));
  s->need_start = true;
  *out = owner.release();
  return ADS_OK;
}

ads_status ads_project(ads_sim* s, const double* vals, double* coef, void* scratch, size_t scratch_bytes) {
  if (!s || !vals || !coef || !scratch) return fail(ADS_EINVAL, "NULL argument");
  size_t need = 0;
  ads_project_scratch_bytes(&s->prm, &need);
  if (scratch_bytes < need) return fail(ADS_ENOMEM, "projection scratch too small");
  return project_impl(s, vals, coef, scratch);
}

ads_status ads_project_static(ads_sim* s, const double* vals, double* coef) {
  if (!s || !vals || !coef) return fail(ADS_EINVAL, "NULL argument");
  size_t need = 0;
  ads_project_scratch_bytes(&s->prm, &need);
  if (need > kStaticScratchBytes)
    return fail(ADS_ENOMEM, "projection staging of " + std::to_string(need) + " bytes exceeds the " +
                                std::to_string(kStaticScratchBytes) + "-byte static buffer (use ads_project)");
  void* buf = nullptr;
  ads_status st = static_scratch_address(&buf);
  if (st != ADS_OK) return st;
  return project_impl(s, vals, coef, buf);
}

}  // extern "C"

namespace {

// The projection's contractions and mass sweeps with their two staging
// arrays in `scratch` (ads_project_scratch_bytes of it).
ads_status project_impl(ads_sim* s, const double* vals, double* coef, void* scratch) {
  const int q = s->q, P = s->P;
  const long long gz = (long long)s->E[2] * q, gy = (long long)s->E[1] * q, gx = (long long)s->E[0] * q;
  double* s1 = (double*)scratch;
  double* s2 = s1 + ((gz * gy * s->nf[0] + 31) / 32) * 32;
  // components last to first: component c > 0 is solved through R_0's slot
  for (int c = s->ncomp - 1; c >= 0; --c) {
    const double* g = vals + c * gz * gy * gx;
    double* b = s->R + c * s->nfree;
    HIPCHECK(launch_proj_contract(g, s1, gz * gy, s->E[0], q, P, s->nf[0], s->off[0], 1, s->d_tab[0], s->stream));
    HIPCHECK(launch_proj_contract(s1, s2, gz, s->E[1], q, P, s->nf[1], s->off[1], s->nf[0], s->d_tab[1],
                                  s->stream));
    HIPCHECK(launch_proj_contract(s2, b, 1, s->E[2], q, P, s->nf[2], s->off[2],
                                  (long long)s->nf[0] * s->nf[1], s->d_tab[2], s->stream));
    // M u = b by three sweeps with the mass factors, in place on R_0
    if (c > 0) HIPCHECK(hipMemcpyAsync(s->R, b, s->nfree * 8, hipMemcpyDeviceToDevice, s->stream));
    ads_status st = enqueue(s, s->projM_l);
    if (st != ADS_OK) return st;
    if (c > 0) HIPCHECK(hipMemcpyAsync(b, s->R, s->nfree * 8, hipMemcpyDeviceToDevice, s->stream));
  }
  HIPCHECK(launch_free_to_full(s->R, coef, s->n, s->nf, s->off, s->ncomp, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  return ADS_OK;
}

}  // namespace

extern "C" {

ads_status ads_set_load(ads_sim* s, const double* b, const double* amp, int32_t namp) {
  if (!s || !b || (namp > 0 && !amp)) return fail(ADS_EINVAL, "NULL argument");
  if (namp < 0 || namp > kAmpCap) return fail(ADS_ENOMEM, "at most 4096 load amplitudes");
  HIPCHECK(launch_full_to_free(b, s->load, s->n, s->nf, s->off, s->ncomp, s->stream));
  HIPCHECK(launch_fill(s->amp, kAmpCap, 0.0, s->stream));
  if (namp > 0) HIPCHECK(hipMemcpyAsync(s->amp, amp, namp * 8, hipMemcpyHostToDevice, s->stream));
  s->namp = namp;
  s->have_load = true;
  ads_status st = build_launches(s);
  if (st != ADS_OK) return st;
  HIPCHECK(hipStreamSynchronize(s->stream));
  return ADS_OK;
}

ads_status ads_set_point_load(ads_sim* s, const double xs[3], const double* amp, int32_t namp) {
  if (!s || !xs || (namp > 0 && !amp)) return fail(ADS_EINVAL, "NULL argument");
  if (s->elastic) return fail(ADS_EINVAL, "point loads are defined for the P-wave");
  if (namp < 0 || namp > kAmpCap) return fail(ADS_ENOMEM, "at most 4096 load amplitudes");
  std::vector<double> v[3];
  for (int d = 0; d < 3; ++d) {
    if (d == 2 && flat_z(s->prm)) {   // two-dimensional: the constant function
      v[2].assign(1, 1.0);
      continue;
    }
    double x = std::min(1.0, std::max(0.0, xs[d]));
    std::vector<double> t = open_knots(s->E[d], s->p);
    int e = std::min(s->E[d] - 1, (int)std::floor(x * s->E[d]));
    double N[8], D[8];
    basis_on_span(t, s->p, e + s->p, x, N, D);
    v[d].assign(s->nf[d], 0.0);
    for (int a = 0; a <= s->p; ++a) {
      int fi = e + a - s->off[d];
      if (fi >= 0 && fi < s->nf[d]) v[d][fi] = N[a];
    }
  }
  std::vector<double> b((size_t)s->nfree);
  for (int z = 0; z < s->nf[2]; ++z)
    for (int y = 0; y < s->nf[1]; ++y)
      for (int x = 0; x < s->nf[0]; ++x)
        b[((size_t)z * s->nf[1] + y) * s->nf[0] + x] = v[2][z] * v[1][y] * v[0][x];
  ads_status st = upload(s, s->load, b.data(), b.size() * 8);
  if (st != ADS_OK) return st;
  HIPCHECK(launch_fill(s->amp, kAmpCap, 0.0, s->stream));
  if (namp > 0) HIPCHECK(hipMemcpyAsync(s->amp, amp, namp * 8, hipMemcpyHostToDevice, s->stream));
  s->namp = namp;
  s->have_load = true;
  if ((st = build_launches(s)) != ADS_OK) return st;
  HIPCHECK(hipStreamSynchronize(s->stream));
  return ADS_OK;
}

ads_status ads_energy(ads_sim* s, double* host_energy) {
  if (!s || !host_energy) return fail(ADS_EINVAL, "NULL argument");
  if (!s->factored || s->need_start) return fail(ADS_ESTATE, "ads_energy before ads_factor");
  const int nd = dot_scratch_doubles();
  double* out = s->red + nd;
  ads_status st = materialize_u(s);
  if (st != ADS_OK) return st;
  if (s->elastic) {
    // u = U^{n+1}, v = U^n
    const long long n3 = 3 * s->nfree;
    const double tau = s->prm.tau;
    HIPCHECK(launch_axpby(s->Y, s->u, s->v, 1.0 / tau, -1.0 / tau, n3, s->stream));
    HIPCHECK(launch_axpby(s->Z, s->u, s->v, 0.5, 0.5, n3, s->stream));
    std::vector<Launch> L(s->energy_l.begin(), s->energy_l.begin() + 1);
    if ((st = enqueue(s, L)) != ADS_OK) return st;
    HIPCHECK(launch_dot(s->Z, s->R, n3, s->red, out + 0, s->stream));   // W.Upsilon W
    L.assign(s->energy_l.begin() + 1, s->energy_l.begin() + 2);
    if ((st = enqueue(s, L)) != ADS_OK) return st;
    HIPCHECK(launch_dot(s->Y, s->R, n3, s->red, out + 1, s->stream));   // V.Upsilon V
    L.assign(s->energy_l.begin() + 2, s->energy_l.end());
    if ((st = enqueue(s, L)) != ADS_OK) return st;
    HIPCHECK(launch_dot(s->R, s->Z, n3, s->red, out + 2, s->stream));   // V.D V
    double h[3];
    HIPCHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
    *host_energy = 0.5 * (h[2] - 0.25 * tau * tau * h[1]) + 0.5 * h[0];
    return ADS_OK;
  }
  // u.Ku, v.Kv, v.Gv
  const double* dots[3][2] = {{s->u, s->R}, {s->v, s->R}, {s->v, s->R}};
  for (int k = 0; k < 3; ++k) {
    std::vector<Launch> one(1, s->energy_l[k]);
    if ((st = enqueue(s, one)) != ADS_OK) return st;
    HIPCHECK(launch_dot(dots[k][0], dots[k][1], s->nfree, s->red, out + k, s->stream));
  }
  double h[3];
  HIPCHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  const double eta = 0.25 * s->prm.tau * s->prm.tau;
  *host_energy = 0.5 * (h[2] - eta * h[1]) + 0.5 * h[0];
  return ADS_OK;
}

ads_status ads_set_coefficient(ads_sim* s, const double* dev_c2, double c2ref) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  if (s->elastic) return fail(ADS_EINVAL, "the wave-speed field is a P-wave parameter");
  if (!quadrature_ok(s))
    return fail(ADS_EINVAL, "a wave-speed field needs the quadrature right-hand side (p = 2 or 3, q = p+1)");
  if (!(c2ref > 0.0) || !std::isfinite(c2ref)) return fail(ADS_EINVAL, "c2ref must be positive and finite");
  if (s->factored) return fail(ADS_ESTATE, "ads_set_coefficient after ads_factor");
  s->coef = dev_c2;
  s->c2ref = c2ref;
  return build_launches(s);
}

ads_status ads_set_scheme(ads_sim* s, int32_t scheme) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  if (scheme != ADS_SCHEME_NEWMARK && scheme != ADS_SCHEME_LITERAL) return fail(ADS_EINVAL, "unknown scheme");
  if (s->elastic && scheme != ADS_SCHEME_NEWMARK) return fail(ADS_EINVAL, "the printed scheme is a P-wave diagnostic");
  if (s->factored) return fail(ADS_ESTATE, "ads_set_scheme after ads_factor");
  s->literal = scheme == ADS_SCHEME_LITERAL;
  s->w_stale = true;   // the predictor's definition follows the scheme
  return build_launches(s);
}

ads_status ads_factor(ads_sim* s) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  const double tau = s->prm.tau;
  ads_status st;
  for (int d = 0; d < 3; ++d) {
    if (!s->elastic) {
      Band A = axpby(1.0, s->Mf[d], 0.25 * tau * tau * s->c2ref, s->Kf[d]);
      if ((st = upload_factor(s, s->fS[d], A)) != ADS_OK) return st;
      if ((st = upload(s, s->d_bandA[d], A.a.data(), A.a.size() * 8)) != ADS_OK) return st;
    } else {
      const double rho = s->prm.rho, mu = s->prm.mu, lam = s->prm.lambda;
      Band A1 = axpby(1.0, s->Mf[d], tau * tau * mu / (4.0 * rho), s->Kf[d]);
      Band A2 = axpby(1.0, s->Mf[d], tau * tau * (2.0 * mu + lam) / (4.0 * rho), s->Kf[d]);
      if ((st = upload_factor(s, s->fS[d], A1)) != ADS_OK) return st;
      if ((st = upload_factor(s, s->fS2[d], A2)) != ADS_OK) return st;
      if ((st = upload(s, s->d_bandA[d], A1.a.data(), A1.a.size() * 8)) != ADS_OK) return st;
      if ((st = upload(s, s->d_bandA2[d], A2.a.data(), A2.a.size() * 8)) != ADS_OK) return st;
    }
  }
  if (s->need_start) {
    if ((st = enqueue(s, s->start_l)) != ADS_OK) return st;
    if (s->elastic) {
      // U^{-1} = U^0 - tau V^0 + Z^0 / 2  (v holds V^0 until the start)
      const long long n3 = 3 * s->nfree;
      HIPCHECK(launch_axpby(s->v, s->u, s->v, 1.0, -tau, n3, s->stream));
      HIPCHECK(launch_axpby(s->v, s->v, s->Z, 1.0, 0.5, n3, s->stream));
    }
    s->need_start = false;
    s->w_stale = true;
  }
  if ((st = sync_predictor(s)) != ADS_OK) return st;
  HIPCHECK(hipStreamSynchronize(s->stream));
  s->factored = true;
  return ADS_OK;
}

ads_status ads_step(ads_sim* s, int32_t nsteps) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  if (nsteps < 0) return fail(ADS_EINVAL, "nsteps < 0");
  if (!s->factored || s->need_start) return fail(ADS_ESTATE, "ads_step before ads_factor");
  ads_status st0 = sync_predictor(s);
  if (st0 != ADS_OK) return st0;
  if (nsteps > 0 && !s->elastic) s->u_stale = true;
  const size_t per = s->step_l.size() + 1;
  for (int k = 0; k < nsteps; ++k) {
    hipEvent_t* evs = nullptr;
    if (s->prof) {
      size_t need = (size_t)(s->prof_steps + 1) * per;
      while (s->ev.size() < need) {
        hipEvent_t e;
        HIPCHECK(hipEventCreate(&e));
        s->ev.push_back(e);
      }
      evs = &s->ev[(size_t)s->prof_steps * per];
      s->prof_steps++;
    }
    ads_status st = enqueue(s, s->step_l, 0, evs);
    if (st != ADS_OK) return st;
  }
  return ADS_OK;
}

ads_status ads_set_launch_shape(ads_sim* s, int32_t rhs_var, int32_t rhs_tz, const int32_t* sweep_w) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  if (s->pooled) return fail(ADS_ESTATE, "launch shapes of a pooled simulation are the pool's");
  int var = s->rhs_var;
  if (rhs_var >= 0) {
    const bool ok = rhs_var == 3 || (quadrature_ok(s) && (s->elastic ? rhs_var == 0 : (rhs_var <= 2 || rhs_var == 4)));
    if (!ok) return fail(ADS_EINVAL, "right-hand-side variant not available for this problem and degree");
    var = rhs_var;
  }
  if (rhs_tz < -1 || rhs_tz > 4096) return fail(ADS_EINVAL, "rhs_tz must be -1 (keep), 0 (automatic) or a depth");
  int w[3] = {s->sweep_w[0], s->sweep_w[1], s->sweep_w[2]};
  if (sweep_w) {
    for (int d = 0; d < 3; ++d) {
      if (sweep_w[d] < 0) continue;
      if (sweep_w[d] != 0 && !sweep_width_fits(sweep_w[d], max_m(s), s->p))
        return fail(ADS_EINVAL, "sweep tile width must be 0 (default), 4, 8 or 16 lines and fit the LDS");
      w[d] = sweep_w[d];
    }
  }
  s->rhs_var = var;
  if (rhs_tz >= 0) s->tz = rhs_tz;
  for (int d = 0; d < 3; ++d) s->sweep_w[d] = w[d];
  return build_launches(s);
}

ads_status ads_set_coupling(ads_sim* s, int32_t fused) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  if (!s->elastic) return fail(ADS_EINVAL, "the couplings are elasticity's");
  if (fused != 0 && fused != 1) return fail(ADS_EINVAL, "fused must be 0 or 1");
  if (s->pooled) return fail(ADS_ESTATE, "launch shapes of a pooled simulation are the pool's");
  s->couple_fused = fused != 0;
  return build_launches(s);
}

int32_t ads_coupling_fused(const ads_sim* s) { return (s && s->elastic && couple_in_plane(s)) ? 1 : 0; }

ads_status ads_tune(ads_sim* s, int32_t* chosen, double* host_ms, int32_t cap) {
  if (!s || !chosen) return fail(ADS_EINVAL, "NULL argument");
  if (!s->factored) return fail(ADS_ESTATE, "ads_tune before ads_factor");
  if (s->pooled) return fail(ADS_ESTATE, "ads_tune on a pooled simulation (the pool fixes its launch classes)");
  // choices cached per process (keyed by problem, degree, precision, field
  // or none, mesh); the lock makes concurrent tuning from several threads safe
  static std::mutex cache_mu;
  static std::map<std::string, int> cache;
  auto cached = [&](const std::string& k, int* v) {
    std::lock_guard<std::mutex> lock(cache_mu);
    auto it = cache.find(k);
    if (it == cache.end()) return false;
    *v = it->second;
    return true;
  };
  auto remember = [&](const std::string& k, int v) {
    std::lock_guard<std::mutex> lock(cache_mu);
    cache[k] = v;
  };
  // the wave-speed field is part of the key: without one the Kronecker form
  // is a candidate, with one it is not
  const std::string key = std::string(s->elastic ? "E" : "P") + std::to_string(s->p) + "/" +
                          std::to_string(s->mixed) + "/" + std::to_string(s->coef != nullptr) + "/" +
                          std::to_string(s->nf[0]) + "x" + std::to_string(s->nf[1]) + "x" + std::to_string(s->nf[2]);
  // candidates: P-wave tile variants 0-2 of the quadrature and the Kronecker
  // form 3 (without a wave-speed field); elasticity quadrature 0 and 3
  std::vector<int> cands;
  if (!quadrature_ok(s)) cands = {3};
  else if (s->elastic) cands = {0, 3};
  else
    for (int v = 0; v <= 4; ++v)
      if (rhs_variant_exists(s->p, s->mixed, v, s->coef != nullptr)) cands.push_back(v);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  // mean ms of 5 back-to-back launches after a warm-up launch
  auto timed = [&](auto&& launch, double* ms) -> ads_status {
    ads_status st = launch();
    if (st != ADS_OK) return st;
    HIPCHECK(hipEventRecord(e0, s->stream));
    const int reps = 5;
    for (int r = 0; r < reps; ++r)
      if ((st = launch()) != ADS_OK) return st;
    HIPCHECK(hipEventRecord(e1, s->stream));
    HIPCHECK(hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHECK(hipEventElapsedTime(&f, e0, e1));
    *ms = f / reps;
    return ADS_OK;
  };
  ads_status st;
  int best = -1;
  if (!cached(key, &best)) {
    double best_ms = 1e30;
    for (int v : cands) {
      s->rhs_var = v;
      if ((st = build_launches(s)) != ADS_OK) return st;
      std::vector<Launch> one(1, s->step_l[0]);
      double per = 0.0;
      if ((st = timed([&] { return enqueue(s, one); }, &per)) != ADS_OK) return st;
      if (host_ms && v < cap) host_ms[v] = per;
      if (per < best_ms) {
        best_ms = per;
        best = v;
      }
    }
    remember(key, best);
  }
  s->rhs_var = best;
  // elasticity: the couplings by separate launches or in the in-plane
  // sweeps, timed over the step's coupling and in-plane launches (they
  // write only the step's temporaries)
  if (s->elastic && plane_couple_fits(s->nf[0], s->nf[1], s->p)) {
    const std::string ckey = key + "/v" + std::to_string(best) + "/C";
    int fused = 0;
    if (!cached(ckey, &fused)) {
      double ms[2] = {0.0, 0.0};
      for (int f = 0; f < 2; ++f) {
        s->couple_fused = f != 0;
        if ((st = build_launches(s)) != ADS_OK) return st;
        std::vector<Launch> cl;
        for (const Launch& l : s->step_l)
          if (l.kind == Launch::KRON || l.kind == Launch::PLANE) cl.push_back(l);
        if ((st = timed([&] { return enqueue(s, cl); }, &ms[f])) != ADS_OK) return st;
      }
      fused = ms[1] < ms[0] ? 1 : 0;
      remember(ckey, fused);
    }
    s->couple_fused = fused != 0;
  }
  // sweep tile widths, per direction: the step's sweeps of that direction,
  // timed on copies of their jobs that solve in place with a plain store (no
  // time update, no step counter), placed after the job arena's tables, so
  // that only the step's temporaries change
  for (int d = 0; d < 3; ++d) {
    if ((st = build_launches(s)) != ADS_OK) return st;
    bool has = false;
    for (const Launch& l : s->step_l) has = has || (l.kind == Launch::SWEEP && l.dir == d);
    if (!has) continue;
    const std::string wkey = key + "/v" + std::to_string(best) + "/W" + std::to_string(d);
    int bw = 0;
    if (!cached(wkey, &bw)) {
      double best_ms = 1e30;
      for (int W : {4, 8, 16}) {
        if (!sweep_width_fits(W, max_m(s), s->p)) continue;
        s->sweep_w[d] = W;
        if ((st = build_launches(s)) != ADS_OK) return st;
        const size_t tail = (s->arena.host.size() + kAlign - 1) / kAlign * kAlign;
        if (tail + sizeof(LaunchHdr) + sizeof(SweepJob) > s->arena.cap) break;
        double tot = 0.0;
        for (const Launch& l : s->step_l) {
          if (l.kind != Launch::SWEEP || l.dir != d) continue;
          SweepJob j;
          std::memcpy(&j, l.host_jobs.data(), sizeof(j));
          j.epi = EPI_STORE;
          j.out = const_cast<double*>(j.in);
          j.counter = nullptr;
          j.tile0 = 0;
          LaunchHdr h{};
          h.njobs = 1;
          h.total_tiles = j.ntiles;
          std::vector<char> buf(sizeof(LaunchHdr) + sizeof(SweepJob));
          std::memcpy(buf.data(), &h, sizeof(h));
          std::memcpy(buf.data() + sizeof(LaunchHdr), &j, sizeof(j));
          HIPCHECK(hipMemcpyAsync(s->arena.d_base + tail, buf.data(), buf.size(), hipMemcpyHostToDevice, s->stream));
          const LaunchHdr* dh = (const LaunchHdr*)(s->arena.d_base + tail);
          double ms = 0.0;
          auto go = [&]() -> ads_status {
            const hipError_t e = launch_sweeps(dh, l.total_tiles, l.w, l.max_m, l.p, s->stream);
            return e == hipSuccess ? ADS_OK : fail(ADS_EDEVICE, std::string("tuner launch: ") + hipGetErrorString(e));
          };
          if ((st = timed(go, &ms)) != ADS_OK) return st;
          tot += ms;
        }
        if (tot < best_ms) {
          best_ms = tot;
          bw = W;
        }
      }
      remember(wkey, bw);
    }
    s->sweep_w[d] = bw;
  }
  if ((st = build_launches(s)) != ADS_OK) return st;
  HIPCHECK(hipStreamSynchronize(s->stream));
  *chosen = best;
  return ADS_OK;
}

ads_status ads_profile(ads_sim* s, int32_t enable) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  s->prof = enable != 0;
  s->prof_steps = 0;
  return ADS_OK;
}

ads_status ads_profile_read(ads_sim* s, double* ms, int32_t* kind, int32_t cap, int32_t* nlaunch, double* step_ms,
                            int32_t step_cap, int32_t* nsteps) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  HIPCHECK(hipStreamSynchronize(s->stream));
  const size_t L = s->step_l.size(), per = L + 1;
  std::vector<double> sum(L, 0.0);
  for (int k = 0; k < s->prof_steps; ++k) {
    hipEvent_t* e = &s->ev[(size_t)k * per];
    for (size_t i = 0; i < L; ++i) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, e[i], e[i + 1]));
      sum[i] += t;
    }
    if (step_ms && k < step_cap) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, e[0], e[L]));
      step_ms[k] = t;
    }
  }
  for (size_t i = 0; i < L && (int)i < cap; ++i) {
    if (ms) ms[i] = s->prof_steps ? sum[i] / s->prof_steps : 0.0;
    if (kind) kind[i] = launch_kind_code(s->step_l[i]);
  }
  if (nlaunch) *nlaunch = (int32_t)L;
  if (nsteps) *nsteps = s->prof_steps;
  s->prof_steps = 0;
  return ADS_OK;
}

ads_status ads_check_finite(ads_sim* s) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  const long long n = s->nfree * s->ncomp;
  ads_status st = materialize_u(s);
  if (st != ADS_OK) return st;
  HIPCHECK(launch_set_u64(s->flag, 0ull, s->stream));
  HIPCHECK(launch_nonfinite(s->u, n, s->flag, s->stream));
  HIPCHECK(launch_nonfinite(s->v, n, s->flag, s->stream));
  if (s->a) HIPCHECK(launch_nonfinite(s->a, n, s->flag, s->stream));
  unsigned long long cnt = 0;
  HIPCHECK(hipMemcpyAsync(&cnt, s->flag, 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  if (cnt) return fail(ADS_ENUMERIC, std::to_string(cnt) + " non-finite state entries");
  return ADS_OK;
}

ads_status ads_get_state(ads_sim* s, double* u, double* v, double* a) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  if (u || v) {
    ads_status st = materialize_u(s);
    if (st != ADS_OK) return st;
  }
  const int nc = s->ncomp;
  if (u) HIPCHECK(launch_free_to_full(s->u, u, s->n, s->nf, s->off, nc, s->stream));
  if (v) HIPCHECK(launch_free_to_full(s->v, v, s->n, s->nf, s->off, nc, s->stream));
  if (a && s->a) HIPCHECK(launch_free_to_full(s->a, a, s->n, s->nf, s->off, 1, s->stream));
  return ADS_OK;
}

ads_status ads_set_state(ads_sim* s, const double* u, const double* v, const double* a, int64_t step) {
  if (!s || !u) return fail(ADS_EINVAL, "NULL argument");
  if (step < 0) return fail(ADS_EINVAL, "step < 0");
  const int nc = s->ncomp;
  HIPCHECK(launch_full_to_free(u, s->u, s->n, s->nf, s->off, nc, s->stream));
  HIPCHECK(launch_full_to_free(v, s->v, s->n, s->nf, s->off, nc, s->stream));
  if (!s->elastic) {
    if (a) HIPCHECK(launch_full_to_free(a, s->a, s->n, s->nf, s->off, 1, s->stream));
    s->need_start = (a == nullptr);
    s->u_stale = false;
    s->w_stale = true;
    if (a) {
      ads_status st = sync_predictor(s);
      if (st != ADS_OK) return st;
    }
  } else {
    s->need_start = (v == nullptr);
  }
  HIPCHECK(launch_set_u64(s->counter, (unsigned long long)step, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  return ADS_OK;
}

ads_status ads_checkpoint_save(ads_sim* s, double* s0, double* s1, double* s2) {
  if (!s || !s0 || !s1 || (!s->elastic && !s2)) return fail(ADS_EINVAL, "NULL argument");
  if (!s->factored || s->need_start) return fail(ADS_ESTATE, "ads_checkpoint_save before ads_factor");
  const int nc = s->ncomp;
  if (s->elastic) {
    HIPCHECK(launch_free_to_full(s->u, s0, s->n, s->nf, s->off, nc, s->stream));
    HIPCHECK(launch_free_to_full(s->v, s1, s->n, s->nf, s->off, nc, s->stream));
    return ADS_OK;
  }
  ads_status st = sync_predictor(s);
  if (st != ADS_OK) return st;
  HIPCHECK(launch_free_to_full(s->w, s0, s->n, s->nf, s->off, 1, s->stream));
  HIPCHECK(launch_free_to_full(step_field1(s), s1, s->n, s->nf, s->off, 1, s->stream));
  HIPCHECK(launch_free_to_full(s->a, s2, s->n, s->nf, s->off, 1, s->stream));
  return ADS_OK;
}

ads_status ads_checkpoint_load(ads_sim* s, const double* s0, const double* s1, const double* s2, int64_t step) {
  if (!s || !s0 || !s1 || (!s->elastic && !s2)) return fail(ADS_EINVAL, "NULL argument");
  if (step < 0) return fail(ADS_EINVAL, "step < 0");
  const int nc = s->ncomp;
  if (s->elastic) {
    HIPCHECK(launch_full_to_free(s0, s->u, s->n, s->nf, s->off, nc, s->stream));
    HIPCHECK(launch_full_to_free(s1, s->v, s->n, s->nf, s->off, nc, s->stream));
  } else {
    HIPCHECK(launch_full_to_free(s0, s->w, s->n, s->nf, s->off, 1, s->stream));
    HIPCHECK(launch_full_to_free(s1, step_field1(s), s->n, s->nf, s->off, 1, s->stream));
    HIPCHECK(launch_full_to_free(s2, s->a, s->n, s->nf, s->off, 1, s->stream));
    s->w_stale = false;
    s->u_stale = true;
  }
  s->need_start = false;
  HIPCHECK(launch_set_u64(s->counter, (unsigned long long)step, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  return ADS_OK;
}

ads_status ads_get_step(ads_sim* s, int64_t* step) {
  if (!s || !step) return fail(ADS_EINVAL, "NULL argument");
  unsigned long long v = 0;
  HIPCHECK(hipMemcpyAsync(&v, s->counter, 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  *step = (int64_t)v;
  return ADS_OK;
}

ads_status ads_destroy(ads_sim* s) {
  if (!s) return fail(ADS_EINVAL, "NULL sim");
  delete s;
  return ADS_OK;
}

}  // extern "C"

// ============================================================================
// Batched pool
// ============================================================================
namespace {

// Launches after the right-hand side: per direction-split solve an in-plane
// (x, y) launch and a z-sweep, a coupling before every elasticity solve but
// the first (elasticity: 6 x 2 + 5; the P-wave uses the first two).
constexpr int kPoolStages = 17;
constexpr int kPoolMaxM = 128;    // free coefficients per direction in pooled simulations
constexpr int kStepEventCap = 1 << 16;   // pool steps timed between two ads_pool_step_times calls
static_assert(kPoolMaxM <= 128, "a pooled z-plane fits in LDS");

bool is_kron_stage(int k) { return k % 3 == 0; }    // stages 3, 6, 9, 12, 15
bool is_plane_stage(int k) { return k % 3 == 1; }   // stages 1, 4, 7, 10, 13, 16

struct PoolLaunch {
  Launch::Kind kind;
  int p, mixed, var, coef;
  int stage;        // 0: right-hand side class, k >= 1: k-th launch after it
  int grid;
  int w;            // sweeps: lines per wave tile (chosen per batch)
  size_t lds;       // in-plane sweeps: dynamic LDS bytes (largest plane of the batch)
  bool coupled;     // in-plane sweeps: some job carries coupling terms
  size_t off, cap;  // table offset/capacity (bytes) in the pool's table region: one table
                    // (header + max_slots jobs) per branch, `boff` bytes apart
  size_t job_size;
  size_t boff;
};

// Concurrent branches of a pool step: the active simulations are split into
// up to two groups whose launch sequences run on two streams (forked from
// and joined back into the pool's stream), so that one group's latency-bound
// stages overlap the other's bandwidth-bound ones.
constexpr int kPoolBranches = 2;

}  // namespace

struct ads_pool {
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t bytes = 0;
  int max_slots = 0;
  char* d_tab = nullptr;
  size_t tab_bytes = 0;
  std::vector<char> h_tab;
  size_t arena_off = 0;
  std::map<size_t, size_t> used;   // arena offset -> size
  struct Slot {
    ads_sim* sim = nullptr;
    size_t off = 0, size = 0;
    bool active = false;
  };
  std::vector<Slot> slots;
  std::vector<PoolLaunch> seq;
  bool dirty = true;
  bool use_graph = true;
  hipGraph_t graph = nullptr, graph2 = nullptr;      // a step of branch 0 (pool stream) and 1 (side)
  hipGraphExec_t exec = nullptr, exec2 = nullptr;
  std::vector<hipEvent_t> ev;
  int nev = 0;
  // P-wave right-hand-side variant per [p-1][mixed][wave-speed field]: by
  // default the Kronecker form (HBM-bound), and the quadrature's 14/13-row
  // tiles (variant 0) with a field; ads_pool_tune measures the others
  int var[kMaxP][2][2];
  // elasticity couplings of every pooled simulation: separate launches or
  // in the in-plane sweeps (ads_pool_tune times both on the batch)
  bool couple_fused = false;
  std::vector<int> w_force;        // per launch class: sweep tile width chosen by the tuner (0: default)
  size_t tune_off = 0;             // table region for the tuner's timing launches
  std::map<std::string, int> tune_cache;   // launch class + batch shape -> choice
  bool prof = false;
  std::vector<hipEvent_t> pev;     // (launches + 1) per profiled step
  int prof_steps = 0;
  std::vector<int> nonempty;       // per launch class: 0 = no jobs in the batch, else its
                                   // launch shape (sweeps: tile width)
  std::vector<int> captured;       // ... when the graph was captured
  int ncu = 0;
  // branches: the number asked for (ads_pool_set_branches), the number the
  // tables are built with (one while profiling), the branch of every slot,
  // and the second stream with the fork and join events
  int want_branches = kPoolBranches, nbranch = kPoolBranches;
  std::vector<int> branch;
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  ~ads_pool() {
    // replays still in flight finish before their graphs and streams go
    if (stream) (void)hipStreamSynchronize(stream);
    if (side) (void)hipStreamSynchronize(side);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (exec2) (void)hipGraphExecDestroy(exec2);
    if (graph2) (void)hipGraphDestroy(graph2);
    if (side) (void)hipStreamDestroy(side);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : pev) (void)hipEventDestroy(e);
    for (Slot& s : slots) delete s.sim;
  }
};

namespace {

void pool_build_seq(ads_pool* P, int ncu) {
  P->seq.clear();
  size_t off = 0;
  auto add = [&](Launch::Kind k, int p, int mixed, int var, int coef, int stage, int grid, size_t js) {
    const size_t one = sizeof(LaunchHdr) + (size_t)P->max_slots * js;
    const size_t boff = (one + kAlign - 1) / kAlign * kAlign;
    PoolLaunch L{k, p, mixed, var, coef, stage, grid, 4, 0, false, off, one, js, boff};
    off += kPoolBranches * boff;
    P->seq.push_back(L);
  };
  // right-hand-side classes: P-wave per degree, precision and wave-speed
  // field (fields only where the quadrature exists), elasticity per degree
  // and precision (Kronecker form)
  for (int p = 1; p <= kMaxP; ++p)
    for (int mixed = 0; mixed <= 1; ++mixed)
      for (int coef = 0; coef <= (quadrature_ok(p) ? 1 : 0); ++coef) {
        int var = quadrature_ok(p) ? P->var[p - 1][mixed][coef] : 3;
        add(Launch::RHS_P, p, mixed, var, coef, 0, rhs_blocks_per_cu(p, mixed, var, coef) * ncu, sizeof(RhsJob));
      }
  for (int p = 1; p <= kMaxP; ++p)
    for (int mixed = 0; mixed <= 1; ++mixed)
      add(Launch::RHS_E, p, mixed, 3, 0, 0, rhs_el_band_blocks_per_cu(p, mixed) * ncu, sizeof(RhsJob));
  for (int k = 1; k <= kPoolStages; ++k) {
    if (is_kron_stage(k)) add(Launch::KRON, 0, 0, 0, 0, k, kron_blocks_per_cu(kMaxP) * ncu, sizeof(KronJob));
    else if (is_plane_stage(k)) add(Launch::PLANE, 0, 0, 0, 0, k, ncu, sizeof(PlaneJob));
    else add(Launch::SWEEP, 0, 0, 0, 0, k, sweep_blocks_per_cu(4, kPoolMaxM, kMaxP) * ncu, sizeof(SweepJob));
  }
  P->w_force.assign(P->seq.size(), 0);
  P->tune_off = off;
  off += (sizeof(LaunchHdr) + (size_t)P->max_slots * sizeof(SweepJob) + kAlign - 1) / kAlign * kAlign;
  P->tab_bytes = off;
}

// The pool chooses the P-wave right-hand-side variant per class and the
// form of the elasticity couplings: an active simulation whose step was
// built with another (a wave-speed field set after admission, or the pool
// retuned) is rebuilt with the pool's.
ads_status pool_align(ads_pool* P) {
  for (ads_pool::Slot& sl : P->slots) {
    if (!sl.active) continue;
    ads_sim* s = sl.sim;
    if (s->elastic) {
      if (s->couple_fused == P->couple_fused) continue;
      s->couple_fused = P->couple_fused;
      ads_status st = build_launches(s);
      if (st != ADS_OK) return st;
      continue;
    }
    if (!quadrature_ok(s->p)) continue;
    const int want = P->var[s->p - 1][s->mixed ? 1 : 0][s->coef != nullptr ? 1 : 0];
    if (rhs_form_var(s->rhs_var, s->coef != nullptr, s->mixed) == want) continue;
    s->rhs_var = want;
    ads_status st = build_launches(s);
    if (st != ADS_OK) return st;
  }
  return ADS_OK;
}

// Gathers the jobs of every active simulation into the merged tables, one
// table per launch class and branch.
ads_status pool_rebuild(ads_pool* P) {
  {
    ads_status st = pool_align(P);
    if (st != ADS_OK) return st;
  }
  std::fill(P->h_tab.begin(), P->h_tab.end(), 0);
  const int nb = P->nbranch;
  P->nonempty.assign(P->seq.size() * kPoolBranches, 0);
  // branches: the active simulations by their unknowns, largest first, each
  // to the branch with fewer so far
  P->branch.assign(P->slots.size(), 0);
  {
    std::vector<std::pair<long long, int>> w;
    for (size_t i = 0; i < P->slots.size(); ++i)
      if (P->slots[i].active) w.push_back({P->slots[i].sim->nfree * P->slots[i].sim->ncomp, (int)i});
    std::stable_sort(w.begin(), w.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    long long load[kPoolBranches] = {};
    for (const auto& e : w) {
      int b = 0;
      for (int c = 1; c < nb; ++c)
        if (load[c] < load[b]) b = c;
      P->branch[e.second] = b;
      load[b] += e.first;
    }
  }
  // launches of each active simulation taken by some launch class: every
  // one of them must be, or that simulation would be stepped incompletely
  std::vector<int> taken(P->slots.size(), 0);
  for (size_t li = 0; li < P->seq.size(); ++li) {
    PoolLaunch& L = P->seq[li];
    std::vector<std::vector<char>> sel[kPoolBranches];
    bool fixed_tz = false, any = false;
    for (size_t i = 0; i < P->slots.size(); ++i) {
      const ads_pool::Slot& sl = P->slots[i];
      if (!sl.active) continue;
      const std::vector<Launch>& st = sl.sim->step_l;
      if ((int)st.size() <= L.stage) continue;
      const Launch& l = st[L.stage];
      if (l.kind != L.kind) continue;
      if (l.kind == Launch::KRON && l.total_tiles == 0) {   // coupling applied in the in-plane sweep
        taken[i]++;
        continue;
      }
      if (L.stage == 0 && (l.p != L.p || l.mixed != L.mixed || l.var != L.var ||
                           (l.kind == Launch::RHS_P && l.coef != L.coef)))
        continue;
      sel[P->branch[i]].push_back(l.host_jobs);
      taken[i]++;
      fixed_tz = fixed_tz || sl.sim->tz > 0;
      any = true;
    }
    if (!any) {
      for (int b = 0; b < kPoolBranches; ++b) {
        LaunchHdr h{};
        std::memcpy(P->h_tab.data() + L.off + b * L.boff, &h, sizeof(h));
      }
      continue;
    }
    // the launch shape is the class's, over both branches: the couplings'
    // largest degree (LDS and instantiation) and grid, the in-plane sweeps'
    // largest plane, the sweeps' tile width for the class's line count
    if (L.kind == Launch::KRON) {
      int pmax = 1;
      for (int b = 0; b < nb; ++b)
        for (const auto& j : sel[b]) pmax = std::max(pmax, ((const KronJob*)j.data())->p);
      L.p = pmax;
      L.grid = kron_blocks_per_cu(pmax) * P->ncu;
    }
    if (L.kind == Launch::PLANE) {
      L.lds = 0;
      L.p = 1;
      L.coupled = false;
      for (int b = 0; b < nb; ++b)
        for (const auto& j : sel[b]) {
          const PlaneJob* r = (const PlaneJob*)j.data();
          L.lds = std::max(L.lds, plane_lds_bytes(r->nx, r->ny, r->p, r->nterm > 0));
          L.p = std::max(L.p, r->p);
          L.coupled = L.coupled || r->nterm > 0;
        }
      L.grid = plane_blocks_per_cu(L.lds, L.p, L.coupled) * P->ncu;
    }
    if (L.kind == Launch::SWEEP) {
      long long lines = 0;
      L.p = 1;
      for (int b = 0; b < nb; ++b)
        for (const auto& j : sel[b]) {
          lines += ((const SweepJob*)j.data())->nlines;
          L.p = std::max(L.p, ((const SweepJob*)j.data())->p);
        }
      const int wf = P->w_force[li];
      L.w = (wf > 0 && sweep_width_fits(wf, kPoolMaxM, L.p)) ? wf : sweep_width_for(lines, kPoolMaxM, P->ncu, L.p);
      L.grid = sweep_blocks_per_cu(L.w, kPoolMaxM, L.p) * P->ncu;
    }
    const int shape = L.kind == Launch::SWEEP ? L.w * 8 + L.p
                      : L.kind == Launch::PLANE ? ((int)L.lds * 8 + L.p) * 2 + (L.coupled ? 1 : 0)
                      : L.kind == Launch::KRON ? L.p : 1 + L.var;
    for (int b = 0; b < nb; ++b) {
      std::vector<std::vector<char>>& sb = sel[b];
      // right-hand sides: z-chunks chosen for the branch's jobs on the
      // persistent grid of this launch
      if ((L.kind == Launch::RHS_P || L.kind == Launch::RHS_E) && !sb.empty() && !fixed_tz) {
        std::vector<std::pair<long long, int>> xy_nfz;
        for (const auto& j : sb) {
          const RhsJob* r = (const RhsJob*)j.data();
          xy_nfz.push_back({(long long)r->tiles[0] * r->tiles[1], r->nf[2]});
        }
        const int k = best_zchunks(xy_nfz, L.var == 3 ? 2 * L.p : L.p, L.grid);
        for (auto& j : sb) {
          RhsJob* r = (RhsJob*)j.data();
          set_zchunks(*r, r->nf[2], k);
        }
      }
      // couplings: z-chunks for the branch's jobs
      if (L.kind == Launch::KRON && !sb.empty()) {
        std::vector<std::pair<long long, int>> xy_nfz;
        for (const auto& j : sb) {
          const KronJob* r = (const KronJob*)j.data();
          xy_nfz.push_back({(long long)r->tiles[0] * r->tiles[1], r->nz});
        }
        const int k = best_zchunks(xy_nfz, 2 * L.p, L.grid);
        for (auto& j : sb) set_kron_zchunks(*(KronJob*)j.data(), k);
      }
      if (L.kind == Launch::SWEEP)
        for (auto& j : sb) {
          SweepJob* r = (SweepJob*)j.data();
          r->ntiles = sweep_groups(r->nlines, L.w);
        }
      std::vector<char> jobs;
      int n = 0, total = 0;
      for (std::vector<char>& j : sb) {
        // every job struct has its own tiling fields: patch tile0
        if (L.kind == Launch::SWEEP) {
          SweepJob* r = (SweepJob*)j.data();
          r->tile0 = total;
          total += r->ntiles;
        } else if (L.kind == Launch::KRON) {
          KronJob* r = (KronJob*)j.data();
          r->tile0 = total;
          total += r->ntiles;
        } else if (L.kind == Launch::PLANE) {
          PlaneJob* r = (PlaneJob*)j.data();
          r->tile0 = total;
          total += r->ntiles;
        } else {
          RhsJob* r = (RhsJob*)j.data();
          r->tile0 = total;
          total += r->ntiles;
        }
        jobs.insert(jobs.end(), j.begin(), j.end());
        ++n;
      }
      LaunchHdr h{};
      h.njobs = n;
      h.total_tiles = total;
      // launch shape (a captured graph holds it): sweep tile width, in-plane
      // LDS size, and the largest degree (instantiation and factor rows)
      P->nonempty[li * kPoolBranches + b] = n == 0 ? 0 : shape;
      char* dst = P->h_tab.data() + L.off + b * L.boff;
      std::memcpy(dst, &h, sizeof(h));
      if (!jobs.empty()) std::memcpy(dst + sizeof(LaunchHdr), jobs.data(), jobs.size());
    }
  }
  for (size_t i = 0; i < P->slots.size(); ++i) {
    const ads_pool::Slot& sl = P->slots[i];
    if (sl.active && taken[i] != (int)sl.sim->step_l.size()) {
      P->dirty = true;
      return fail(ADS_EINVAL, "pool slot " + std::to_string(i) + ": " + std::to_string(sl.sim->step_l.size() - taken[i]) +
                                  " of its launches match no launch class of the pool");
    }
  }
  HIPCHECK(hipMemcpyAsync(P->d_tab, P->h_tab.data(), P->tab_bytes, hipMemcpyHostToDevice, P->stream));
  HIPCHECK(hipStreamSynchronize(P->stream));
  P->dirty = false;
  return ADS_OK;
}

// True when launch class li has jobs in some branch.
bool class_used(const ads_pool* P, size_t li) {
  for (int b = 0; b < kPoolBranches; ++b)
    if (P->nonempty[li * kPoolBranches + b]) return true;
  return false;
}

// One pool step of branch b on stream s: the branch's launch of every
// non-empty class, in class order (with per-launch events when profiling,
// where the tables hold one branch).
ads_status pool_enqueue(ads_pool* P, int b, hipStream_t s, hipEvent_t* evs = nullptr) {
  if (evs) HIPCHECK(hipEventRecord(evs[0], s));
  for (size_t li = 0; li < P->seq.size(); ++li) {
    const PoolLaunch& L = P->seq[li];
    if (P->nonempty[li * kPoolBranches + b]) {
      const LaunchHdr* h = (const LaunchHdr*)(P->d_tab + L.off + b * L.boff);
      hipError_t e = hipSuccess;
      switch (L.kind) {
        case Launch::RHS_P: e = launch_rhs_pwave(L.p, L.mixed, L.var, L.coef, h, L.grid, s); break;
        case Launch::RHS_E: e = launch_rhs_elastic_band(L.p, L.mixed, h, L.grid, s); break;
        case Launch::SWEEP: e = launch_sweeps(h, L.grid, L.w, kPoolMaxM, L.p, s); break;
        case Launch::KRON: e = launch_kron(h, L.grid, L.p, s); break;
        case Launch::PLANE: e = launch_planes(h, L.grid, L.lds, L.p, L.coupled, s); break;
      }
      if (e != hipSuccess) return fail(ADS_EDEVICE, std::string("pool launch: ") + hipGetErrorString(e));
    }
    // every class closes its interval (empty ones with no launch)
    if (evs) HIPCHECK(hipEventRecord(evs[li + 1], s));
  }
  return ADS_OK;
}

// True when branch 1 has any launch.
bool second_branch(const ads_pool* P) {
  for (size_t li = 0; li < P->seq.size(); ++li)
    if (P->nonempty[li * kPoolBranches + 1]) return true;
  return false;
}

}  // namespace

extern "C" {

ads_status ads_pool_create(void* ws, size_t bytes, int32_t max_slots, void* stream, int32_t use_graph,
                           ads_pool** out) {
  if (!ws || !out) return fail(ADS_EINVAL, "NULL argument");
  if (((uintptr_t)ws) % kAlign) return fail(ADS_EINVAL, "workspace must be 256-byte aligned");
  if (max_slots < 1 || max_slots > 256) return fail(ADS_EINVAL, "max_slots must be in [1, 256]");
  if (use_graph && !stream) return fail(ADS_EINVAL, "graph replay needs a non-default stream");
  HIPCHECK(set_attributes_once());
  int dev = 0, ncu = 0;
  HIPCHECK(hipGetDevice(&dev));
  HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  ads_pool* P = new ads_pool();
  P->stream = (hipStream_t)stream;
  P->ws = (char*)ws;
  P->bytes = bytes;
  P->max_slots = max_slots;
  P->use_graph = use_graph != 0;
  P->slots.resize(max_slots);
  for (auto& a : P->var)
    for (auto& b : a) {
      b[0] = 3;   // no wave-speed field: the Kronecker form
      b[1] = 0;   // with one: the quadrature's first tile variant
    }
  P->ncu = ncu;
  if (hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming) != hipSuccess) {
    delete P;
    return fail(ADS_EDEVICE, "pool side stream or events");
  }
  pool_build_seq(P, ncu);
  P->arena_off = (P->tab_bytes + kAlign - 1) / kAlign * kAlign;
  if (P->arena_off >= bytes) {
    delete P;
    return fail(ADS_ENOMEM, "pool workspace smaller than its job tables");
  }
  P->d_tab = P->ws;
  P->h_tab.assign(P->tab_bytes, 0);
  ads_status st = pool_rebuild(P);
  if (st != ADS_OK) {
    delete P;
    return st;
  }
  *out = P;
  return ADS_OK;
}

ads_status ads_pool_admit(ads_pool* P, const ads_params* prm, const double* dev_u0, const double* dev_v0,
                          int32_t* slot) {
  if (!P || !prm || !slot) return fail(ADS_EINVAL, "NULL argument");
  std::string why;
  if (!valid_params(prm, why)) return fail(ADS_EINVAL, why);
  for (int d = 0; d < 3; ++d)
    if (free_count(*prm, d) > kPoolMaxM) return fail(ADS_EINVAL, "pooled meshes: <= 128 free coefficients");
  if (prm->precision == ADS_MIXED_BF16)
    return fail(ADS_EINVAL, "ADS_MIXED_BF16 (two right-hand-side passes) is not pooled");
  if (prm->nquad != 0 && prm->nquad != prm->p + 1)
    return fail(ADS_EINVAL, "pooled simulations use q = p+1 Gauss points");
  int free_slot = -1;
  for (int i = 0; i < P->max_slots; ++i)
    if (!P->slots[i].sim) {
      free_slot = i;
      break;
    }
  if (free_slot < 0) return fail(ADS_ENOMEM, "no free slot");
  size_t need = 0;
  ads_workspace_bytes(prm, &need);
  need = (need + kAlign - 1) / kAlign * kAlign;
  // first fit over the gaps between allocated blocks
  size_t cur = P->arena_off, found = (size_t)-1;
  for (auto& kv : P->used) {
    if (kv.first >= cur + need) {
      found = cur;
      break;
    }
    cur = std::max(cur, kv.first + kv.second);
  }
  if (found == (size_t)-1 && cur + need <= P->bytes) found = cur;
  if (found == (size_t)-1) return fail(ADS_ENOMEM, "not enough free pool memory");
  ads_sim* s = nullptr;
  // elasticity takes the Kronecker form in every pool
  g_force_var = (prm->problem == ADS_ELASTIC || !quadrature_ok(prm->p))
                    ? 3 : P->var[prm->p - 1][prm->precision == ADS_MIXED_FP32 ? 1 : 0][0];
  ads_status st = ads_create(prm, P->ws + found, need, P->stream, dev_u0, dev_v0, &s);
  g_force_var = -1;
  if (st != ADS_OK) return st;
  s->pooled = true;
  s->pool_dirty = &P->dirty;
  P->used[found] = need;
  P->slots[free_slot] = ads_pool::Slot{s, found, need, false};
  *slot = free_slot;
  return ADS_OK;
}

ads_status ads_pool_sim(ads_pool* P, int32_t slot, ads_sim** sim) {
  if (!P || !sim || slot < 0 || slot >= P->max_slots || !P->slots[slot].sim) return fail(ADS_EINVAL, "bad slot");
  *sim = P->slots[slot].sim;
  return ADS_OK;
}

ads_status ads_pool_activate(ads_pool* P, int32_t slot) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].sim) return fail(ADS_EINVAL, "bad slot");
  ads_sim* s = P->slots[slot].sim;
  if (!s->factored || s->need_start) return fail(ADS_ESTATE, "activate before ads_factor");
  P->slots[slot].active = true;
  P->dirty = true;
  return ADS_OK;
}

ads_status ads_pool_step(ads_pool* P, int32_t nsteps) {
  if (!P || nsteps < 0) return fail(ADS_EINVAL, "bad argument");
  ads_status st;
  // the active simulations' stepping fields w, b (a state set since the
  // last step), then their u and u' are formed from (w, b, a) when read
  for (int i = 0; i < P->max_slots; ++i) {
    ads_sim* s = P->slots[i].sim;
    if (!s || !P->slots[i].active) continue;
    if ((st = sync_predictor(s)) != ADS_OK) return st;
    if (nsteps > 0 && !s->elastic) s->u_stale = true;
  }
  // profiled steps time every launch class over the whole batch: one branch
  const int nb = P->prof ? 1 : P->want_branches;
  if (nb != P->nbranch) {
    P->nbranch = nb;
    P->dirty = true;
  }
  if (P->dirty && (st = pool_rebuild(P)) != ADS_OK) return st;
  const bool two = second_branch(P);
  // the graphs hold the non-empty launch classes of each branch; re-capture
  // only when that set changes (tables alone change between replays)
  if ((P->exec || P->exec2) && P->captured != P->nonempty) {
    HIPCHECK(hipStreamSynchronize(P->stream));
    HIPCHECK(hipStreamSynchronize(P->side));
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->exec2) (void)hipGraphExecDestroy(P->exec2);
    if (P->graph2) (void)hipGraphDestroy(P->graph2);
    P->exec = P->exec2 = nullptr;
    P->graph = P->graph2 = nullptr;
  }
  auto capture = [&](int b, hipStream_t s, hipGraph_t* g, hipGraphExec_t* x) -> ads_status {
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ads_status cs = pool_enqueue(P, b, s);
    hipGraph_t gg = nullptr;
    hipError_t e = hipStreamEndCapture(s, &gg);
    if (cs != ADS_OK) return cs;
    if (e != hipSuccess) return fail(ADS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    *g = gg;
    HIPCHECK(hipGraphInstantiate(x, gg, nullptr, nullptr, 0));
    return ADS_OK;
  };
  if (P->use_graph && !P->prof && !P->exec) {
    P->captured = P->nonempty;
    if ((st = capture(0, P->stream, &P->graph, &P->exec)) != ADS_OK) return st;
    if (two && (st = capture(1, P->side, &P->graph2, &P->exec2)) != ADS_OK) return st;
  }
  // two branches: the side stream starts after the pool stream's earlier
  // work and runs its steps beside the pool stream's; it is joined back
  // before the last step's event, so that the call's steps are complete on
  // the pool stream (stream-ordered reads of any simulation see them)
  if (two && nsteps > 0) {
    HIPCHECK(hipEventRecord(P->fork_ev, P->stream));
    HIPCHECK(hipStreamWaitEvent(P->side, P->fork_ev, 0));
  }
  for (int k = 0; k < nsteps; ++k) {
    if (P->nev == 0) {
      if (P->ev.empty()) {
        hipEvent_t e0;
        HIPCHECK(hipEventCreate(&e0));
        P->ev.push_back(e0);
      }
      HIPCHECK(hipEventRecord(P->ev[0], P->stream));
      P->nev = 1;
    }
    if (P->prof) {
      const size_t per = P->seq.size() + 1;
      while (P->pev.size() < (size_t)(P->prof_steps + 1) * per) {
        hipEvent_t e;
        HIPCHECK(hipEventCreate(&e));
        P->pev.push_back(e);
      }
      if ((st = pool_enqueue(P, 0, P->stream, &P->pev[(size_t)P->prof_steps * per])) != ADS_OK) return st;
      P->prof_steps++;
    } else if (P->use_graph) {
      HIPCHECK(hipGraphLaunch(P->exec, P->stream));
      if (two) HIPCHECK(hipGraphLaunch(P->exec2, P->side));
    } else {
      if ((st = pool_enqueue(P, 0, P->stream)) != ADS_OK) return st;
      if (two && (st = pool_enqueue(P, 1, P->side)) != ADS_OK) return st;
    }
    if (two && k == nsteps - 1) {
      HIPCHECK(hipEventRecord(P->join_ev, P->side));
      HIPCHECK(hipStreamWaitEvent(P->stream, P->join_ev, 0));
    }
    // step times are kept for at most kStepEventCap steps between reads
    if (P->nev > kStepEventCap) continue;
    if ((int)P->ev.size() <= P->nev) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e));
      P->ev.push_back(e);
    }
    HIPCHECK(hipEventRecord(P->ev[P->nev], P->stream));
    P->nev++;
  }
  return ADS_OK;
}

ads_status ads_pool_tune(ads_pool* P, int32_t* nchanged, int32_t* host_shape, int32_t cap) {
  if (!P || !nchanged) return fail(ADS_EINVAL, "NULL argument");
  ads_status st;
  if (P->dirty && (st = pool_rebuild(P)) != ADS_OK) return st;
  *nchanged = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  // mean ms of `reps` back-to-back launches after one warm-up launch
  auto timed = [&](auto&& launch, double* ms) -> ads_status {
    if (launch() != hipSuccess) return fail(ADS_EDEVICE, "tuner launch failed");
    HIPCHECK(hipEventRecord(e0, P->stream));
    const int reps = 5;
    for (int r = 0; r < reps; ++r)
      if (launch() != hipSuccess) return fail(ADS_EDEVICE, "tuner launch failed");
    HIPCHECK(hipEventRecord(e1, P->stream));
    HIPCHECK(hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHECK(hipEventElapsedTime(&f, e0, e1));
    *ms = f / reps;
    return ADS_OK;
  };
  // the class's gathered jobs of branch tb (header + table in the host
  // copy): a launch is timed alone on the table of its first non-empty
  // branch, the launch a step runs
  size_t tb = 0;
  auto table = [&](const PoolLaunch& L) { return L.off + tb * L.boff; };
  auto jobs_of = [&](const PoolLaunch& L, auto* tag) {
    using J = std::remove_pointer_t<decltype(tag)>;
    LaunchHdr h;
    std::memcpy(&h, P->h_tab.data() + table(L), sizeof(h));
    std::vector<J> v(h.njobs);
    if (h.njobs) std::memcpy(v.data(), P->h_tab.data() + table(L) + sizeof(LaunchHdr), h.njobs * sizeof(J));
    return v;
  };
  for (size_t li = 0; li < P->seq.size(); ++li) {
    if (!class_used(P, li)) continue;
    tb = P->nonempty[li * kPoolBranches] ? 0 : 1;
    PoolLaunch& L = P->seq[li];
    if (L.kind == Launch::RHS_P && quadrature_ok(L.p)) {
      // right-hand side: quadrature tile variants (and the Kronecker form
      // without a wave-speed field), timed on the batch's own jobs (they
      // write only the right-hand-side buffers)
      std::vector<std::string> shp;
      for (const RhsJob& j : jobs_of(L, (RhsJob*)nullptr))
        shp.push_back(std::to_string(j.nf[0]) + "x" + std::to_string(j.nf[1]) + "x" + std::to_string(j.nf[2]));
      std::sort(shp.begin(), shp.end());
      std::string key = "R" + std::to_string(li);
      for (const std::string& x : shp) key += "/" + x;
      int& cur = P->var[L.p - 1][L.mixed][L.coef];
      const int before = cur;
      auto it = P->tune_cache.find(key);
      int best = before;
      if (it != P->tune_cache.end()) {
        best = it->second;
      } else {
        double best_ms = 1e30;
        for (int v = 0; v <= 4; ++v) {
          if (!rhs_variant_exists(L.p, L.mixed, v, L.coef)) continue;
          cur = v;
          L.var = v;
          L.grid = rhs_blocks_per_cu(L.p, L.mixed, v, L.coef) * P->ncu;
          if ((st = pool_rebuild(P)) != ADS_OK) return st;
          const LaunchHdr* h = (const LaunchHdr*)(P->d_tab + table(L));
          double ms = 0.0;
          if ((st = timed([&] { return launch_rhs_pwave(L.p, L.mixed, L.var, L.coef, h, L.grid, P->stream); },
                          &ms)) != ADS_OK)
            return st;
          if (ms < best_ms) {
            best_ms = ms;
            best = v;
          }
        }
        P->tune_cache[key] = best;
      }
      cur = best;
      L.var = best;
      L.grid = rhs_blocks_per_cu(L.p, L.mixed, best, L.coef) * P->ncu;
      if (best != before) ++*nchanged;
      if ((st = pool_rebuild(P)) != ADS_OK) return st;
    } else if (L.kind == Launch::SWEEP) {
      // sweeps: tile widths, timed on a copy of the batch's table whose jobs
      // solve in place with the plain store epilogue (no time update, no
      // step counter): only the step's temporaries are touched
      long long lines = 0;
      for (const SweepJob& j : jobs_of(L, (SweepJob*)nullptr)) lines += j.nlines;
      const std::string key = "S" + std::to_string(li) + "/" + std::to_string(lines) + "/" + std::to_string(L.p);
      const int before = L.w;
      auto it = P->tune_cache.find(key);
      int best = before;
      if (it != P->tune_cache.end()) {
        best = it->second;
      } else {
        double best_ms = 1e30;
        for (int W : {4, 8, 16}) {
          if (!sweep_width_fits(W, kPoolMaxM, L.p)) continue;
          P->w_force[li] = W;
          if ((st = pool_rebuild(P)) != ADS_OK) return st;
          std::vector<SweepJob> js = jobs_of(L, (SweepJob*)nullptr);
          for (SweepJob& j : js) {
            j.epi = EPI_STORE;
            j.out = const_cast<double*>(j.in);
            j.counter = nullptr;
          }
          LaunchHdr th{};
          std::memcpy(&th, P->h_tab.data() + table(L), sizeof(th));
          std::vector<char> buf(sizeof(LaunchHdr) + js.size() * sizeof(SweepJob));
          std::memcpy(buf.data(), &th, sizeof(th));
          std::memcpy(buf.data() + sizeof(LaunchHdr), js.data(), js.size() * sizeof(SweepJob));
          HIPCHECK(hipMemcpyAsync(P->d_tab + P->tune_off, buf.data(), buf.size(), hipMemcpyHostToDevice, P->stream));
          const LaunchHdr* h = (const LaunchHdr*)(P->d_tab + P->tune_off);
          double ms = 0.0;
          if ((st = timed([&] { return launch_sweeps(h, L.grid, L.w, kPoolMaxM, L.p, P->stream); }, &ms)) != ADS_OK)
            return st;
          if (ms < best_ms) {
            best_ms = ms;
            best = W;
          }
        }
        P->tune_cache[key] = best;
      }
      P->w_force[li] = best;
      if (best != before) ++*nchanged;
      if ((st = pool_rebuild(P)) != ADS_OK) return st;
    }
  }
  // elasticity couplings: separate launches or in the in-plane sweeps,
  // timed over the batch's coupling and in-plane classes in both branches
  // (they write only the step's temporaries); planes of every simulation
  // share the in-plane launches, so the form can pay in a batch where it
  // does not for one simulation
  {
    std::vector<std::string> shp;
    for (const ads_pool::Slot& sl : P->slots)
      if (sl.active && sl.sim->elastic && plane_couple_fits(sl.sim->nf[0], sl.sim->nf[1], sl.sim->p))
        shp.push_back(std::to_string(sl.sim->p) + ":" + std::to_string(sl.sim->nf[0]) + "x" +
                      std::to_string(sl.sim->nf[1]) + "x" + std::to_string(sl.sim->nf[2]));
    if (!shp.empty()) {
      std::sort(shp.begin(), shp.end());
      std::string key = "C";
      for (const std::string& x : shp) key += "/" + x;
      const bool before = P->couple_fused;
      int best = before ? 1 : 0;
      auto it = P->tune_cache.find(key);
      if (it != P->tune_cache.end()) {
        best = it->second;
      } else {
        double ms[2] = {0.0, 0.0};
        for (int f = 0; f < 2; ++f) {
          P->couple_fused = f != 0;
          if ((st = pool_rebuild(P)) != ADS_OK) return st;
          auto go = [&]() -> hipError_t {
            for (size_t li = 0; li < P->seq.size(); ++li) {
              const PoolLaunch& L = P->seq[li];
              if (L.kind != Launch::KRON && L.kind != Launch::PLANE) continue;
              for (int b = 0; b < kPoolBranches; ++b) {
                if (!P->nonempty[li * kPoolBranches + b]) continue;
                const LaunchHdr* h = (const LaunchHdr*)(P->d_tab + L.off + b * L.boff);
                const hipError_t e = L.kind == Launch::KRON ? launch_kron(h, L.grid, L.p, P->stream)
                                                            : launch_planes(h, L.grid, L.lds, L.p, L.coupled, P->stream);
                if (e != hipSuccess) return e;
              }
            }
            return hipSuccess;
          };
          if ((st = timed(go, &ms[f])) != ADS_OK) return st;
        }
        best = ms[1] < ms[0] ? 1 : 0;
        P->tune_cache[key] = best;
      }
      P->couple_fused = best != 0;
      if (P->couple_fused != before) ++*nchanged;
      if ((st = pool_rebuild(P)) != ADS_OK) return st;
    }
  }
  HIPCHECK(hipStreamSynchronize(P->stream));
  if (host_shape)
    for (size_t li = 0; li < P->seq.size() && (int)li < cap; ++li) {
      const PoolLaunch& L = P->seq[li];
      host_shape[li] = !class_used(P, li) ? -1
                       : (L.kind == Launch::RHS_P || L.kind == Launch::RHS_E) ? L.var
                       : L.kind == Launch::SWEEP ? L.w : 0;
    }
  return ADS_OK;
}

ads_status ads_pool_profile(ads_pool* P, int32_t enable) {
  if (!P) return fail(ADS_EINVAL, "NULL pool");
  P->prof = enable != 0;
  P->prof_steps = 0;
  return ADS_OK;
}

ads_status ads_pool_set_branches(ads_pool* P, int32_t n) {
  if (!P) return fail(ADS_EINVAL, "NULL pool");
  if (n < 1 || n > kPoolBranches) return fail(ADS_EINVAL, "branches must be 1 or 2");
  P->want_branches = n;
  return ADS_OK;
}

ads_status ads_pool_profile_read(ads_pool* P, double* ms, int32_t* kind, int32_t* pp, int32_t* mixed, int32_t cap,
                                 int32_t* nlaunch) {
  if (!P) return fail(ADS_EINVAL, "NULL pool");
  HIPCHECK(hipStreamSynchronize(P->stream));
  const size_t L = P->seq.size(), per = L + 1;
  for (size_t i = 0; i < L && (int)i < cap; ++i) {
    double sum = 0.0;
    for (int k = 0; k < P->prof_steps; ++k) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, P->pev[k * per + i], P->pev[k * per + i + 1]));
      sum += t;
    }
    const PoolLaunch& l = P->seq[i];
    if (ms) ms[i] = !class_used(P, i) ? -1.0 : (P->prof_steps ? sum / P->prof_steps : 0.0);
    if (kind) {
      // 0 / 5 right-hand sides, 6 in-plane sweeps, 3 z-sweeps, 4 couplings
      kind[i] = l.kind == Launch::RHS_P ? 0 : l.kind == Launch::RHS_E ? 5 : l.kind == Launch::KRON ? 4
                : l.kind == Launch::PLANE ? 6 : 3;
    }
    if (pp) pp[i] = l.p;
    if (mixed) mixed[i] = l.mixed;
  }
  if (nlaunch) *nlaunch = (int32_t)L;
  P->prof_steps = 0;
  return ADS_OK;
}

ads_status ads_pool_retire(ads_pool* P, int32_t slot, double* dev_u, double* dev_v, double* dev_a) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].sim) return fail(ADS_EINVAL, "bad slot");
  ads_pool::Slot& sl = P->slots[slot];
  // the final state, copied out on the pool's stream before the memory is
  // released (later admissions reuse it in stream order)
  if (dev_u || dev_v || dev_a) {
    ads_status st = ads_get_state(sl.sim, dev_u, dev_v, dev_a);
    if (st != ADS_OK) return st;
  }
  delete sl.sim;
  P->used.erase(sl.off);
  if (sl.active) P->dirty = true;
  sl = ads_pool::Slot{};
  return ADS_OK;
}

ads_status ads_pool_step_times(ads_pool* P, double* ms, int32_t cap, int32_t* n) {
  if (!P || !n) return fail(ADS_EINVAL, "NULL argument");
  HIPCHECK(hipStreamSynchronize(P->stream));
  int cnt = 0;
  for (int k = 1; k < P->nev; ++k) {
    float t = 0.f;
    HIPCHECK(hipEventElapsedTime(&t, P->ev[k - 1], P->ev[k]));
    if (ms && cnt < cap) ms[cnt] = t;
    ++cnt;
  }
  *n = std::min(cnt, cap);
  P->nev = 0;
  return ADS_OK;
}

ads_status ads_pool_info(ads_pool* P, int32_t* active, size_t* used_bytes, size_t* free_bytes) {
  if (!P) return fail(ADS_EINVAL, "NULL pool");
  int a = 0;
  for (auto& s : P->slots) a += s.active ? 1 : 0;
  size_t u = 0;
  for (auto& kv : P->used) u += kv.second;
  if (active) *active = a;
  if (used_bytes) *used_bytes = u;
  if (free_bytes) *free_bytes = P->bytes - P->arena_off - u;
  return ADS_OK;
}

ads_status ads_pool_destroy(ads_pool* P) {
  if (!P) return fail(ADS_EINVAL, "NULL pool");
  delete P;
  return ADS_OK;
}

}  // extern "C"
