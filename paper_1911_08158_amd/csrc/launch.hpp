// Kernel launchers (defined in the k_*.hip translation units).
#pragma once

#include "common.hpp"

namespace ads {

// Launchers take the device header of a job table (LaunchHdr followed by
// the jobs) and a grid size (all tiles, or a persistent grid that loops).
// Sweeps: a workgroup takes groups of 4W lines (one W-line tile per wave);
// job tile counts are in groups.
// pmax: the largest spline degree among the launch's jobs (1..5).
int sweep_width_for(long long lines, int max_m, int ncu, int pmax);
bool sweep_width_fits(int W, int max_m, int pmax);
int sweep_groups(long long lines, int W);
int sweep_blocks_per_cu(int W, int max_m, int pmax);
hipError_t launch_sweeps(const LaunchHdr* d_hdr, int grid, int W, int max_m, int pmax, hipStream_t s);
hipError_t sweep_set_attributes();
// In-plane sweeps: one workgroup per z-plane (PlaneJob tiles are planes);
// a plane of nx x ny unknowns fits when plane_lds_bytes <= 160 KiB.
size_t plane_lds_bytes(int nx, int ny, int p);
bool plane_fits(int nx, int ny, int p);
// ... with coupling terms (PlaneJob::nterm > 0): the LDS, and whether a
// plane takes them (at most 4,608 unknowns, and the LDS fits).
size_t plane_lds_bytes(int nx, int ny, int p, bool coupled);
bool plane_couple_fits(int nx, int ny, int p);
// coupled: the launch holds jobs with coupling terms.
int plane_blocks_per_cu(size_t lds_bytes, int pmax, bool coupled);
hipError_t launch_planes(const LaunchHdr* d_hdr, int grid, size_t lds_bytes, int pmax, bool coupled, hipStream_t s);

// P-wave right-hand side: variants 0-2 are tile shapes of the quadrature
// kernel; variant 3 is the Kronecker (assembled band) form, for jobs
// without a wave-speed field only.  coef: the jobs carry a wave-speed
// field (RhsJob::coef).
bool rhs_variant_exists(int p, int mixed, int var, int coef);
int rhs_tile_x(int p, int var);
int rhs_tile_y(int p, int mixed, int var);
int rhs_blocks_per_cu(int p, int mixed, int var, int coef);
hipError_t launch_rhs_pwave(int p, int mixed, int var, int coef, const LaunchHdr* d_hdr, int grid, hipStream_t s);
int rhs_band_tile_x();
int rhs_band_tile_y();
int rhs_band_blocks_per_cu(int p, int mixed);
hipError_t launch_rhs_band(int p, int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s);
int rhs_el_tile_x(int p);
int rhs_el_tile_y(int p);
hipError_t launch_rhs_elastic(int p, const LaunchHdr* d_hdr, int grid, hipStream_t s);
// Elasticity right-hand side in the Kronecker form (band passes; FP64, or
// FP32 stiffness-type passes with mixed = 1)
int rhs_el_band_tile_x();
int rhs_el_band_tile_y(int p);
int rhs_el_band_blocks_per_cu(int p, int mixed);
hipError_t launch_rhs_elastic_band(int p, int mixed, const LaunchHdr* d_hdr, int grid, hipStream_t s);

hipError_t launch_kron(const LaunchHdr* d_hdr, int grid, int pmax, hipStream_t s);
hipError_t kron_set_attributes();
int kron_tile_x();
int kron_tile_y();
int kron_blocks_per_cu(int pmax);

hipError_t launch_full_to_free(const double* full, double* fr, const int n[3], const int nf[3],
                               const int off[3], int ncomp, hipStream_t s);
hipError_t launch_free_to_full(const double* fr, double* full, const int n[3], const int nf[3],
                               const int off[3], int ncomp, hipStream_t s);
hipError_t launch_proj_contract(const double* in, double* out, long long outer, int E, int q, int P, int nf,
                                int off, long long inner, const double* tab, hipStream_t s);
hipError_t launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s);
hipError_t launch_fill(double* p, long long n, double v, hipStream_t s);
hipError_t launch_axpby(double* out, const double* x, const double* y, double a, double b, long long n,
                        hipStream_t s);
hipError_t launch_lin3(double* out, const double* x, const double* y, const double* z, double b, double c,
                       long long n, hipStream_t s);
hipError_t launch_nonfinite(const double* x, long long n, unsigned long long* cnt, hipStream_t s);
// out = x . y (deterministic two-pass reduction through dot_scratch_doubles() partial sums)
int dot_scratch_doubles();
hipError_t launch_dot(const double* x, const double* y, long long n, double* partial, double* out, hipStream_t s);

}  // namespace ads
