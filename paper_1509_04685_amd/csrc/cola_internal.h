// Internal declarations of libcola: host-side cosmology, mesh geometry, FFT plans and kernel
// launchers.  Not part of the public C ABI (include/cola.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cola.h"
#include "fft_core.h"

namespace cola {

// Records the failing call and HIP error for cola_last_error; returns COLA_ERR_HIP.
int hip_fail(hipError_t e, const char* what);

// Force cache of a workspace (api.cpp): forget whatever force the workspace held (every call that
// writes a workspace), record that it holds the force of state P at node `node` corrected by the
// network with parameter array `net` (nullptr: plain), and ask whether it holds that force.
void ws_forget(const void* ws);
void ws_record(const void* ws, const cola_particles* P, int node, const void* net);
bool ws_holds(const void* ws, const cola_particles* P, int node, const void* net, bool any_net);

// ------------------------------------------------------------------ profiler (profiler.cpp)
enum ProfKind {
    PROF_FILL = 0, PROF_DEPOSIT, PROF_Z_R2C, PROF_Y_FWD, PROF_X_FWD, PROF_X_GREEN, PROF_Y_SPLIT,
    PROF_Y_INV, PROF_Z_C2R, PROF_GKD, PROF_GATHER, PROF_IC, PROF_X_INV_MULT, PROF_PK, PROF_COPY,
    PROF_OTHER, PROF_KICK, PROF_PK_DEPOSIT, PROF_DEP_SORT, PROF_DEP_TILE, PROF_LC_CONV, PROF_LC_WGRAD, PROF_LC_MISC,
    PROF_FOF, PROF_PK_ALIAS, PROF_Z_C2R3,
    PROF_NUM_KINDS
};
// Brackets one kernel launch with an event pair when the profiler is enabled.  tag: a size label
// (the mesh side for FFT passes) so that reads can separate launches of different sizes.
class ProfScope {
  public:
    ProfScope(int kind, hipStream_t st, long tag = 0);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    int kind_;
    long tag_;
    hipStream_t st_;
    hipEvent_t start_ = nullptr;
    bool counted_ = false;
};

// ------------------------------------------------------------------ cosmology (float64, host)
struct Growth {
    double d1, d2, dd1_da, dd2_da;
};
double hubble_e(double a, double om);
Growth growth(double a, double om);
double kick_integral(double a0, double a1, double om);
double drift_integral(double a0, double a1, double om);
std::vector<double> time_nodes(const cola_problem& p);
double bbks_gamma(const cola_cosmology& c);
double bbks_transfer(double k, double gamma);
double linear_amplitude(const cola_cosmology& c);

struct Schedule {
    double omega_m;
    std::vector<double> a, d1, d2;          // per node
    std::vector<double> k_out, k_in, drift;  // per interval j -> j+1
};
Schedule make_schedule(const cola_problem& p, const cola_cosmology& c);

// ------------------------------------------------------------------ mesh geometry
// A cubic mesh of n cells per side.  A workspace buffer of total_c() float2 holds either a real
// field [x][y][z] with rows of 2 nzp floats (nzp >= n/2 + 1 rounded up to 16: rows start on
// 128-byte boundaries) or the transposed half spectrum [kz][x][y], kz planes of n^2 values `plane`
// float2 apart.
struct Mesh3 {
    int n = 0;
    int m = 0;     // n / 2
    int nzp = 0;   // padded complex row length of the real layout
    long plane = 0;  // float2 between kz planes of the transposed spectrum (n^2 plus a pad)
    long row_c() const { return nzp; }
    long total_c() const {
        const long real = (long)n * n * nzp, spec = (long)(m + 1) * plane;
        return real > spec ? real : spec;
    }
    size_t bytes() const { return (size_t)total_c() * sizeof(float2); }
};
Mesh3 make_mesh(int n);
bool fft_size_ok(int n);  // even, >= 4, factors 2 and 3 only
FftPlan make_plan(int n, bool reverse = false);
FftPlan make_plan_r(int n, int R, bool reverse);
// Times the admissible shapes of every FFT kernel at mesh size n on scratch buffers S, A, B
// (overwritten; A differs from S and B) and keeps the fastest for the process.
hipError_t autotune_fft(int n, float2* S, float2* A, float2* B, const float2* tw, hipStream_t st,
                        std::string* report);

// Pins the kernel shape of one pass kind ("z_r2c", "z_c2r", "cols_y", "cols_x", "x_green",
// "y_split", "x_mult") at mesh size n for the rest of the process; a cola_status.
int set_fft_shape(int n, const char* kind, int R, int width, int stat);

// ------------------------------------------------------------------ launchers (fft.hip)
hipError_t launch_twiddles(float2* tw, int len, hipStream_t st);

// Forward 3D r2c: real rows at `in` (in_row floats apart, batch stride in_bstride floats) with
// y = pa * x + pb applied on load -> transposed half spectrum `out` (batch stride out_bstride
// float2), out of place (the z pass transposes).  z, then y, then x.
hipError_t fft3d_r2c(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                     const Mesh3& g, const float2* tw, int n_real, float pa, float pb, hipStream_t st);

// Radial transfer of the Green's function (the learned form's filter): T(u) the cubic Hermite
// interpolant of the n knots (u[j], t[j]) with slopes m[j] (green_slopes), u = |m| / (N/2) for the
// signed mode integers m of an N^3 mesh, constant beyond the end knots.
struct GreenFilter {
    int n = 0;
    float u[10] = {};
    float t[10] = {};
    float m[10] = {};
    float u_last = 0.0f, t_last = 1.0f;
};
// The knot slopes of the transfer: 0 at the first knot, centred differences inside, one-sided at
// the last; knots past the n-th padded with u = 3e38 (never reached), the last knot copied out.
inline void green_slopes(GreenFilter& gf) {
    for (int j = 0; j < gf.n; ++j) {
        if (j == 0) gf.m[j] = 0.0f;
        else if (j == gf.n - 1) gf.m[j] = (gf.t[j] - gf.t[j - 1]) / (gf.u[j] - gf.u[j - 1]);
        else gf.m[j] = (gf.t[j + 1] - gf.t[j - 1]) / (gf.u[j + 1] - gf.u[j - 1]);
    }
    for (int j = gf.n; j < 10; ++j) {
        gf.u[j] = 3.0e38f;
        gf.t[j] = gf.t[gf.n - 1];
        gf.m[j] = 0.0f;
    }
    gf.u_last = gf.u[gf.n - 1];
    gf.t_last = gf.t[gf.n - 1];
}

// PM force from the y-transformed spectrum in P (z and y forward passes done), with Q, R free
// buffers of the same size (all distinct):
//   fused x (forward, Green 1/(k^2 n^3), inverse) -> P = G P, Q = i k_x G P;
//   y inverse: P -> P (times i k_y), R (plain);  Q -> Q;
//   one z c2r pass of Q (F_x), P (F_y) and R (times i k_z: F_z) writing the components
//   interleaved: F[(x n + y) frow + 3 z + c], c = 0, 1, 2 for x, y, z, z = 0 .. n + 1 (the ghost
//   cells z = n, n + 1 repeat z = 0, 1), frow = force_row3(n) floats per row (3 (n + 2) rounded
//   up to whole 128-byte lines), fstride floats between realizations.
// P, Q, R are overwritten; F must not overlap them.  gf (optional): the Green's function is
// multiplied by gf's T.
long force_row3(int n);
hipError_t pm_force_interleaved(float2* P, float2* Q, float2* R, float* F, long frow, long fstride, long bstride,
                                const Mesh3& g, const float2* tw, float kf, int n_real, hipStream_t st,
                                const GreenFilter* gf = nullptr);
// z r2c + y forward only (first half of the PM force transform), out of place
hipError_t fft_zy_forward(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                          const Mesh3& g, const float2* tw, int n_real, float pa, float pb,
                          hipStream_t st);

// Multiplier types for the inverse transforms of the initial conditions.
enum MulType { MUL_SCALE = 0, MUL_IK = 1, MUL_KK = 2 };
// Inverse 3D c2r of mult(k) * spec: spec is a full forward spectrum, work a scratch spectrum of
// the same size (may be spec itself), out real rows of out_row floats (not overlapping work).
hipError_t fft3d_c2r_mult(const float2* spec, long spec_bstride, float2* work, long work_bstride,
                          float* out, long out_row, long out_bstride, const Mesh3& g, const float2* tw,
                          int n_real, int mtype, int axis_a, int axis_b, float kf, float scale,
                          hipStream_t st);

// transposed spectrum <-> numpy rfftn layout [x][y][kz] copies
hipError_t copy_unpad_to_pad(const float2* src, float2* dst, const Mesh3& g, hipStream_t st);
hipError_t copy_pad_to_unpad(const float2* src, float2* dst, const Mesh3& g, hipStream_t st);

// ------------------------------------------------------------------ launchers (pm_kernels.hip)
struct ParticlePtrs {
    float* x[3];
    float* p[3];
    const float* psi1[3];
    const float* psi2[3];
};

// Geometry of a CIC mesh relative to the Lagrangian lattice.
struct LatticeGeom {
    int n_part;     // N_p
    int n_mesh;     // cells per side of this mesh
    float inv_h;    // n_mesh / L
    float qoff;     // lattice offset in this mesh's cells (0.5 * n_mesh / N_g)
    long row;       // floats per mesh row (force meshes: per row of interleaved (x, y, z) cells)
    long mesh_bstride;  // floats between realizations
};

struct KickDrift {
    float kick;     // (3/2) Omega_m K for this kick (0: no kick)
    float d1;       // D1 at the node of the force
    float d2m;      // D2 - D1^2 at that node
    float drift;    // Dr of the drift (0 with no drift)
    float dd1, dd2; // growth increments of the drift
    int los = -1;   // drift along this axis only (the redshift-space mapping); -1: every axis
};

hipError_t launch_fill(float* p, long n, float v, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
hipError_t launch_fill_d(double* p, long n, double v, hipStream_t st);
hipError_t cic_deposit_absolute(const float* const pos[3], long n, int n_mesh, float inv_h, long row,
                                float* mesh, hipStream_t st);
hipError_t density_finish(float* mesh, long row, int n_mesh, float scale, float offset, hipStream_t st);
// The gathers read the interleaved force mesh F of pm_force_interleaved (fgeom.row floats per
// row, fgeom.mesh_bstride between realizations).
hipError_t gather_kick_drift(const ParticlePtrs& P, long n_per_real, int n_real, const LatticeGeom& fgeom,
                             const float* F, const KickDrift& kd, hipStream_t st);
hipError_t gather_force(const ParticlePtrs& P, long n_per_real, int n_real, const LatticeGeom& fgeom,
                        const float* F, float* const acc[3], hipStream_t st);

// Exclusive scan of nkeys counts: start[k] = sum of count[0..k), start[nkeys] = total (the sum,
// known to the caller), cursor = start.  block_sums holds ceil(nkeys / 1024) entries.
hipError_t scan_counts(const uint32_t* count, uint32_t* start, uint32_t* cursor, uint32_t* block_sums, long nkeys,
                       uint32_t total, hipStream_t st);

// ------------------------------------------------------------------ tiled deposit (deposit_sorted.hip)
struct TileGeom {
    int n = 0;             // mesh cells per side
    int tx = 1, ty = 1, tz = 1;
    int ntx = 1, nty = 1, ntz = 1;
    int lx = 0, ly = 0, lz = 0;  // log2 of the tile sides (all powers of two)
    long ntiles = 0;
    long nkeys = 0;        // ntiles * 8 categories
};
struct SortBufs {
    uint32_t* keys = nullptr;     // per particle
    float4* recs = nullptr;       // per particle: (local cell bits, fx, fy, fz)
    float4* sorted = nullptr;     // records in key order
    uint32_t* count = nullptr;    // per key (per realization stride kstride)
    uint32_t* start = nullptr;    // exclusive prefix, nkeys + 1 entries
    uint32_t* cursor = nullptr;
    uint32_t* block_sums = nullptr;
    long kstride = 0;
    int nblocks = 0;
};
TileGeom make_tiles(int n, long n_particles);
size_t sort_bytes(long n_particles_per_real, const TileGeom& tg, int n_real);
SortBufs carve_sort(void* base, long npr, const TileGeom& tg, int n_real);
// CIC deposit of every particle (drifted on the fly when `drift`, with the force gathered from
// the interleaved force mesh F of geometry fg) onto a mesh of dg's geometry, written as
// delta = rho * scale + offset.
hipError_t sorted_deposit(const ParticlePtrs& P, long npr, int n_real, const LatticeGeom& dg, bool drift,
                          const LatticeGeom& fg, const float* F, const KickDrift& kd, const TileGeom& tg,
                          const SortBufs& sb, float* mesh, float scale, float offset, hipStream_t st);

// The step's gather, kick and drift (as gather_kick_drift with a drift) fused with the binning of
// the moved particles onto fg's mesh for the next force evaluation; sorted_deposit_binned then
// finishes that deposit (sort and tile passes).  F: the interleaved force mesh, with the ghost
// cells; dg: the geometry of the density mesh the particles are binned for.
hipError_t gather_kick_drift_bin(const ParticlePtrs& P, long npr, int n_real, const LatticeGeom& fg, const float* F,
                                 const LatticeGeom& dg, const KickDrift& kd, const TileGeom& tg, const SortBufs& sb,
                                 hipStream_t st);
hipError_t sorted_deposit_binned(long npr, int n_real, const LatticeGeom& dg, const TileGeom& tg, const SortBufs& sb,
                                 float* mesh, float scale, float offset, hipStream_t st);
// Rewrites the ghost cells (z = 0, 1 again at z = n, n + 1) of n_real interleaved force meshes with
// `row` floats per row, after something other than the z c2r pass changed the meshes.
hipError_t mesh_ghosts(float* F, long row, int n, long bstride, int n_real, hipStream_t st);

// The same deposit for absolute positions pos[3] (n floats each, wrapped into the mesh), one
// realization, onto a mesh of n_mesh cells per side with rows of `row` floats.
hipError_t sorted_deposit_absolute(const float* const pos[3], long n, int n_mesh, float inv_h, const TileGeom& tg,
                                   const SortBufs& sb, float* mesh, long row, float scale, float offset,
                                   hipStream_t st);

// ------------------------------------------------------------------ launchers (ic_kernels.hip)
hipError_t ic_noise(float* w, int n_part, const uint64_t* seeds_host, int n_real, long bstride,
                    hipStream_t st);
hipError_t ic_scale_spectrum(float2* spec, long bstride, const Mesh3& g, int n_real, float kf,
                             double amp, double gamma, double n_s, double norm, hipStream_t st);
// S = phi_xx phi_yy + phi_xx phi_zz + phi_yy phi_zz  (first call, mode 0) or S -= phi^2 (mode 1)
hipError_t lpt2_source(float* s, const float* a, const float* b, const float* c, long n, int mode,
                       hipStream_t st);
// x = d1 psi1 + d2 psi2, p = c1 psi1 + c2 psi2.
hipError_t ic_set_state(const ParticlePtrs& P, long n, float d1, float d2, float c1, float c2, hipStream_t st);

// ------------------------------------------------------------------ launchers (pk_kernels.hip)
hipError_t pk_bin(const float2* spec, long bstride, const Mesh3& g, int n_real, int n_bins,
                  double* ksum, double* psum, double* cnt, double kf, hipStream_t st);
// Multipoles ell = 0, 2, 4 about the axis los: sums of w |delta|^2 / W^2 L_ell(mu), mu = m_los / |m|.
hipError_t pk_bin_multipoles(const float2* spec, long bstride, const Mesh3& g, int n_real, int n_bins, int los,
                             double* ksum, double* p0, double* p2, double* p4, double* cnt, double kf,
                             hipStream_t st);
// P_ell = (2 ell + 1) sum_ell / cnt * pnorm, k_mean = ksum / cnt.
hipError_t pk_finish_multipoles(double* kmean, double* p0, double* p2, double* p4, const double* cnt, long n,
                                double pnorm, hipStream_t st);
hipError_t pk_finish(double* kmean, double* pk, double* cnt, long n, double pnorm, hipStream_t st);
// Jing (2005) aliasing correction (pk_kernels.hip): floats of scratch per realization that
// pk_alias_pass needs (the aliasing table of every mode class and the bin slopes)
long pk_alias_scratch_floats(int n, int n_bins);
// One iteration: slopes from the current estimate (k_mean, pk, n_modes final), the aliasing sum
// of every mode class for its bin's slope, then pk rebinned as |delta|^2 / C and finished.
// scratch: n_real * sstride floats, sstride >= pk_alias_scratch_floats.
hipError_t pk_alias_pass(const float2* spec, long bstride, const Mesh3& g, int n_real, int n_bins,
                         const double* k_mean, double* pk, const double* n_modes, double pnorm, double kf,
                         float* scratch, long sstride, hipStream_t st);

}  // namespace cola
