// C-ABI entry points of libcola: validation, workspace carving and the order of the passes.
// Every check runs on the host before the first launch, so error returns leave nothing queued.

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "cola_internal.h"
#include "lc_internal.h"

using namespace cola;

thread_local char g_last_error[512] = "";

namespace cola {
int hip_fail(hipError_t e, const char* what) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return COLA_ERR_HIP;
}

// Which force the meshes of a workspace hold: the state that owns it (its x[0] array), the node
// and the network that corrected it (its parameter array; nullptr for the plain mesh force).
// Every call that writes a workspace forgets its entry; the calls that leave a node's force
// behind record it.  A state's own (force_node, force_ws) fields can only veto a cached force,
// so a workspace shared between states, or overwritten by any other call, is never trusted.
namespace {
struct ForceTag {
    const void* owner;
    int node;
    const void* net;
};
std::mutex g_tag_mu;
std::unordered_map<const void*, ForceTag> g_tags;
}  // namespace

void ws_forget(const void* ws) {
    if (!ws) return;
    std::lock_guard<std::mutex> lock(g_tag_mu);
    g_tags.erase(ws);
}

void ws_record(const void* ws, const cola_particles* P, int node, const void* net) {
    std::lock_guard<std::mutex> lock(g_tag_mu);
    g_tags[ws] = ForceTag{P->x[0], node, net};
}

// any_net: accept the force of any network (or none) -- the caller only needs the force the
// state's own run used at that node.
bool ws_holds(const void* ws, const cola_particles* P, int node, const void* net, bool any_net) {
    if (!(P->force_node == node && P->force_ws == ws)) return false;
    std::lock_guard<std::mutex> lock(g_tag_mu);
    auto it = g_tags.find(ws);
    if (it == g_tags.end()) return false;
    const ForceTag& t = it->second;
    return t.owner == P->x[0] && t.node == node && (any_net || t.net == net);
}
}  // namespace cola

namespace {

constexpr int kMaxMesh = 1536;  // keeps per-realization mesh offsets below 2^31


#define COLA_TRY(expr)                                       \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(_e, #expr);    \
    } while (0)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace: three mesh buffers S, A, B (real fields or transposed spectra; the z passes are
// out of place), the interleaved force mesh F, two P(k) buffers K (the deposit) and K2 (its
// spectrum), the deposit's sort buffers and the twiddle tables.  After a force evaluation F holds
// (F_x, F_y, F_z) of every cell, interleaved (pm_force_interleaved).
struct Layout {
    Mesh3 g;   // force mesh, N_g
    Mesh3 gp;  // Lagrangian lattice, N_p
    Mesh3 gk;  // P(k) mesh (n = 0 when absent)
    long cstride = 0;  // float2 per realization in S, A, B
    long frow = 0;     // floats per row of F
    long fstride = 0;  // floats per realization in F
    long kstride = 0;  // float2 per realization in K, K2
    TileGeom tg;  // force-mesh tiles of the deposit
    TileGeom tk;  // P(k)-mesh tiles
    size_t off_s = 0, off_a = 0, off_b = 0, off_f = 0, off_k = 0, off_k2 = 0, off_twg = 0, off_twp = 0,
           off_twk = 0, off_sort = 0;
    size_t total = 0;
};

Layout layout_of(const cola_problem& p, int n_pk) {
    Layout L;
    L.g = make_mesh(p.n_part * p.pm_factor);
    L.gp = make_mesh(p.n_part);
    L.cstride = std::max(L.g.total_c(), L.gp.total_c());
    size_t cb = align256((size_t)L.cstride * sizeof(float2) * p.n_real);
    size_t off = 0;
    L.off_s = off; off += cb;
    L.off_a = off; off += cb;
    L.off_b = off; off += cb;
    L.frow = force_row3(L.g.n);
    L.fstride = (long)L.g.n * L.g.n * L.frow;
    L.off_f = off; off += align256((size_t)L.fstride * sizeof(float) * p.n_real);
    if (n_pk > 0) {
        L.gk = make_mesh(n_pk);
        L.kstride = L.gk.total_c();
        const size_t kb = align256((size_t)L.kstride * sizeof(float2) * p.n_real);
        L.off_k = off; off += kb;
        L.off_k2 = off; off += kb;
    }
    const long npr = (long)p.n_part * p.n_part * p.n_part;
    L.tg = make_tiles(L.g.n, npr);
    size_t sb = sort_bytes(npr, L.tg, p.n_real);
    if (n_pk > 0) {
        L.tk = make_tiles(n_pk, npr);
        sb = std::max(sb, sort_bytes(npr, L.tk, p.n_real));
    }
    L.off_sort = off; off += align256(sb);
    L.off_twg = off; off += align256((size_t)L.g.n * sizeof(float2));
    L.off_twp = off; off += align256((size_t)L.gp.n * sizeof(float2));
    L.off_twk = off; off += align256((size_t)(n_pk > 0 ? n_pk : 1) * sizeof(float2));
    L.total = off;
    return L;
}

int check_problem(const cola_problem* p) {
    if (!p) return COLA_ERR_INVALID_ARG;
    if (!std::isfinite(p->box) || !std::isfinite(p->z_init) || !std::isfinite(p->a_final) ||
        (p->sampling == 2 && !std::isfinite(p->sampling_power)))
        return COLA_ERR_NONFINITE;
    if (!(p->box > 0.0)) return COLA_ERR_INVALID_ARG;
    if (p->n_part < 2 || p->pm_factor < 1 || p->n_real < 1) return COLA_ERR_INVALID_ARG;
    if (p->n_steps < 2 || p->sampling < 0 || p->sampling > 2) return COLA_ERR_INVALID_ARG;
    if (p->sampling == 2 && (!std::isfinite(p->sampling_power) || !(p->sampling_power > 0.0)))
        return COLA_ERR_INVALID_ARG;
    if (p->frame != 0 && p->frame != 1) return COLA_ERR_INVALID_ARG;
    if (!(p->z_init > -1.0) || !std::isfinite(p->z_init)) return COLA_ERR_INVALID_ARG;
    double a0 = 1.0 / (1.0 + p->z_init);
    if (!(p->a_final > a0) || !std::isfinite(p->a_final)) return COLA_ERR_INVALID_ARG;
    long ng = (long)p->n_part * p->pm_factor;
    if (ng > kMaxMesh || !fft_size_ok((int)ng) || !fft_size_ok(p->n_part)) return COLA_ERR_UNSUPPORTED_SIZE;
    return COLA_OK;
}

int check_cosmo(const cola_cosmology* c) {
    if (!c) return COLA_ERR_INVALID_ARG;
    if (!std::isfinite(c->omega_m) || !std::isfinite(c->omega_b) || !std::isfinite(c->h) || !std::isfinite(c->n_s) ||
        !std::isfinite(c->sigma_8))
        return COLA_ERR_NONFINITE;
    if (!(c->omega_m > 0.0 && c->omega_m <= 1.0) || !(c->h > 0.0) || !(c->sigma_8 > 0.0) ||
        !(c->omega_b >= 0.0 && c->omega_b < c->omega_m) || !std::isfinite(c->n_s))
        return COLA_ERR_INVALID_ARG;
    return COLA_OK;
}

int check_particles(const cola_particles* P) {
    if (!P) return COLA_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (!P->x[d] || !P->p[d] || !P->psi1[d] || !P->psi2[d]) return COLA_ERR_INVALID_ARG;
    return COLA_OK;
}

ParticlePtrs ptrs_of(const cola_particles* P) {
    ParticlePtrs q;
    for (int d = 0; d < 3; ++d) {
        q.x[d] = P->x[d];
        q.p[d] = P->p[d];
        q.psi1[d] = P->psi1[d];
        q.psi2[d] = P->psi2[d];
    }
    return q;
}

struct Ws {
    float2 *S, *A, *B, *K, *K2, *twg, *twp, *twk;
    float* F;
    void* sort;
};

Ws carve(void* ws, const Layout& L) {
    char* b = static_cast<char*>(ws);
    Ws w;
    w.S = reinterpret_cast<float2*>(b + L.off_s);
    w.A = reinterpret_cast<float2*>(b + L.off_a);
    w.B = reinterpret_cast<float2*>(b + L.off_b);
    w.F = reinterpret_cast<float*>(b + L.off_f);
    w.K = L.kstride ? reinterpret_cast<float2*>(b + L.off_k) : nullptr;
    w.K2 = L.kstride ? reinterpret_cast<float2*>(b + L.off_k2) : nullptr;
    w.twg = reinterpret_cast<float2*>(b + L.off_twg);
    w.twp = reinterpret_cast<float2*>(b + L.off_twp);
    w.twk = reinterpret_cast<float2*>(b + L.off_twk);
    w.sort = b + L.off_sort;
    return w;
}

// The force mesh's cells relative to the lattice, with the rows of the interleaved force mesh F
// (force_geom) or of the density mesh in S (dens_geom).
LatticeGeom force_geom(const cola_problem& p, const Layout& L) {
    LatticeGeom g;
    g.n_part = p.n_part;
    g.n_mesh = L.g.n;
    g.inv_h = (float)(L.g.n / p.box);
    g.qoff = 0.5f;
    g.row = L.frow;
    g.mesh_bstride = L.fstride;
    return g;
}
LatticeGeom dens_geom(const cola_problem& p, const Layout& L) {
    LatticeGeom g = force_geom(p, L);
    g.row = 2L * L.g.nzp;
    g.mesh_bstride = 2L * L.cstride;
    return g;
}

// The network correction at each force evaluation: its parameters, activations (x0 per
// realization, the rest shared) and scales.
struct LcHook {
    const void* id;  // the network's parameter array: identifies the corrected force in the cache
    LcParams P;
    LcActs A;
    long x0_stride;
    float in_scale[4];
    float out_scale;
    float out_scale_slope;
    float out_band;
    int n_knots;
    float knot_a[8], knot_v[8];
    int n_gknots;
    float gknot_u[10], gknot_t[8][10];
    // The Green's-function filter at a: each knot's T interpolated over the schedule's knot_a
    // (row 0 alone without a schedule); false without a filter.
    bool filter_at(double a, GreenFilter& gf) const {
        if (n_gknots < 2) return false;
        gf.n = n_gknots;
        int i = 0;
        double t = 0.0;
        if (n_knots >= 2 && a > knot_a[0]) {
            if (a >= knot_a[n_knots - 1]) {
                i = n_knots - 1;
            } else {
                while (i + 2 < n_knots && a >= knot_a[i + 1]) ++i;
                t = (a - knot_a[i]) / ((double)knot_a[i + 1] - knot_a[i]);
            }
        }
        for (int j = 0; j < n_gknots; ++j) {
            gf.u[j] = gknot_u[j];
            const double v0 = gknot_t[i][j];
            const double v1 = t > 0.0 ? gknot_t[i + 1][j] : v0;
            gf.t[j] = (float)(v0 + t * (v1 - v0));
        }
        green_slopes(gf);
        return true;
    }
    // out_scale (1 + slope (1 - a)), times the knot schedule at a when there is one
    float scale_at(double a) const {
        double s = out_scale * (1.0 + out_scale_slope * (1.0 - a));
        if (n_knots >= 2) {
            double v = knot_v[0];
            if (a >= knot_a[n_knots - 1]) {
                v = knot_v[n_knots - 1];
            } else if (a > knot_a[0]) {
                int i = 0;
                while (i + 2 < n_knots && a >= knot_a[i + 1]) ++i;
                const double t = (a - knot_a[i]) / ((double)knot_a[i + 1] - knot_a[i]);
                v = knot_v[i] + t * ((double)knot_v[i + 1] - knot_v[i]);
            }
            s *= v;
        }
        return (float)s;
    }
};

// Density, forward transform and force mesh for the current positions: F ends up holding the
// interleaved (F_x, F_y, F_z) rows; with a network hook, dF is added to it.  binned: the particles
// were already binned for this deposit (gather_kick_drift_bin).
hipError_t compute_force(const cola_problem& p, const Layout& L, const Ws& w, const ParticlePtrs& P,
                         hipStream_t st, const LcHook* lc = nullptr, double a_node = 1.0, bool binned = false) {
    const long npr = (long)p.n_part * p.n_part * p.n_part;
    LatticeGeom dg = dens_geom(p, L);
    const double cells = (double)L.g.n * L.g.n * L.g.n;
    SortBufs sb = carve_sort(w.sort, npr, L.tg, p.n_real);
    KickDrift none{};
    float* dens = reinterpret_cast<float*>(w.S);
    const float dscale = (float)(cells / (double)npr);
    hipError_t e = binned ? sorted_deposit_binned(npr, p.n_real, dg, L.tg, sb, dens, dscale, -1.0f, st)
                          : sorted_deposit(P, npr, p.n_real, dg, false, dg, nullptr, none, L.tg, sb, dens, dscale,
                                           -1.0f, st);
    if (e != hipSuccess) return e;
    const long row = 2L * L.g.nzp, bs = 2L * L.cstride;
    if (lc)
        for (int r = 0; r < p.n_real; ++r)
            if ((e = lc_pack_delta(reinterpret_cast<const float*>(w.S) + r * bs, row, L.g.n, lc->in_scale[0],
                                   lc->A.x0 + r * lc->x0_stride, st)) != hipSuccess)
                return e;
    e = fft_zy_forward(reinterpret_cast<const float*>(w.S), row, bs, w.A, L.cstride, L.g, w.twg, p.n_real, 1.0f,
                       0.0f, st);
    if (e != hipSuccess) return e;
    GreenFilter gf;
    const bool filt = lc && lc->filter_at(a_node, gf);
    e = pm_force_interleaved(w.A, w.B, w.S, w.F, L.frow, L.fstride, L.cstride, L.g, w.twg,
                             (float)(2.0 * M_PI / p.box), p.n_real, st, filt ? &gf : nullptr);
    if (e != hipSuccess || !lc) return e;
    for (int r = 0; r < p.n_real; ++r)
        if ((e = lc_forward_fields(lc->P, lc->A.a1, lc->A.x0 + r * lc->x0_stride, w.F + r * L.fstride, L.frow, L.g.n,
                                   lc->in_scale, lc->scale_at(a_node), lc->out_band, lc->A.t, st)) != hipSuccess)
            return e;
    return mesh_ghosts(w.F, L.frow, L.g.n, L.fstride, p.n_real, st);  // the gathers read z pairs through the ghosts
}

// With the LPT frame switched off (PM only) the kick uses g alone and the drift p alone: the
// 2LPT terms of the bracket and of the drift are zero.
KickDrift frame_terms(KickDrift kd, const cola_problem& p) {
    if (p.frame == 1) {
        kd.d1 = 0.0f;
        kd.d2m = 0.0f;
        kd.dd1 = 0.0f;
        kd.dd2 = 0.0f;
    }
    return kd;
}

int step_impl(const cola_problem* prob, const cola_cosmology* cosmo, int32_t j_begin, int32_t j_end,
              cola_particles* io, void* ws, size_t ws_bytes, void* stream, const LcHook* lc) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if ((s = check_cosmo(cosmo)) != COLA_OK) return s;
    if ((s = check_particles(io)) != COLA_OK) return s;
    if (!ws) return COLA_ERR_INVALID_ARG;
    if (j_begin != io->node || j_begin < 0 || j_end < j_begin || j_end >= prob->n_steps) return COLA_ERR_STATE;
    Layout L = layout_of(*prob, 0);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    const cola_problem& p = *prob;
    ParticlePtrs P = ptrs_of(io);
    Schedule sc = make_schedule(p, *cosmo);
    const double c32 = 1.5 * sc.omega_m;
    const long npr = (long)p.n_part * p.n_part * p.n_part;
    LatticeGeom fg = force_geom(p, L), dg = dens_geom(p, L);

    const void* net_id = lc ? lc->id : nullptr;
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(w.twg, L.g.n, st));
    const bool cached = ws_holds(ws, io, j_begin, net_id, false);
    ws_forget(ws);
    if (!cached) COLA_TRY(compute_force(p, L, w, P, st, lc, sc.a[j_begin]));
    if (j_end == j_begin) {  // nothing to step: the node's force is now cached
        io->force_node = j_begin;
        io->force_ws = ws;
        ws_record(ws, io, j_begin, net_id);
        return COLA_OK;
    }
    double pending = 0.0;  // kick still owed to the current node (merged with the next kick)
    for (int j = j_begin; j < j_end; ++j) {
        KickDrift kd;
        kd.kick = (float)(c32 * (pending + sc.k_out[j]));
        kd.d1 = (float)sc.d1[j];
        kd.d2m = (float)(sc.d2[j] - sc.d1[j] * sc.d1[j]);
        kd.drift = (float)sc.drift[j];
        kd.dd1 = (float)(sc.d1[j + 1] - sc.d1[j]);
        kd.dd2 = (float)(sc.d2[j + 1] - sc.d2[j]);
        COLA_TRY(gather_kick_drift_bin(P, npr, p.n_real, fg, w.F, dg, frame_terms(kd, p), L.tg,
                                       carve_sort(w.sort, npr, L.tg, p.n_real), st));
        COLA_TRY(compute_force(p, L, w, P, st, lc, sc.a[j + 1], true));
        pending = sc.k_in[j];
    }
    KickDrift kd{};
    kd.kick = (float)(c32 * pending);
    kd.d1 = (float)sc.d1[j_end];
    kd.d2m = (float)(sc.d2[j_end] - sc.d1[j_end] * sc.d1[j_end]);
    COLA_TRY(gather_kick_drift(P, npr, p.n_real, fg, w.F, frame_terms(kd, p), st));
    io->node = j_end;
    io->force_node = j_end;
    io->force_ws = ws;
    ws_record(ws, io, j_end, net_id);
    return COLA_OK;
}

}  // namespace

extern "C" {

const char* cola_version(void) { return "libcola 0.1 (gfx950)"; }

const char* cola_last_error(void) { return g_last_error; }

const char* cola_status_string(int status) {
    switch (status) {
        case COLA_OK: return "ok";
        case COLA_ERR_INVALID_ARG: return "invalid argument (NULL pointer or out-of-range parameter)";
        case COLA_ERR_UNSUPPORTED_SIZE:
            return "unsupported mesh size (must be even, <= 1536, with prime factors 2 and 3 only)";
        case COLA_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case COLA_ERR_HIP: return "HIP runtime error";
        case COLA_ERR_STATE: return "particle state does not fit the call (node range)";
        case COLA_ERR_NONFINITE: return "non-finite floating-point argument (NaN or infinity)";
        default: return "unknown status";
    }
}

size_t cola_workspace_bytes(const cola_problem* prob, int32_t n_pk) {
    if (check_problem(prob) != COLA_OK) return 0;
    if (n_pk < 0 || (n_pk > 0 && (!fft_size_ok(n_pk) || n_pk > kMaxMesh))) return 0;
    return layout_of(*prob, n_pk).total;
}

int cola_schedule_table(const cola_problem* prob, const cola_cosmology* cosmo, double* out) {
    int s = check_problem(prob);
    if (s != COLA_OK) return s;
    if ((s = check_cosmo(cosmo)) != COLA_OK) return s;
    if (!out) return COLA_ERR_INVALID_ARG;
    Schedule sc = make_schedule(*prob, *cosmo);
    int n = prob->n_steps;
    for (int j = 0; j < n; ++j) {
        double* r = out + 6 * j;
        r[0] = sc.a[j];
        r[1] = sc.d1[j];
        r[2] = sc.d2[j];
        r[3] = j + 1 < n ? sc.k_out[j] : 0.0;
        r[4] = j + 1 < n ? sc.k_in[j] : 0.0;
        r[5] = j + 1 < n ? sc.drift[j] : 0.0;
    }
    return COLA_OK;
}

double cola_linear_power(const cola_cosmology* cosmo, double k) {
    if (check_cosmo(cosmo) != COLA_OK || !(k >= 0.0)) return -1.0;
    if (k == 0.0) return 0.0;
    double t = bbks_transfer(k, bbks_gamma(*cosmo));
    return linear_amplitude(*cosmo) * std::pow(k, cosmo->n_s) * t * t;
}

int cola_ic_2lpt(const cola_problem* prob, const cola_cosmology* cosmo, const uint64_t* seeds,
                 cola_particles* out, void* ws, size_t ws_bytes, void* stream) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if ((s = check_cosmo(cosmo)) != COLA_OK) return s;
    if ((s = check_particles(out)) != COLA_OK) return s;
    if (!seeds || !ws) return COLA_ERR_INVALID_ARG;
    Layout L = layout_of(*prob, 0);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    const cola_problem& p = *prob;
    const int np = p.n_part;
    const long npr = (long)np * np * np;
    const Mesh3& gp = L.gp;
    const float kf = (float)(2.0 * M_PI / p.box);
    const float inv_n3 = (float)(1.0 / (double)npr);
    ParticlePtrs P = ptrs_of(out);
    ws_forget(ws);

    (void)hipGetLastError();  // drop a stale error left by other code on this thread
    COLA_TRY(launch_twiddles(w.twp, gp.n, st));
    // white noise -> delta_k in S
    COLA_TRY(ic_noise(out->p[0], np, seeds, p.n_real, npr, st));
    COLA_TRY(fft3d_r2c(out->p[0], np, npr, w.S, L.cstride, gp, w.twp, p.n_real, 1.0f, 0.0f, st));
    double amp = linear_amplitude(*cosmo), gamma = bbks_gamma(*cosmo);
    COLA_TRY(ic_scale_spectrum(w.S, L.cstride, gp, p.n_real, kf, amp, gamma, cosmo->n_s,
                               (double)npr / (p.box * p.box * p.box), st));
    // second-order source S(q) in p[0]; phi_ii in x[0..2], phi_ij scratch in p[1]
    for (int a = 0; a < 3; ++a)
        COLA_TRY(fft3d_c2r_mult(w.S, L.cstride, w.A, L.cstride, out->x[a], np, npr, gp, w.twp, p.n_real, MUL_KK,
                                a, a, kf, inv_n3, st));
    const long ntot = npr * p.n_real;
    COLA_TRY(lpt2_source(out->p[0], out->x[0], out->x[1], out->x[2], ntot, 0, st));
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto& pr : pairs) {
        COLA_TRY(fft3d_c2r_mult(w.S, L.cstride, w.A, L.cstride, out->p[1], np, npr, gp, w.twp, p.n_real, MUL_KK,
                                pr[0], pr[1], kf, inv_n3, st));
        COLA_TRY(lpt2_source(out->p[0], out->p[1], nullptr, nullptr, ntot, 1, st));
    }
    COLA_TRY(fft3d_r2c(out->p[0], np, npr, w.B, L.cstride, gp, w.twp, p.n_real, 1.0f, 0.0f, st));
    for (int d = 0; d < 3; ++d) {
        COLA_TRY(fft3d_c2r_mult(w.B, L.cstride, w.A, L.cstride, out->psi2[d], np, npr, gp, w.twp, p.n_real,
                                MUL_IK, d, d, kf, -inv_n3, st));
        COLA_TRY(fft3d_c2r_mult(w.S, L.cstride, w.A, L.cstride, out->psi1[d], np, npr, gp, w.twp, p.n_real,
                                MUL_IK, d, d, kf, inv_n3, st));
    }
    const double a0 = 1.0 / (1.0 + p.z_init);
    Growth g0 = growth(a0, cosmo->omega_m);
    // PM only: the full 2LPT momentum a^2 dD/dt = a^3 E(a) dD/da; COLA: zero residual
    const double mom = p.frame == 1 ? a0 * a0 * a0 * hubble_e(a0, cosmo->omega_m) : 0.0;
    COLA_TRY(ic_set_state(P, ntot, (float)g0.d1, (float)g0.d2, (float)(mom * g0.dd1_da), (float)(mom * g0.dd2_da),
                          st));
    out->node = 0;
    out->force_node = -1;
    out->force_ws = nullptr;
    return COLA_OK;
}

int cola_pm_force(const cola_problem* prob, const cola_particles* in, float* acc[3], void* ws,
                  size_t ws_bytes, void* stream) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if ((s = check_particles(in)) != COLA_OK) return s;
    if (!acc || !acc[0] || !acc[1] || !acc[2] || !ws) return COLA_ERR_INVALID_ARG;
    Layout L = layout_of(*prob, 0);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    ParticlePtrs P = ptrs_of(in);
    ws_forget(ws);
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(w.twg, L.g.n, st));
    COLA_TRY(compute_force(*prob, L, w, P, st));
    const long npr = (long)prob->n_part * prob->n_part * prob->n_part;
    COLA_TRY(gather_force(P, npr, prob->n_real, force_geom(*prob, L), w.F, acc, st));
    return COLA_OK;
}

int cola_step(const cola_problem* prob, const cola_cosmology* cosmo, int32_t j_begin, int32_t j_end,
              cola_particles* io, void* ws, size_t ws_bytes, void* stream) {
    return step_impl(prob, cosmo, j_begin, j_end, io, ws, ws_bytes, stream, nullptr);
}

}  // extern "C"

namespace {
// Validates a network for a problem's force mesh and fills the step's hook; a cola_status.
int make_hook(const cola_problem* prob, const cola_lc_net* net, void* lc_ws, size_t lc_ws_bytes, LcHook& h) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if ((s = lc_check_net(net, false)) != COLA_OK) return s;
    const int ng = prob->n_part * prob->pm_factor;
    if (!lc_mesh_ok(ng)) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!lc_ws) return COLA_ERR_INVALID_ARG;
    const LcWsLayout LL = lc_ws_layout(ng, net->channels, prob->n_real, false);
    if (lc_ws_bytes < LL.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    h.id = net->params;
    h.P = lc_params_of(net);
    h.A = lc_carve(lc_ws, LL);
    h.x0_stride = LL.x0_stride;
    for (int i = 0; i < 4; ++i) h.in_scale[i] = net->in_scale[i];
    h.out_scale = net->out_scale;
    h.out_scale_slope = net->out_scale_slope;
    h.out_band = net->out_band;
    h.n_knots = net->n_knots;
    for (int i = 0; i < 8; ++i) {
        h.knot_a[i] = net->knot_a[i];
        h.knot_v[i] = net->knot_v[i];
    }
    h.n_gknots = net->n_gknots;
    for (int j = 0; j < 10; ++j) {
        h.gknot_u[j] = net->gknot_u[j];
        for (int i = 0; i < 8; ++i) h.gknot_t[i][j] = net->gknot_t[i][j];
    }
    return COLA_OK;
}
}  // namespace

extern "C" {

int cola_step_lc(const cola_problem* prob, const cola_cosmology* cosmo, int32_t j_begin, int32_t j_end,
                 cola_particles* io, const cola_lc_net* net, void* lc_ws, size_t lc_ws_bytes, void* ws,
                 size_t ws_bytes, void* stream) {
    LcHook h;
    const int s = make_hook(prob, net, lc_ws, lc_ws_bytes, h);
    if (s != COLA_OK) return s;
    return step_impl(prob, cosmo, j_begin, j_end, io, ws, ws_bytes, stream, &h);
}

int cola_pm_force_lc(const cola_problem* prob, const cola_particles* in, const cola_lc_net* net, double a,
                     void* lc_ws, size_t lc_ws_bytes, float* acc[3], void* ws, size_t ws_bytes, void* stream) {
    LcHook h;
    int s = make_hook(prob, net, lc_ws, lc_ws_bytes, h);
    if (s != COLA_OK) return s;
    if ((s = check_particles(in)) != COLA_OK) return s;
    if (!std::isfinite(a)) return COLA_ERR_NONFINITE;
    if (!acc || !acc[0] || !acc[1] || !acc[2] || !ws || !(a > 0.0)) return COLA_ERR_INVALID_ARG;
    Layout L = layout_of(*prob, 0);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    ParticlePtrs P = ptrs_of(in);
    ws_forget(ws);
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(w.twg, L.g.n, st));
    COLA_TRY(compute_force(*prob, L, w, P, st, &h, a));
    const long npr = (long)prob->n_part * prob->n_part * prob->n_part;
    COLA_TRY(gather_force(P, npr, prob->n_real, force_geom(*prob, L), w.F, acc, st));
    return COLA_OK;
}

int cola_fft_set_shape(int32_t n, const char* kind, int32_t values_per_thread, int32_t width, int32_t use_static) {
    return set_fft_shape(n, kind, values_per_thread, width, use_static);
}

namespace {

// P(k) of the state (Sec. 2.5); alias_iters > 0 adds that many iterations of the Jing (2005)
// aliasing correction.
int power_spectrum_impl(const cola_problem* prob, const cola_cosmology* cosmo, cola_particles* in, double a_out,
                        int32_t n_pk, int32_t n_bins, int alias_iters, double* k_mean, double* pk, double* n_modes,
                        void* ws, size_t ws_bytes, void* stream) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if ((s = check_cosmo(cosmo)) != COLA_OK) return s;
    if ((s = check_particles(in)) != COLA_OK) return s;
    if (!k_mean || !pk || !n_modes || !ws) return COLA_ERR_INVALID_ARG;
    if (!std::isfinite(a_out)) return COLA_ERR_NONFINITE;
    if (n_bins < 1 || n_bins > 4096) return COLA_ERR_INVALID_ARG;
    if (!fft_size_ok(n_pk) || n_pk > kMaxMesh) return COLA_ERR_UNSUPPORTED_SIZE;
    if (in->node < 0 || in->node >= prob->n_steps) return COLA_ERR_STATE;
    const cola_problem& p = *prob;
    Layout L = layout_of(p, n_pk);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    Schedule sc = make_schedule(p, *cosmo);
    const int j = in->node;
    const double aj = sc.a[j];
    const bool on_node = std::fabs(a_out - aj) <= 1e-12 * aj;
    if (!on_node && !(j + 1 < p.n_steps && a_out > aj && a_out < sc.a[j + 1])) return COLA_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    ParticlePtrs P = ptrs_of(in);
    const long npr = (long)p.n_part * p.n_part * p.n_part;
    LatticeGeom fg = force_geom(p, L);
    KickDrift kd{};
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(w.twg, L.g.n, st));
    COLA_TRY(launch_twiddles(w.twk, n_pk, st));
    if (!on_node) {
        // the force the state's own run used at node j (any network); without one cached, the
        // plain mesh force is evaluated and cached
        if (!ws_holds(ws, in, j, nullptr, true)) {
            ws_forget(ws);
            COLA_TRY(compute_force(p, L, w, P, st));
            in->force_node = j;
            in->force_ws = ws;
            ws_record(ws, in, j, nullptr);
        }
        Growth go = growth(a_out, sc.omega_m);
        kd.kick = (float)(1.5 * sc.omega_m * sc.k_out[j]);
        kd.d1 = (float)sc.d1[j];
        kd.d2m = (float)(sc.d2[j] - sc.d1[j] * sc.d1[j]);
        kd.drift = (float)drift_integral(aj, a_out, sc.omega_m);
        kd.dd1 = (float)(go.d1 - sc.d1[j]);
        kd.dd2 = (float)(go.d2 - sc.d2[j]);
        kd = frame_terms(kd, p);
    }
    const Mesh3& gk = L.gk;
    LatticeGeom dg;
    dg.n_part = p.n_part;
    dg.n_mesh = n_pk;
    dg.inv_h = (float)(n_pk / p.box);
    dg.qoff = (float)(0.5 * (double)n_pk / (double)L.g.n);
    dg.row = 2L * gk.nzp;
    dg.mesh_bstride = 2L * L.kstride;
    double cells = (double)n_pk * n_pk * n_pk;
    SortBufs sb = carve_sort(w.sort, npr, L.tk, p.n_real);
    COLA_TRY(sorted_deposit(P, npr, p.n_real, dg, !on_node, fg, w.F, kd, L.tk, sb, reinterpret_cast<float*>(w.K),
                            (float)(cells / (double)npr), -1.0f, st));
    COLA_TRY(fft3d_r2c(reinterpret_cast<const float*>(w.K), 2L * gk.nzp, 2L * L.kstride, w.K2, L.kstride, gk, w.twk,
                       p.n_real, 1.0f, 0.0f, st));
    const long nb = (long)n_bins * p.n_real;
    COLA_TRY(launch_fill_d(k_mean, nb, 0.0, st));
    COLA_TRY(launch_fill_d(pk, nb, 0.0, st));
    COLA_TRY(launch_fill_d(n_modes, nb, 0.0, st));
    COLA_TRY(pk_bin(w.K2, L.kstride, gk, p.n_real, n_bins, k_mean, pk, n_modes, 2.0 * M_PI / p.box, st));
    double pnorm = p.box * p.box * p.box / (cells * cells);
    COLA_TRY(pk_finish(k_mean, pk, n_modes, nb, pnorm, st));
    if (alias_iters > 0) {
        // the density mesh K is free once transformed: it holds the aliasing tables
        const long sstride = 2L * L.kstride;
        if (pk_alias_scratch_floats(n_pk, n_bins) > sstride) return COLA_ERR_WORKSPACE_TOO_SMALL;
        for (int it = 0; it < alias_iters; ++it)
            COLA_TRY(pk_alias_pass(w.K2, L.kstride, gk, p.n_real, n_bins, k_mean, pk, n_modes, pnorm,
                                   2.0 * M_PI / p.box, reinterpret_cast<float*>(w.K), sstride, st));
    }
    return COLA_OK;
}

}  // namespace

int cola_power_spectrum(const cola_problem* prob, const cola_cosmology* cosmo, cola_particles* in,
                        double a_out, int32_t n_pk, int32_t n_bins, double* k_mean, double* pk,
                        double* n_modes, void* ws, size_t ws_bytes, void* stream) {
    return power_spectrum_impl(prob, cosmo, in, a_out, n_pk, n_bins, 0, k_mean, pk, n_modes, ws, ws_bytes, stream);
}

int cola_power_spectrum_jing(const cola_problem* prob, const cola_cosmology* cosmo, cola_particles* in,
                             double a_out, int32_t n_pk, int32_t n_bins, int32_t iterations, double* k_mean,
                             double* pk, double* n_modes, void* ws, size_t ws_bytes, void* stream) {
    if (iterations < 1 || iterations > 16) return COLA_ERR_INVALID_ARG;
    return power_spectrum_impl(prob, cosmo, in, a_out, n_pk, n_bins, iterations, k_mean, pk, n_modes, ws, ws_bytes,
                               stream);
}

int cola_power_multipoles(const cola_problem* prob, const cola_cosmology* cosmo, cola_particles* in, double a_out,
                          int32_t los, int32_t redshift_space, int32_t n_pk, int32_t n_bins, double* k_mean,
                          double* p0, double* p2, double* p4, double* n_modes, void* ws, size_t ws_bytes,
                          void* stream) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if ((s = check_cosmo(cosmo)) != COLA_OK) return s;
    if ((s = check_particles(in)) != COLA_OK) return s;
    if (!k_mean || !p0 || !p2 || !p4 || !n_modes || !ws) return COLA_ERR_INVALID_ARG;
    if (!std::isfinite(a_out)) return COLA_ERR_NONFINITE;
    if (n_bins < 1 || n_bins > 4096 || los < 0 || los > 2) return COLA_ERR_INVALID_ARG;
    if (!fft_size_ok(n_pk) || n_pk > kMaxMesh) return COLA_ERR_UNSUPPORTED_SIZE;
    if (in->node < 0 || in->node >= prob->n_steps) return COLA_ERR_STATE;
    const cola_problem& p = *prob;
    Layout L = layout_of(p, n_pk);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    Schedule sc = make_schedule(p, *cosmo);
    const int j = in->node;
    const double aj = sc.a[j];
    // velocities are synced only at a node: the output must sit on the state's node
    if (!(std::fabs(a_out - aj) <= 1e-12 * aj)) return COLA_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    ParticlePtrs P = ptrs_of(in);
    const long npr = (long)p.n_part * p.n_part * p.n_part;
    LatticeGeom fg = force_geom(p, L);
    // Eq. 5, plane-parallel: s = x + v_los / (a H) along axis los, v = a dx/dt the peculiar
    // velocity.  With p = a^2 dx/dt (H0 = 1) the shift is p_los / (a^2 E(a)); in the COLA frame
    // p = p_res + a^3 E (dD1/da Psi1 + dD2/da Psi2), which adds a (dD1/da Psi1 + dD2/da Psi2).
    KickDrift kd{};
    kd.los = los;
    if (redshift_space) {
        const double e = hubble_e(aj, sc.omega_m);
        Growth ga = growth(aj, sc.omega_m);
        kd.drift = (float)(1.0 / (aj * aj * e));
        kd.dd1 = p.frame == 1 ? 0.0f : (float)(aj * ga.dd1_da);
        kd.dd2 = p.frame == 1 ? 0.0f : (float)(aj * ga.dd2_da);
    }
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(w.twk, n_pk, st));
    const Mesh3& gk = L.gk;
    LatticeGeom dg;
    dg.n_part = p.n_part;
    dg.n_mesh = n_pk;
    dg.inv_h = (float)(n_pk / p.box);
    dg.qoff = (float)(0.5 * (double)n_pk / (double)L.g.n);
    dg.row = 2L * gk.nzp;
    dg.mesh_bstride = 2L * L.kstride;
    double cells = (double)n_pk * n_pk * n_pk;
    SortBufs sb = carve_sort(w.sort, npr, L.tk, p.n_real);
    COLA_TRY(sorted_deposit(P, npr, p.n_real, dg, redshift_space != 0, fg, w.F, kd, L.tk, sb,
                            reinterpret_cast<float*>(w.K), (float)(cells / (double)npr), -1.0f, st));
    COLA_TRY(fft3d_r2c(reinterpret_cast<const float*>(w.K), 2L * gk.nzp, 2L * L.kstride, w.K2, L.kstride, gk, w.twk,
                       p.n_real, 1.0f, 0.0f, st));
    const long nb = (long)n_bins * p.n_real;
    for (double* o : {k_mean, p0, p2, p4, n_modes}) COLA_TRY(launch_fill_d(o, nb, 0.0, st));
    COLA_TRY(pk_bin_multipoles(w.K2, L.kstride, gk, p.n_real, n_bins, los, k_mean, p0, p2, p4, n_modes,
                               2.0 * M_PI / p.box, st));
    COLA_TRY(pk_finish_multipoles(k_mean, p0, p2, p4, n_modes, nb, p.box * p.box * p.box / (cells * cells), st));
    return COLA_OK;
}

// ---------------------------------------------------------------- component entry points

size_t cola_cic_workspace_bytes(int64_t n, int32_t n_mesh) {
    if (n < 1 || n > (int64_t)INT32_MAX - 1 || n_mesh < 2 || n_mesh > kMaxMesh) return 0;
    const TileGeom tg = make_tiles(n_mesh, (long)n);
    if (tg.nkeys + 1 > (long)INT32_MAX) return 0;  // 32-bit tile keys
    return sort_bytes((long)n, tg, 1);
}

int cola_cic_density(const float* pos[3], int64_t n, int32_t n_mesh, double box, float* delta, void* ws,
                     size_t ws_bytes, void* stream) {
    if (!std::isfinite(box)) return COLA_ERR_NONFINITE;
    if (!pos || !pos[0] || !pos[1] || !pos[2] || !delta || !ws || n < 1 || n > (int64_t)INT32_MAX - 1 ||
        n_mesh < 2 || n_mesh > kMaxMesh || !(box > 0.0))
        return COLA_ERR_INVALID_ARG;
    const size_t need = cola_cic_workspace_bytes(n, n_mesh);
    if (need == 0) return COLA_ERR_UNSUPPORTED_SIZE;
    if (ws_bytes < need) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TileGeom tg = make_tiles(n_mesh, (long)n);
    const SortBufs sb = carve_sort(ws, (long)n, tg, 1);
    const double cells = (double)n_mesh * n_mesh * n_mesh;
    ws_forget(ws);
    (void)hipGetLastError();
    COLA_TRY(sorted_deposit_absolute(pos, (long)n, n_mesh, (float)(n_mesh / box), tg, sb, delta, n_mesh,
                                     (float)(cells / (double)n), -1.0f, st));
    return COLA_OK;
}

int cola_autotune(const cola_problem* prob, int32_t n_pk, void* ws, size_t ws_bytes, void* stream, char* report,
                  size_t report_len) {
    int s;
    if ((s = check_problem(prob)) != COLA_OK) return s;
    if (!ws) return COLA_ERR_INVALID_ARG;
    if (n_pk < 0 || (n_pk > 0 && (!fft_size_ok(n_pk) || n_pk > kMaxMesh))) return COLA_ERR_UNSUPPORTED_SIZE;
    Layout L = layout_of(*prob, n_pk);
    if (ws_bytes < L.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ws w = carve(ws, L);
    ws_forget(ws);
    std::string rep;
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(w.twg, L.g.n, st));
    COLA_TRY(autotune_fft(L.g.n, w.S, w.A, w.B, w.twg, st, &rep));
    if (L.gp.n != L.g.n) {
        COLA_TRY(launch_twiddles(w.twp, L.gp.n, st));
        COLA_TRY(autotune_fft(L.gp.n, w.S, w.A, w.B, w.twp, st, &rep));
    }
    if (n_pk > 0 && n_pk != L.g.n && n_pk != L.gp.n) {
        COLA_TRY(launch_twiddles(w.twk, n_pk, st));
        if (n_pk <= L.g.n) COLA_TRY(autotune_fft(n_pk, w.S, w.A, w.B, w.twk, st, &rep));
        else COLA_TRY(autotune_fft(n_pk, w.K, w.K2, w.K, w.twk, st, &rep));
    }
    if (report && report_len > 0) {
        std::snprintf(report, report_len, "%s", rep.c_str());
    }
    return COLA_OK;
}

int cola_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst) return COLA_ERR_INVALID_ARG;
    (void)hipGetLastError();
    COLA_TRY(launch_copy(src, dst, bytes, static_cast<hipStream_t>(stream)));
    return COLA_OK;
}

size_t cola_fft_workspace_bytes(int32_t n) {
    if (!fft_size_ok(n) || n > kMaxMesh) return 0;
    Mesh3 g = make_mesh(n);
    return align256(g.bytes()) + align256((size_t)n * sizeof(float2));
}

int cola_fft_r2c(int32_t n, const float* in, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!fft_size_ok(n) || n > kMaxMesh) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!in || !out || !ws) return COLA_ERR_INVALID_ARG;
    if (ws_bytes < cola_fft_workspace_bytes(n)) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Mesh3 g = make_mesh(n);
    float2* spec = static_cast<float2*>(ws);
    float2* tw = reinterpret_cast<float2*>(static_cast<char*>(ws) + align256(g.bytes()));
    ws_forget(ws);
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(tw, n, st));
    COLA_TRY(fft3d_r2c(in, n, 0, spec, 0, g, tw, 1, 1.0f, 0.0f, st));
    COLA_TRY(copy_pad_to_unpad(spec, reinterpret_cast<float2*>(out), g, st));
    return COLA_OK;
}

int cola_fft_c2r(int32_t n, const float* in, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!fft_size_ok(n) || n > kMaxMesh) return COLA_ERR_UNSUPPORTED_SIZE;
    if (!in || !out || !ws) return COLA_ERR_INVALID_ARG;
    if (ws_bytes < cola_fft_workspace_bytes(n)) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Mesh3 g = make_mesh(n);
    float2* spec = static_cast<float2*>(ws);
    float2* tw = reinterpret_cast<float2*>(static_cast<char*>(ws) + align256(g.bytes()));
    ws_forget(ws);
    (void)hipGetLastError();
    COLA_TRY(launch_twiddles(tw, n, st));
    COLA_TRY(copy_unpad_to_pad(reinterpret_cast<const float2*>(in), spec, g, st));
    COLA_TRY(fft3d_c2r_mult(spec, 0, spec, 0, out, n, 0, g, tw, 1, MUL_SCALE, 0, 0, 1.0f, 1.0f, st));
    return COLA_OK;
}

}  // extern "C"
