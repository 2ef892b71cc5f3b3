// Friends-of-friends haloes (Sec. 2.1: linking length 0.2 of the mean inter-particle separation,
// after Davis et al. 1985), their catalogue and the binned Warren mass function (Sec. 2.5).
//
// Two particles are friends when their periodic distance is below the linking length b; groups
// are the connected components of the friendship graph, labelled by their smallest particle
// index.  The decision is taken in float32 with every operation rounded on its own:
//   d = x_j - x_i;  d -= L if d > L/2;  d += L if d < -L/2      (per axis)
//   d2 = (dx*dx + dy*dy) + dz*dz;   friends iff d2 < b2,  b2 = float32(b) * float32(b).
//
// Passes (one stream, all device work):
//   bin      cell of every particle on a grid of cells no smaller than b, counts per cell;
//   scan     exclusive scan of the counts (shared with the tiled deposit);
//   scatter  particle records {x, y, z, index} in cell order;
//   link     one thread per record: the pairs with the records after it in its own cell and
//            with every record of the 13 "forward" neighbour cells (each unordered pair of
//            cells once); a friend pair joins its two trees in a lock-free union-find;
//   finish   every particle's root, written back as its label (full compression), and the
//            group sizes at the roots.
//
// Union-find invariant: a root is only hooked under a smaller root (compare-and-swap on the
// root's own entry) and path halving only replaces a parent by one of its ancestors, so every
// non-root entry holds a smaller index than its own.  Walks therefore end, no cycle can form,
// and the root of each tree is the smallest index in it.  Each failed compare-and-swap means
// another thread completed a hook, and at most n - 1 hooks exist, so every thread exits.
//
// Cost: the link pass tests every pair in each cell and between forward neighbours, so its time
// grows with the square of the particles per cell.  At the mean density there is about one
// particle per cell; the densest cells of the z = 0 runs hold a few hundred.  Positions that
// pile a large fraction of all particles into one cell (a degenerate input) make the pass
// quadratic in n.

#include <algorithm>
#include <cmath>

#include "cola_internal.h"
#include "lc_internal.h"
#include "wave_ops.h"

namespace cola {

namespace {

constexpr int kFofMaxBins = 64;

struct FofGrid {
    int nc;          // cells per side
    float inv_cell;  // nc / L
    long ncell;
};

struct MassBins {
    int nb;
    int32_t lo[kFofMaxBins + 1];  // particle-count edges: bin b holds lo[b] <= N < lo[b + 1]
};

__device__ __forceinline__ int cell1(float x, float inv_cell, int nc) {
    int c = (int)floorf(x * inv_cell);
    c %= nc;
    c = c < 0 ? c + nc : c;
    return min(max(c, 0), nc - 1);  // a non-finite coordinate still maps into the grid
}

__device__ __forceinline__ uint32_t cell3(float x, float y, float z, const FofGrid& g) {
    const int cx = cell1(x, g.inv_cell, g.nc), cy = cell1(y, g.inv_cell, g.nc), cz = cell1(z, g.inv_cell, g.nc);
    return (uint32_t)(((long)cx * g.nc + cy) * g.nc + cz);
}

__device__ __forceinline__ int32_t ld_parent(const int32_t* p, int32_t x) {
    return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_parent(int32_t* p, int32_t x, int32_t v) {
    __hip_atomic_store(p + x, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.
__device__ __forceinline__ int32_t fof_find(int32_t* parent, int32_t x) {
    while (true) {
        const int32_t p = ld_parent(parent, x);
        if (p == x) return x;
        const int32_t gp = ld_parent(parent, p);
        if (gp != p) st_parent(parent, x, gp);
        x = gp;
    }
}

__device__ __forceinline__ void fof_union(int32_t* parent, int32_t a, int32_t b) {
    // friends inside a halo mostly share a parent already (path halving points them at the root):
    // then the sets are joined and both find walks are skipped
    const int32_t pa = ld_parent(parent, a), pb = ld_parent(parent, b);
    if (pa == pb) return;
    a = pa;
    b = pb;
    while (true) {
        int32_t ra = fof_find(parent, a), rb = fof_find(parent, b);
        if (ra == rb) return;
        if (ra > rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        if (atomicCAS(parent + rb, rb, ra) == rb) return;  // rb was still a root: hooked
        a = ra;
        b = rb;
    }
}

__device__ __forceinline__ float min_image(float d, float box, float half) {
    if (d > half) return d - box;
    if (d < -half) return d + box;
    return d;
}

__device__ __forceinline__ float d2_of(float4 a, float4 b, float box, float half) {
#pragma clang fp contract(off)  // each product and sum rounded on its own, no fused multiply-add
    const float dx = min_image(b.x - a.x, box, half);
    const float dy = min_image(b.y - a.y, box, half);
    const float dz = min_image(b.z - a.z, box, half);
    const float sxy = dx * dx + dy * dy;
    return sxy + dz * dz;
}

__global__ void k_fof_bin(const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
                          long n, FofGrid g, uint32_t* cell_of, uint32_t* count) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;  // every lane takes part in the wave-level counting
    uint32_t c = 0;
    if (valid) {
        c = cell3(px[i], py[i], pz[i], g);
        cell_of[i] = c;
    }
    (void)wave_increment(count, c, valid);
}

__global__ void k_fof_scatter(const float* __restrict__ px, const float* __restrict__ py,
                              const float* __restrict__ pz, long n, const uint32_t* cell_of, uint32_t* cursor,
                              float4* recs, int32_t* parent) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    const uint32_t slot = wave_increment(cursor, valid ? cell_of[i] : 0u, valid);
    if (!valid) return;
    recs[slot] = make_float4(px[i], py[i], pz[i], __int_as_float((int)i));
    parent[i] = (int32_t)i;
}

// Offsets (ox, oy, oz) in {-1, 0, 1}^3 that are lexicographically after (0, 0, 0).
__constant__ int8_t kForward[13][3] = {{0, 0, 1},  {0, 1, -1}, {0, 1, 0},  {0, 1, 1},  {1, -1, -1},
                                       {1, -1, 0}, {1, -1, 1}, {1, 0, -1}, {1, 0, 0},  {1, 0, 1},
                                       {1, 1, -1}, {1, 1, 0},  {1, 1, 1}};

__global__ void k_fof_link(const float4* __restrict__ recs, long n, FofGrid g, const uint32_t* __restrict__ start,
                           float box, float link2, int32_t* parent) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float4 a = recs[t];
    const int32_t i = __float_as_int(a.w);
    const float half = 0.5f * box;
    const int cx = cell1(a.x, g.inv_cell, g.nc), cy = cell1(a.y, g.inv_cell, g.nc), cz = cell1(a.z, g.inv_cell, g.nc);
    // the record ranges of the own cell (the records after this one) and of the 13 forward
    // neighbours, all requested before the first is used (one memory round trip, not fourteen)
    uint32_t rb[14], re[14];
    rb[0] = (uint32_t)t + 1;
    re[0] = start[((long)cx * g.nc + cy) * g.nc + cz + 1];
    const int ncells = g.nc < 3 ? 1 : 14;  // a single cell holds every particle
    if (ncells == 14) {
#pragma unroll
        for (int o = 0; o < 13; ++o) {
            const int ux = (cx + kForward[o][0] + g.nc) % g.nc;
            const int uy = (cy + kForward[o][1] + g.nc) % g.nc;
            const int uz = (cz + kForward[o][2] + g.nc) % g.nc;
            const long c = ((long)ux * g.nc + uy) * g.nc + uz;
            rb[o + 1] = start[c];
            re[o + 1] = start[c + 1];
        }
    }
    for (int q = 0; q < ncells; ++q) {
        for (uint32_t k = rb[q]; k < re[q]; ++k) {
            const float4 b = recs[k];
            if (d2_of(a, b, box, half) < link2) fof_union(parent, i, __float_as_int(b.w));
        }
    }
}

// Every entry becomes its root (writes of an ancestor over a parent keep the forest valid for
// concurrent walks); sizes are counted at the roots.
__global__ void k_fof_finish(int32_t* parent, long n, int32_t* size) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t r = (int32_t)i;
    while (true) {
        const int32_t p = ld_parent(parent, r);
        if (p == r) break;
        r = p;
    }
    if (r != (int32_t)i) st_parent(parent, (int32_t)i, r);
    atomicAdd(size + r, 1);
}

// ---- catalogue

__global__ void k_cat_flag(const int32_t* size, long n, int32_t n_min, uint32_t* flag) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = size[i] >= n_min ? 1u : 0u;
}

__global__ void k_cat_total(const uint32_t* flag, uint32_t* hidx, long n, int64_t* n_halos) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const uint32_t total = hidx[n - 1] + flag[n - 1];
    hidx[n] = total;
    *n_halos = (int64_t)total;
}

__global__ void k_cat_fill(const uint32_t* flag, const uint32_t* hidx, const int32_t* size, long n, double m_p,
                           int32_t* root, int32_t* count, double* mass, double* cx, double* cy, double* cz) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint32_t h = hidx[i];
    const double N = (double)size[i];
    root[h] = (int32_t)i;
    count[h] = size[i];
    mass[h] = m_p * N * (1.0 - pow(N, -0.6));
    cx[h] = 0.0;
    cy[h] = 0.0;
    cz[h] = 0.0;
}

__global__ void k_cat_sum(const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
                          long n, const int32_t* group, const uint32_t* flag, const uint32_t* hidx, float box,
                          double* cx, double* cy, double* cz) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = group[i];
    if (r < 0 || r >= n || !flag[r]) return;  // a label outside the particle range is ignored
    const uint32_t h = hidx[r];
    const float half = 0.5f * box;
    atomicAdd(cx + h, (double)min_image(px[i] - px[r], box, half));
    atomicAdd(cy + h, (double)min_image(py[i] - py[r], box, half));
    atomicAdd(cz + h, (double)min_image(pz[i] - pz[r], box, half));
}

__device__ __forceinline__ double wrap_box(double c, double box) {
    return c >= box ? c - box : (c < 0.0 ? c + box : c);
}

__global__ void k_cat_com(const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
                          const uint32_t* flag, const uint32_t* hidx, const int32_t* size, long n, double box,
                          double* cx, double* cy, double* cz) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint32_t h = hidx[i];
    const double N = (double)size[i];
    cx[h] = wrap_box((double)px[i] + cx[h] / N, box);
    cy[h] = wrap_box((double)py[i] + cy[h] / N, box);
    cz[h] = wrap_box((double)pz[i] + cz[h] / N, box);
}

// ---- mass histogram

__global__ void k_fof_hist(const int32_t* size, long n, MassBins mb, unsigned long long* counts) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = size[i];
    if (s < mb.lo[0] || s >= mb.lo[mb.nb]) return;
    int b = 0;
    while (b + 1 < mb.nb && s >= mb.lo[b + 1]) ++b;
    atomicAdd(counts + b, 1ull);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

unsigned blocks_of(long n) { return (unsigned)((n + 255) / 256); }

// Cells per side: cells of side L / nc no smaller than b (with a margin of 1e-3 for the float32
// cell coordinate), at most ceil(cbrt(n)) per side; grids of fewer than 3 cells collapse to one
// cell so that the 13 forward neighbours are distinct cells.
FofGrid fof_grid(long n, double box, double link) {
    FofGrid g;
    const double by_link = std::floor(box / (link * 1.001));
    const double by_count = std::ceil(std::cbrt((double)std::max(1L, n)));
    int nc = (int)std::max(1.0, std::min(std::min(by_link, by_count), 1290.0));
    if (nc < 3) nc = 1;
    g.nc = nc;
    g.inv_cell = (float)(nc / box);
    g.ncell = (long)nc * nc * nc;
    return g;
}

struct FofWs {
    uint32_t* cell_of;  // n + 1 (catalogue: the halo flags)
    float4* recs;       // n
    uint32_t* count;    // keys + 1
    uint32_t* start;    // keys + 1 (catalogue: the halo index scan)
    uint32_t* cursor;   // keys + 1
    uint32_t* block_sums;
    size_t total;
};

// keys: the cells of the grid, or n + 1 for the halo-index scan, whichever is larger.
FofWs fof_ws(long n, const FofGrid& g, void* base) {
    FofWs w{};
    char* b = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = b ? b + off : nullptr;
        off += lc_align(bytes);
        return p;
    };
    const long keys = std::max(g.ncell, n + 1);
    w.cell_of = reinterpret_cast<uint32_t*>(take((size_t)(n + 1) * 4));
    w.recs = reinterpret_cast<float4*>(take((size_t)n * 16));
    w.count = reinterpret_cast<uint32_t*>(take((size_t)(keys + 1) * 4));
    w.start = reinterpret_cast<uint32_t*>(take((size_t)(keys + 1) * 4));
    w.cursor = reinterpret_cast<uint32_t*>(take((size_t)(keys + 1) * 4));
    w.block_sums = reinterpret_cast<uint32_t*>(take((size_t)((keys + 1023) / 1024 + 1) * 4));
    w.total = off;
    return w;
}

bool pos_ok(const float* const pos[3], long n) {
    return pos && pos[0] && pos[1] && pos[2] && n >= 1 && n <= (long)INT32_MAX - 1;
}

double warren(double N, double m_p) { return m_p * N * (1.0 - std::pow(N, -0.6)); }

// Smallest N >= 1 whose Warren mass reaches m (INT32_MAX if no N below it does).
int32_t first_n_reaching(double m, double m_p) {
    long lo = 1, hi = (long)INT32_MAX - 1;
    if (warren(1.0, m_p) >= m) return 1;
    if (!(warren((double)hi, m_p) >= m)) return INT32_MAX;
    while (hi - lo > 1) {  // warren(lo) < m <= warren(hi); the mass increases with N
        const long mid = lo + (hi - lo) / 2;
        if (warren((double)mid, m_p) >= m) hi = mid;
        else lo = mid;
    }
    return (int32_t)hi;
}

}  // namespace

}  // namespace cola

using namespace cola;

#define FOF_TRY(expr)                                        \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(_e, #expr);    \
    } while (0)

extern "C" {

size_t cola_fof_workspace_bytes(int64_t n, double box, double link) {
    if (n < 1 || n > (int64_t)INT32_MAX - 1 || !std::isfinite(box) || !(box > 0.0) || !std::isfinite(link) ||
        !(link > 0.0))
        return 0;
    return fof_ws((long)n, fof_grid((long)n, box, link), nullptr).total;
}

int cola_fof(const float* pos[3], int64_t n, double box, double link, int32_t* group, int32_t* group_size, void* ws,
             size_t ws_bytes, void* stream) {
    if (!std::isfinite(box) || !std::isfinite(link)) return COLA_ERR_NONFINITE;
    if (!pos_ok(pos, (long)n) || !std::isfinite(box) || !(box > 0.0) || !std::isfinite(link) || !(link > 0.0) ||
        !(link < 0.5 * box) || !group || !group_size || !ws)
        return COLA_ERR_INVALID_ARG;
    const FofGrid g = fof_grid((long)n, box, link);
    const FofWs w = fof_ws((long)n, g, ws);
    if (ws_bytes < w.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ws_forget(ws);
    (void)hipGetLastError();
    const float link2 = (float)link * (float)link;
    ProfScope ps(PROF_FOF, st, g.nc);
    FOF_TRY(launch_fill(reinterpret_cast<float*>(w.count), g.ncell, 0.0f, st));
    FOF_TRY(launch_fill(reinterpret_cast<float*>(group_size), (long)n, 0.0f, st));
    hipLaunchKernelGGL(k_fof_bin, dim3(blocks_of(n)), dim3(256), 0, st, pos[0], pos[1], pos[2], (long)n, g,
                       w.cell_of, w.count);
    FOF_TRY(hipGetLastError());
    FOF_TRY(scan_counts(w.count, w.start, w.cursor, w.block_sums, g.ncell, (uint32_t)n, st));
    hipLaunchKernelGGL(k_fof_scatter, dim3(blocks_of(n)), dim3(256), 0, st, pos[0], pos[1], pos[2], (long)n,
                       w.cell_of, w.cursor, w.recs, group);
    hipLaunchKernelGGL(k_fof_link, dim3(blocks_of(n)), dim3(256), 0, st, w.recs, (long)n, g, w.start, (float)box,
                       link2, group);
    hipLaunchKernelGGL(k_fof_finish, dim3(blocks_of(n)), dim3(256), 0, st, group, (long)n, group_size);
    FOF_TRY(hipGetLastError());
    return COLA_OK;
}

int cola_fof_catalogue(const float* pos[3], int64_t n, double box, const int32_t* group, const int32_t* group_size,
                       int32_t n_min, double particle_mass, int64_t max_halos, int32_t* halo_root, int32_t* halo_n,
                       double* halo_mass, double* halo_com[3], int64_t* n_halos, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!std::isfinite(box) || !std::isfinite(particle_mass)) return COLA_ERR_NONFINITE;
    if (!pos_ok(pos, (long)n) || !std::isfinite(box) || !(box > 0.0) || !group || !group_size || n_min < 1 ||
        !std::isfinite(particle_mass) || !(particle_mass > 0.0) || !halo_root || !halo_n || !halo_mass ||
        !halo_com || !halo_com[0] || !halo_com[1] || !halo_com[2] || !n_halos || !ws)
        return COLA_ERR_INVALID_ARG;
    if (max_halos < n / n_min) return COLA_ERR_INVALID_ARG;  // room for every possible halo
    // the halo-index scan needs n + 1 keys, which every workspace of cola_fof_workspace_bytes has
    const FofWs w = fof_ws((long)n, FofGrid{1, 1.0f, 1}, ws);
    if (ws_bytes < w.total) return COLA_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ws_forget(ws);
    (void)hipGetLastError();
    ProfScope ps(PROF_FOF, st, -1);
    uint32_t* flag = w.cell_of;
    uint32_t* hidx = w.start;
    hipLaunchKernelGGL(k_cat_flag, dim3(blocks_of(n)), dim3(256), 0, st, group_size, (long)n, n_min, flag);
    FOF_TRY(hipGetLastError());
    FOF_TRY(scan_counts(flag, hidx, w.cursor, w.block_sums, (long)n, 0u, st));
    hipLaunchKernelGGL(k_cat_total, dim3(1), dim3(64), 0, st, flag, hidx, (long)n, n_halos);
    hipLaunchKernelGGL(k_cat_fill, dim3(blocks_of(n)), dim3(256), 0, st, flag, hidx, group_size, (long)n,
                       particle_mass, halo_root, halo_n, halo_mass, halo_com[0], halo_com[1], halo_com[2]);
    hipLaunchKernelGGL(k_cat_sum, dim3(blocks_of(n)), dim3(256), 0, st, pos[0], pos[1], pos[2], (long)n, group, flag,
                       hidx, (float)box, halo_com[0], halo_com[1], halo_com[2]);
    hipLaunchKernelGGL(k_cat_com, dim3(blocks_of(n)), dim3(256), 0, st, pos[0], pos[1], pos[2], flag, hidx,
                       group_size, (long)n, box, halo_com[0], halo_com[1], halo_com[2]);
    FOF_TRY(hipGetLastError());
    return COLA_OK;
}

int cola_fof_mass_histogram(const int32_t* group_size, int64_t n, int32_t n_min, double particle_mass,
                            const double* log10_mass_edges, int32_t n_bins, uint64_t* counts, void* stream) {
    if (!std::isfinite(particle_mass)) return COLA_ERR_NONFINITE;
    if (!group_size || n < 1 || n > (int64_t)INT32_MAX - 1 || n_min < 1 || !std::isfinite(particle_mass) ||
        !(particle_mass > 0.0) || !log10_mass_edges || n_bins < 1 || n_bins > kFofMaxBins || !counts)
        return COLA_ERR_INVALID_ARG;
    MassBins mb{};
    mb.nb = n_bins;
    for (int b = 0; b <= n_bins; ++b) {
        const double e = log10_mass_edges[b];
        if (!std::isfinite(e)) return COLA_ERR_NONFINITE;
        if (b > 0 && !(e > log10_mass_edges[b - 1])) return COLA_ERR_INVALID_ARG;
        mb.lo[b] = std::max(first_n_reaching(std::pow(10.0, e), particle_mass), n_min);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    ProfScope ps(PROF_FOF, st, -2);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(kFofMaxBins), 0, st, reinterpret_cast<unsigned long long*>(counts),
                       n_bins);
    hipLaunchKernelGGL(k_fof_hist, dim3(blocks_of(n)), dim3(256), 0, st, group_size, (long)n, mb,
                       reinterpret_cast<unsigned long long*>(counts));
    FOF_TRY(hipGetLastError());
    return COLA_OK;
}

double cola_particle_mass(const cola_cosmology* cosmo, double box, int32_t n_part) {
    // Omega_m times the critical density today (2.775e11 h^2 M_sun Mpc^-3) per particle volume
    if (!cosmo || !(box > 0.0) || n_part < 1) return 0.0;
    const double cell = box / n_part;
    return cosmo->omega_m * 2.775e11 * cell * cell * cell;
}

}  // extern "C"
