// Cloud-in-cell mass assignment by tile ownership (Sec. 2.2: CIC onto the force mesh; Sec. 2.5:
// CIC onto the P(k) mesh), without atomics to HBM and without clearing the mesh first.
//
// The mesh is cut into tiles of TX x TY x TZ cells.  Each particle gets a key
//   key = tile(home cell) * 8 + category,   category = 4 [x on the tile's upper face]
//                                                      + 2 [y on it] + [z on it],
// where the home cell is the lower CIC corner.  A particle's eight corners land in its own tile
// and, only along axes where its category bit is set, in the next tile up.  After a counting sort
// by key, the block that owns tile M reads its own bin and, from each of the seven tiles M - d
// (d in {0,1}^3, d != 0), just the categories that contain d -- the particles whose corners reach
// into M.  It accumulates the corners that fall inside M in LDS and writes every cell of M once,
// already converted to delta = rho * scale + offset.
//
// Passes: bin (key + cell record per particle, wave-aggregated counts), exclusive scan of the
// counts, scatter of the records into key order, tile accumulation.  Records keep the CIC
// fractions exactly as computed from the lattice index and displacement.

#include "cola_internal.h"
#include "force_gather.h"
#include "wave_ops.h"

namespace cola {

// Tiles of tx x tx x tz cells: tx = 8 and tz = 64 where they divide n, with tz lowered (down to 16)
// while a tile would hold more than about 1024 particles on average -- on a mesh with a particle
// per cell (PM_grid 1) the 4096-particle tiles of 8 x 8 x 64 made the tile pass and the sort
// counters (many waves on one key) slower: 0.19 + 0.25 ms against 0.13 + 0.16 ms for 8 x 8 x 16.
TileGeom make_tiles(int n, long n_particles) {
    TileGeom t;
    t.n = n;
    t.tx = 1;
    for (int c : {8, 4, 2})
        if (n % c == 0) { t.tx = c; break; }
    t.ty = t.tx;
    const double per_cell = (double)n_particles / ((double)n * n * n);
    t.tz = 1;
    for (int c : {64, 32, 16, 8, 4, 2})
        if (n % c == 0 && (c <= 16 || (double)t.tx * t.ty * c * per_cell <= 1024.0)) { t.tz = c; break; }
    t.ntx = n / t.tx;
    t.nty = n / t.ty;
    t.ntz = n / t.tz;
    t.ntiles = (long)t.ntx * t.nty * t.ntz;
    t.nkeys = t.ntiles * 8;
    auto lg = [](int v) { int l = 0; while ((1 << l) < v) ++l; return l; };
    t.lx = lg(t.tx);
    t.ly = lg(t.ty);
    t.lz = lg(t.tz);
    return t;
}

namespace {

struct CellC {
    int m;
    float f;
};

// 32-bit index arithmetic: i * n_mesh < 1536^2 and a lattice index < 1536^3 < 2^32.
__device__ __forceinline__ CellC cell_c(int i, float x, int n_part, int n_mesh, float inv_h, float qoff) {
    const uint32_t a = (uint32_t)i * (uint32_t)n_mesh;
    const int q = (int)(a / (uint32_t)n_part);
    const int rem = (int)(a - (uint32_t)q * (uint32_t)n_part);
    float w = (float)rem / (float)n_part + qoff + x * inv_h;
    float fl = floorf(w);
    CellC c;
    c.f = w - fl;
    int m = (q + (int)fl) % n_mesh;
    m = m < 0 ? m + n_mesh : m;
    c.m = min(max(m, 0), n_mesh - 1);
    return c;
}

__device__ __forceinline__ void lagr_idx(uint32_t p, int n_part, int& i, int& j, int& l) {
    const uint32_t np = (uint32_t)n_part, np2 = np * np;
    const uint32_t ii = p / np2, r = p - ii * np2, jj = r / np;
    i = (int)ii;
    j = (int)jj;
    l = (int)(r - jj * np);
}

// The per-particle key and record arrays are written once and read once, in particle order:
// non-temporal, so that they do not evict mesh and count lines from L2 (the tile pass also
// stores the mesh this way).
__device__ __forceinline__ void store_rec_stream(float4* p, float4 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
}
__device__ __forceinline__ float4 load_rec_stream(const float4* p) {
    float4 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    v.z = __builtin_nontemporal_load(&p->z);
    v.w = __builtin_nontemporal_load(&p->w);
    return v;
}

// Binning of the particles onto the mesh of dg (key and cell record per particle, counts per
// key).  MODE 0: at their positions; 1: drifted on the fly (kick with the force gathered from fg's
// meshes, then the drift of kd) without changing the state -- outputs between nodes and the
// redshift-space mapping; 2: the step's gather, kick and drift, written back to p and x, then
// binned at the new positions for the next force evaluation (dg = fg).
template <int MODE>
__global__ void __launch_bounds__(256) k_dep_bin(ParticlePtrs P, long npr, LatticeGeom dg, TileGeom tg,
                                                 LatticeGeom fg, const float* F, KickDrift kd, SortBufs sb) {
    constexpr bool DRIFT = MODE != 0;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const bool valid = p < npr;
    const long gid = (long)r * npr + p;
    uint32_t key = 0;
    float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
        int idx[3];
        lagr_idx((uint32_t)p, dg.n_part, idx[0], idx[1], idx[2]);
        float x[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = __builtin_nontemporal_load(P.x[d] + gid);
        // x is issued first: loads complete in order, so the gather, whose addresses need only x,
        // waits for these three and not for the nine below
        __builtin_amdgcn_sched_barrier(0);
        if (DRIFT) {
            // The particle arrays are read before the force gather, so both are in flight together.
            // All nine are loaded without a branch: loads guarded per axis (by the line of sight)
            // made the compiler wait for each axis's loads before issuing the next, which added a
            // memory round trip to every wave.
            float s1[3], s2[3], pv[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s1[d] = __builtin_nontemporal_load(P.psi1[d] + gid);
                s2[d] = __builtin_nontemporal_load(P.psi2[d] + gid);
                pv[d] = __builtin_nontemporal_load(P.p[d] + gid);
            }
            float g[3] = {0.0f, 0.0f, 0.0f};
            if (kd.kick != 0.0f) {  // no force mesh is read for a pure drift (redshift-space mapping)
                CellC c[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) c[d] = cell_c(idx[d], x[d], fg.n_part, fg.n_mesh, fg.inv_h, fg.qoff);
                gather_interleaved(F + (long)r * fg.mesh_bstride, fg.row, fg.n_mesh, c[0].m, c[1].m, c[2].m, c[0].f,
                                   c[1].f, c[2].f, g);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (kd.los >= 0 && d != kd.los) continue;
                const float ph = pv[d] + kd.kick * (g[d] - kd.d1 * s1[d] - kd.d2m * s2[d]);
                x[d] = x[d] + ph * kd.drift + kd.dd1 * s1[d] + kd.dd2 * s2[d];
                if (MODE == 2) {
                    __builtin_nontemporal_store(ph, P.p[d] + gid);
                    __builtin_nontemporal_store(x[d], P.x[d] + gid);
                }
            }
        }
        CellC c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) c[d] = cell_c(idx[d], x[d], dg.n_part, dg.n_mesh, dg.inv_h, dg.qoff);
        const int lx = c[0].m % tg.tx, ly = c[1].m % tg.ty, lz = c[2].m % tg.tz;
        const long tile = ((long)(c[0].m / tg.tx) * tg.nty + c[1].m / tg.ty) * tg.ntz + c[2].m / tg.tz;
        const int cat = ((lx == tg.tx - 1) ? 4 : 0) | ((ly == tg.ty - 1) ? 2 : 0) | ((lz == tg.tz - 1) ? 1 : 0);
        key = (uint32_t)(tile * 8 + cat);
        const int local = (((lx << tg.ly) + ly) << tg.lz) + lz;
        rec = make_float4(__int_as_float(local), c[0].f, c[1].f, c[2].f);
        __builtin_nontemporal_store(key, sb.keys + gid);
        store_rec_stream(sb.recs + gid, rec);
    }
    (void)wave_increment(sb.count + (long)r * sb.kstride, key, valid);
}

// Binning of absolute positions (the component entry point): the cell of a coordinate is
// floor(pos / H) modulo the mesh, the fraction pos / H minus that floor.  Everything after the
// binning is the step's deposit.
__global__ void k_dep_bin_abs(const float* px, const float* py, const float* pz, long n, int n_mesh, float inv_h,
                              TileGeom tg, SortBufs sb) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n;
    uint32_t key = 0;
    if (valid) {
        const float* ps[3] = {px, py, pz};
        CellC c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            // rounded product: contracted into u - floor(u) as one fused multiply-add, the
            // fraction of a coordinate that rounds up to a node would come out negative
            const float u = __fmul_rn(__builtin_nontemporal_load(ps[d] + p), inv_h);
            const float fl = floorf(u);
            c[d].f = u - fl;
            int m = (int)fl % n_mesh;
            m = m < 0 ? m + n_mesh : m;
            c[d].m = min(max(m, 0), n_mesh - 1);
        }
        const int lx = c[0].m % tg.tx, ly = c[1].m % tg.ty, lz = c[2].m % tg.tz;
        const long tile = ((long)(c[0].m / tg.tx) * tg.nty + c[1].m / tg.ty) * tg.ntz + c[2].m / tg.tz;
        const int cat = ((lx == tg.tx - 1) ? 4 : 0) | ((ly == tg.ty - 1) ? 2 : 0) | ((lz == tg.tz - 1) ? 1 : 0);
        key = (uint32_t)(tile * 8 + cat);
        const int local = (((lx << tg.ly) + ly) << tg.lz) + lz;
        __builtin_nontemporal_store(key, sb.keys + p);
        store_rec_stream(sb.recs + p, make_float4(__int_as_float(local), c[0].f, c[1].f, c[2].f));
    }
    (void)wave_increment(sb.count, key, valid);
}

// Exclusive scan, phase 1: each block scans 1024 counts (4 per thread) and stores its total.
__global__ void k_scan_blocks(const uint32_t* count, uint32_t* start, uint32_t* block_sums, long nkeys,
                              long kstride, int nblocks) {
    __shared__ uint32_t sh[256];
    const int r = blockIdx.y;
    count += (long)r * kstride;
    start += (long)r * kstride;
    block_sums += (long)r * nblocks;
    const long base = (long)blockIdx.x * 1024 + threadIdx.x * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < nkeys) ? count[base + i] : 0u;
        s += v[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // Hillis-Steele inclusive scan of thread sums
        uint32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = sh[threadIdx.x] - s;  // exclusive prefix of this thread
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < nkeys) start[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 255) block_sums[blockIdx.x] = sh[255];
}

// Phase 2: one block scans the block totals (up to 8192) in place, exclusive.
__global__ void k_scan_totals(uint32_t* block_sums, int nblocks) {
    __shared__ uint32_t sh[1024];
    const int r = blockIdx.y;
    block_sums += (long)r * nblocks;
    const int per = (nblocks + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nblocks) s += block_sums[b0 + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = sh[threadIdx.x] - s;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nblocks) {
            uint32_t v = block_sums[b0 + i];
            block_sums[b0 + i] = run;
            run += v;
        }
}

// Phase 3: add the block offsets; cursor = start; start[nkeys] = total.
__global__ void k_scan_finish(uint32_t* start, uint32_t* cursor, const uint32_t* block_sums,
                              long nkeys, long kstride, int nblocks, uint32_t total) {
    const int r = blockIdx.y;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    start += (long)r * kstride;
    cursor += (long)r * kstride;
    block_sums += (long)r * nblocks;
    if (i < nkeys) {
        uint32_t v = start[i] + block_sums[i / 1024];
        start[i] = v;
        cursor[i] = v;
    } else if (i == nkeys) {
        start[i] = total;
    }
}

__global__ void k_dep_scatter(long npr, SortBufs sb) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const bool valid = p < npr;
    const long gid = (long)r * npr + p;
    uint32_t key = valid ? __builtin_nontemporal_load(sb.keys + gid) : 0u;
    float4 rec = valid ? load_rec_stream(sb.recs + gid) : make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t slot = wave_increment(sb.cursor + (long)r * sb.kstride, key, valid);
    if (valid) sb.sorted[(long)r * npr + slot] = rec;
}

// The 14 (offset d, category range) pairs a tile pulls: from tile M - d, the categories c with
// (c & d) == d, grouped into contiguous runs [c_lo, c_hi).
struct Pull {
    int d, c_lo, c_hi;
};
__constant__ Pull kPulls[14] = {{0, 0, 8}, {4, 4, 8}, {2, 2, 4}, {2, 6, 8}, {1, 1, 2}, {1, 3, 4}, {1, 5, 6},
                                {1, 7, 8}, {6, 6, 8}, {5, 5, 6}, {5, 7, 8}, {3, 3, 4}, {3, 7, 8}, {7, 7, 8}};
// The offsets d of kPulls packed 3 bits each (entry q at bits 3q), for a register lookup.
constexpr unsigned long long pack_pull_offsets() {
    const int d[14] = {0, 4, 2, 2, 1, 1, 1, 1, 6, 5, 5, 3, 3, 7};
    unsigned long long v = 0;
    for (int q = 0; q < 14; ++q) v |= (unsigned long long)d[q] << (3 * q);
    return v;
}
constexpr unsigned long long kPullOffsets = pack_pull_offsets();

// One block per tile: pull the records whose corners reach into the tile, accumulate in LDS,
// write every cell of the tile once as delta = rho * scale + offset.  The 14 record ranges are
// fetched in parallel first, then all threads sweep their concatenation.
__global__ void __launch_bounds__(256) k_dep_tile(TileGeom tg, SortBufs sb, long npr, float* mesh, long row,
                                                  long mesh_bstride, float scale, float offset) {
    // Cell masses accumulate as 32.32 fixed point in 64-bit integers: LDS integer atomics run at
    // tens of times the rate of LDS float atomics on this hardware, and integer sums do not depend
    // on the order of the adds (the deposit is bitwise reproducible).  A CIC weight is rounded to
    // 2^-32; a cell overflows only beyond 2^32 particles.
    extern __shared__ unsigned long long acc[];
    __shared__ uint32_t rb[14], rlen[15];
    const int r = blockIdx.y;
    const long tile = blockIdx.x;
    const int ncell = tg.tx * tg.ty * tg.tz;
    const int tzi = (int)(tile % tg.ntz);
    const int tyi = (int)((tile / tg.ntz) % tg.nty);
    const int txi = (int)(tile / ((long)tg.ntz * tg.nty));
    const uint32_t* start = sb.start + (long)r * sb.kstride;
    const float4* recs = sb.sorted + (long)r * npr;
    // The 14 range bounds are requested first, so that their latency overlaps the LDS clear.
    uint32_t b = 0, e = 0;
    if (threadIdx.x < 14) {
        const Pull pl = kPulls[threadIdx.x];
        const int dx = (pl.d >> 2) & 1, dy = (pl.d >> 1) & 1, dz = pl.d & 1;
        const int sx = txi - dx < 0 ? tg.ntx - 1 : txi - dx;
        const int sy = tyi - dy < 0 ? tg.nty - 1 : tyi - dy;
        const int sz = tzi - dz < 0 ? tg.ntz - 1 : tzi - dz;
        const long src = ((long)sx * tg.nty + sy) * tg.ntz + sz;
        b = start[src * 8 + pl.c_lo];
        e = start[src * 8 + pl.c_hi];
    }
    for (int i = threadIdx.x; i < ncell; i += blockDim.x) acc[i] = 0ull;
    if (threadIdx.x < 64) {  // first wave: exclusive prefix of the range lengths by a lane scan
        const uint32_t len = threadIdx.x < 14 ? e - b : 0u;
        uint32_t inc = len;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off);
            if ((int)threadIdx.x >= off) inc += y;
        }
        if (threadIdx.x < 14) {
            rb[threadIdx.x] = b;
            rlen[threadIdx.x] = inc - len;
        }
        if (threadIdx.x == 13) rlen[14] = inc;
    }
    __syncthreads();
    const uint32_t total = rlen[14];
    uint32_t rl[14];  // range starts in the concatenation (non-decreasing)
#pragma unroll
    for (int k = 0; k < 14; ++k) rl[k] = rlen[k];
    // Each thread sweeps a contiguous chunk of the concatenated records, so that the lanes of a
    // wave work on records far apart in the sorted order: records of one key range are in
    // Lagrangian order, and neighbouring particles hit the same cells -- consecutive records on
    // consecutive lanes would serialise the LDS atomics.
    const uint32_t chunk = (total + blockDim.x - 1) / blockDim.x;
    const uint32_t i0 = threadIdx.x * chunk;
    const uint32_t i1 = min(total, i0 + chunk);
    for (uint32_t i = i0; i < i1; ++i) {
        int q = 0;  // the last range starting at or before i (empty ranges share their start)
#pragma unroll
        for (int k = 1; k < 14; ++k) q += i >= rl[k] ? 1 : 0;
        const int d = (int)((kPullOffsets >> (3 * q)) & 7u);
        const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
        const float4 rec = recs[rb[q] + (i - rlen[q])];
        const int local = __float_as_int(rec.x);
        const int lz = local & (tg.tz - 1), ly = (local >> tg.lz) & (tg.ty - 1), lx = local >> (tg.lz + tg.ly);
        const int hx = lx - dx * tg.tx, hy = ly - dy * tg.ty, hz = lz - dz * tg.tz;
        const float wx[2] = {1.0f - rec.y, rec.y}, wy[2] = {1.0f - rec.z, rec.z}, wz[2] = {1.0f - rec.w, rec.w};
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            const int ux = hx + cx;
            if (ux < 0 || ux >= tg.tx) continue;
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) {
                const int uy = hy + cy;
                if (uy < 0 || uy >= tg.ty) continue;
#pragma unroll
                for (int cz = 0; cz < 2; ++cz) {
                    const int uz = hz + cz;
                    if (uz < 0 || uz >= tg.tz) continue;
                    // clamped at 0: the conversion of a negative weight would wrap to ~2^32
                    atomicAdd(&acc[(((ux << tg.ly) + uy) << tg.lz) + uz],
                              __float2ull_rn(fmaxf(wx[cx] * wy[cy] * wz[cz] * 4294967296.0f, 0.0f)));
                }
            }
        }
    }
    __syncthreads();
    float* out = mesh + (long)r * mesh_bstride;
    const double unit = 2.3283064365386962890625e-10;  // 2^-32
    auto cell = [&](int i) { return fmaf((float)((double)acc[i] * unit), scale, offset); };
    if ((tg.tz & 3) == 0) {  // rows of the tile are whole float4s
        for (int i4 = threadIdx.x; i4 < (ncell >> 2); i4 += blockDim.x) {
            const int i = i4 << 2;
            const int uz = i & (tg.tz - 1), uy = (i >> tg.lz) & (tg.ty - 1), ux = i >> (tg.lz + tg.ly);
            const long gx = (long)txi * tg.tx + ux, gy = (long)tyi * tg.ty + uy, gz = (long)tzi * tg.tz + uz;
            const float4 a = make_float4(cell(i), cell(i + 1), cell(i + 2), cell(i + 3));
            store_rec_stream(reinterpret_cast<float4*>(out + (gx * tg.n + gy) * row + gz), a);
        }
    } else {
        for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
            const int uz = i & (tg.tz - 1), uy = (i >> tg.lz) & (tg.ty - 1), ux = i >> (tg.lz + tg.ly);
            const long gx = (long)txi * tg.tx + ux, gy = (long)tyi * tg.ty + uy, gz = (long)tzi * tg.tz + uz;
            out[(gx * tg.n + gy) * row + gz] = cell(i);
        }
    }
}

}  // namespace

hipError_t scan_counts(const uint32_t* count, uint32_t* start, uint32_t* cursor, uint32_t* block_sums, long nkeys,
                       uint32_t total, hipStream_t st) {
    const int nblocks = (int)((nkeys + 1023) / 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nblocks, 1), dim3(256), 0, st, count, start, block_sums, nkeys, 0L,
                       nblocks);
    hipLaunchKernelGGL(k_scan_totals, dim3(1, 1), dim3(1024), 0, st, block_sums, nblocks);
    hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)((nkeys + 1 + 255) / 256), 1), dim3(256), 0, st, start, cursor,
                       block_sums, nkeys, 0L, nblocks, total);
    return hipGetLastError();
}

size_t sort_bytes(long n_particles_per_real, const TileGeom& tg, int n_real) {
    size_t nkp = (size_t)tg.nkeys + 1;
    size_t nblocks = (size_t)((tg.nkeys + 1023) / 1024);
    size_t per = (size_t)n_particles_per_real * (4 + 16 + 16) + nkp * 4 * 3 + nblocks * 4 + 256 * 6;
    return per * (size_t)n_real + 1024;
}

SortBufs carve_sort(void* base, long npr, const TileGeom& tg, int n_real) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    char* b = static_cast<char*>(base);
    SortBufs s;
    s.kstride = tg.nkeys + 1;
    s.nblocks = (int)((tg.nkeys + 1023) / 1024);
    size_t off = 0;
    s.keys = reinterpret_cast<uint32_t*>(b + off); off = al(off + (size_t)npr * n_real * 4);
    s.recs = reinterpret_cast<float4*>(b + off); off = al(off + (size_t)npr * n_real * 16);
    s.sorted = reinterpret_cast<float4*>(b + off); off = al(off + (size_t)npr * n_real * 16);
    s.count = reinterpret_cast<uint32_t*>(b + off); off = al(off + (size_t)s.kstride * n_real * 4);
    s.start = reinterpret_cast<uint32_t*>(b + off); off = al(off + (size_t)s.kstride * n_real * 4);
    s.cursor = reinterpret_cast<uint32_t*>(b + off); off = al(off + (size_t)s.kstride * n_real * 4);
    s.block_sums = reinterpret_cast<uint32_t*>(b + off);
    return s;
}

namespace {
// Scan of the key counts, scatter of the records into key order, tile accumulation: the passes
// after the binning, shared by the step's deposit and the deposit of absolute positions.
hipError_t sort_and_tile(long npr, int n_real, const TileGeom& tg, const SortBufs& sb, float* mesh, long row,
                         long mesh_bstride, float scale, float offset, hipStream_t st) {
    const dim3 pgrid((unsigned)((npr + 255) / 256), n_real);
    {
        ProfScope ps(PROF_DEP_SORT, st);
        hipLaunchKernelGGL(k_scan_blocks, dim3(sb.nblocks, n_real), dim3(256), 0, st, sb.count, sb.start,
                           sb.block_sums, tg.nkeys, sb.kstride, sb.nblocks);
        hipLaunchKernelGGL(k_scan_totals, dim3(1, n_real), dim3(1024), 0, st, sb.block_sums, sb.nblocks);
        hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)((tg.nkeys + 1 + 255) / 256), n_real), dim3(256), 0, st,
                           sb.start, sb.cursor, sb.block_sums, tg.nkeys, sb.kstride, sb.nblocks,
                           (uint32_t)npr);
        hipLaunchKernelGGL(k_dep_scatter, pgrid, dim3(256), 0, st, npr, sb);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps(PROF_DEP_TILE, st);
        size_t lds = (size_t)tg.tx * tg.ty * tg.tz * sizeof(unsigned long long);
        hipLaunchKernelGGL(k_dep_tile, dim3((unsigned)tg.ntiles, n_real), dim3(256), lds, st, tg, sb, npr, mesh, row,
                           mesh_bstride, scale, offset);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t sorted_deposit_absolute(const float* const pos[3], long n, int n_mesh, float inv_h, const TileGeom& tg,
                                   const SortBufs& sb, float* mesh, long row, float scale, float offset,
                                   hipStream_t st) {
    hipError_t e = launch_fill(reinterpret_cast<float*>(sb.count), sb.kstride, 0.0f, st);
    if (e != hipSuccess) return e;
    {
        ProfScope ps(PROF_DEPOSIT, st);
        hipLaunchKernelGGL(k_dep_bin_abs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos[0], pos[1], pos[2],
                           n, n_mesh, inv_h, tg, sb);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return sort_and_tile(n, 1, tg, sb, mesh, row, 0, scale, offset, st);
}

hipError_t sorted_deposit(const ParticlePtrs& P, long npr, int n_real, const LatticeGeom& dg, bool drift,
                          const LatticeGeom& fg, const float* F, const KickDrift& kd, const TileGeom& tg,
                          const SortBufs& sb, float* mesh, float scale, float offset, hipStream_t st) {
    const dim3 pgrid((unsigned)((npr + 255) / 256), n_real);
    hipError_t e = launch_fill(reinterpret_cast<float*>(sb.count), sb.kstride * n_real, 0.0f, st);
    if (e != hipSuccess) return e;
    {
        ProfScope ps(drift ? PROF_PK_DEPOSIT : PROF_DEPOSIT, st);
        if (drift)
            hipLaunchKernelGGL(k_dep_bin<1>, pgrid, dim3(256), 0, st, P, npr, dg, tg, fg, F, kd, sb);
        else
            hipLaunchKernelGGL(k_dep_bin<0>, pgrid, dim3(256), 0, st, P, npr, dg, tg, fg, F, kd, sb);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sort_and_tile(npr, n_real, tg, sb, mesh, dg.row, dg.mesh_bstride, scale, offset, st);
}

hipError_t gather_kick_drift_bin(const ParticlePtrs& P, long npr, int n_real, const LatticeGeom& fg, const float* F,
                                 const LatticeGeom& dg, const KickDrift& kd, const TileGeom& tg, const SortBufs& sb,
                                 hipStream_t st) {
    hipError_t e = launch_fill(reinterpret_cast<float*>(sb.count), sb.kstride * n_real, 0.0f, st);
    if (e != hipSuccess) return e;
    KickDrift k = kd;
    k.los = -1;
    ProfScope ps(PROF_GKD, st);
    hipLaunchKernelGGL(k_dep_bin<2>, dim3((unsigned)((npr + 255) / 256), n_real), dim3(256), 0, st, P, npr, dg, tg,
                       fg, F, k, sb);
    return hipGetLastError();
}

hipError_t sorted_deposit_binned(long npr, int n_real, const LatticeGeom& dg, const TileGeom& tg, const SortBufs& sb,
                                 float* mesh, float scale, float offset, hipStream_t st) {
    return sort_and_tile(npr, n_real, tg, sb, mesh, dg.row, dg.mesh_bstride, scale, offset, st);
}

}  // namespace cola
