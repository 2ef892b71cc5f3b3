// Particle kernels of the COLA particle-mesh step (Sec. 2.2; Eq. 1-2):
//   CIC mass assignment onto the force mesh, CIC interpolation of the interleaved force mesh back
//   to the particles fused with the COLA kick and drift in the frame of the 2LPT trajectories.
//
// Particles are structure-of-arrays in Lagrangian order; the position is never stored as an
// absolute float.  Along each axis the cell coordinate is split into an exact integer part from
// the lattice index and a small float part from the displacement:
//   u = (i * n_mesh) / N_p  +  [ ((i * n_mesh) mod N_p) / N_p + qoff + x * n_mesh / L ],
// so the CIC fraction keeps the precision of the displacement (about 1e-6 cell) even on 1536^3
// meshes where an absolute float coordinate would only resolve 1e-4 cell.

#include "cola_internal.h"
#include "force_gather.h"

namespace cola {

struct Cell {
    int m;    // lower node, wrapped into [0, n)
    float f;  // fraction towards m + 1
};

// 32-bit index arithmetic throughout: i * n_mesh < 1536^2 and a lattice index < 1536^3 < 2^32
// (64-bit divisions are long instruction sequences on this hardware).
__device__ __forceinline__ Cell cell_of(int i, float x, int n_part, int n_mesh, float inv_h, float qoff) {
    const uint32_t a = (uint32_t)i * (uint32_t)n_mesh;
    const int q = (int)(a / (uint32_t)n_part);
    const int rem = (int)(a - (uint32_t)q * (uint32_t)n_part);
    float w = (float)rem / (float)n_part + qoff + x * inv_h;
    float fl = floorf(w);
    Cell c;
    c.f = w - fl;
    int m = (q + (int)fl) % n_mesh;
    m = m < 0 ? m + n_mesh : m;
    c.m = min(max(m, 0), n_mesh - 1);  // a non-finite position still maps inside the mesh
    return c;
}

__device__ __forceinline__ int wrap1(int m, int n) { return m + 1 == n ? 0 : m + 1; }

__device__ __forceinline__ void lagr_index(uint32_t p, int n_part, int& i, int& j, int& l) {
    const uint32_t np = (uint32_t)n_part, np2 = np * np;
    const uint32_t ii = p / np2, r = p - ii * np2, jj = r / np;
    i = (int)ii;
    j = (int)jj;
    l = (int)(r - jj * np);
}

__device__ __forceinline__ void deposit8(float* mesh, long row, int n, const Cell& cx, const Cell& cy,
                                         const Cell& cz) {
    const int xs[2] = {cx.m, wrap1(cx.m, n)}, ys[2] = {cy.m, wrap1(cy.m, n)}, zs[2] = {cz.m, wrap1(cz.m, n)};
    const float wx[2] = {1.0f - cx.f, cx.f}, wy[2] = {1.0f - cy.f, cy.f}, wz[2] = {1.0f - cz.f, cz.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            long r = ((long)xs[a] * n + ys[b]) * row;
            float wab = wx[a] * wy[b];
            atomicAdd(&mesh[r + zs[0]], wab * wz[0]);
            atomicAdd(&mesh[r + zs[1]], wab * wz[1]);
        }
}

// ------------------------------------------------------------------ fills

__global__ void k_fill(float* p, long n, float v) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_d(double* p, long n, double v) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

static unsigned grid_for(long n, int block) {
    long b = (n + block - 1) / block;
    if (b > 65535L * 16) b = 65535L * 16;
    return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_fill(float* p, long n, float v, hipStream_t st) {
    ProfScope ps(PROF_FILL, st);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_d(double* p, long n, double v, hipStream_t st) {
    ProfScope ps(PROF_FILL, st);
    hipLaunchKernelGGL(k_fill_d, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Plain streaming copy (16-byte vectors plus a byte tail): the yardstick for HBM counters.
__global__ void k_copy(const uint4* src, uint4* dst, long n16) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
__global__ void k_copy_tail(const unsigned char* src, unsigned char* dst, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
    long n16 = (long)(bytes / 16);
    long tail = (long)(bytes - (size_t)n16 * 16);
    ProfScope ps(PROF_COPY, st);
    if (n16 > 0)
        hipLaunchKernelGGL(k_copy, dim3(grid_for(n16, 256)), dim3(256), 0, st, static_cast<const uint4*>(src),
                           static_cast<uint4*>(dst), n16);
    if (tail > 0)
        hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, st,
                           static_cast<const unsigned char*>(src) + n16 * 16,
                           static_cast<unsigned char*>(dst) + n16 * 16, tail);
    return hipGetLastError();
}

// ------------------------------------------------------------------ CIC deposit

__global__ void k_deposit_abs(const float* px, const float* py, const float* pz, long n, int n_mesh,
                              float inv_h, long row, float* mesh) {
    long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n) return;
    Cell c[3];
    const float* ps[3] = {px, py, pz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float u = __fmul_rn(ps[d][gid], inv_h);  // rounded, so that u - floor(u) >= 0
        float fl = floorf(u);
        c[d].f = u - fl;
        int m = (int)fl % n_mesh;
        m = m < 0 ? m + n_mesh : m;
        c[d].m = min(max(m, 0), n_mesh - 1);
    }
    deposit8(mesh, row, n_mesh, c[0], c[1], c[2]);
}

hipError_t cic_deposit_absolute(const float* const pos[3], long n, int n_mesh, float inv_h, long row,
                                float* mesh, hipStream_t st) {
    ProfScope ps(PROF_DEPOSIT, st);
    hipLaunchKernelGGL(k_deposit_abs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos[0], pos[1],
                       pos[2], n, n_mesh, inv_h, row, mesh);
    return hipGetLastError();
}

__global__ void k_density_finish(float* mesh, long row, int n, float scale, float offset) {
    long total = (long)n * n * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        long r = i / n;
        int z = (int)(i - r * n);
        float* c = mesh + r * row + z;
        *c = fmaf(*c, scale, offset);
    }
}

// Cells z = 0, 1 (six floats) copied to z = n, n + 1 in every row of an interleaved force mesh.
__global__ void k_mesh_ghosts(float* F, long row, int n, long bstride) {
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;  // row index
    if (r >= (long)n * n) return;
    float* f = F + (long)blockIdx.y * bstride + r * row;
#pragma unroll
    for (int k = 0; k < 6; ++k) f[3L * n + k] = f[k];
}

hipError_t mesh_ghosts(float* F, long row, int n, long bstride, int n_real, hipStream_t st) {
    ProfScope ps(PROF_OTHER, st);
    hipLaunchKernelGGL(k_mesh_ghosts, dim3((unsigned)(((long)n * n + 255) / 256), n_real), dim3(256), 0, st, F, row,
                       n, bstride);
    return hipGetLastError();
}

hipError_t density_finish(float* mesh, long row, int n_mesh, float scale, float offset, hipStream_t st) {
    long total = (long)n_mesh * n_mesh * n_mesh;
    ProfScope ps(PROF_OTHER, st);
    hipLaunchKernelGGL(k_density_finish, dim3(grid_for(total, 256)), dim3(256), 0, st, mesh, row, n_mesh,
                       scale, offset);
    return hipGetLastError();
}

// ------------------------------------------------------------------ gather + kick + drift

__device__ __forceinline__ float bracket(float g, float d1, float d2m, float s1, float s2) {
    return g - d1 * s1 - d2m * s2;
}

// p += kick [g - D1 psi1 - (D2 - D1^2) psi2];  x += p Dr + dD1 psi1 + dD2 psi2.
// Grid: (particle blocks, realizations).  Every particle array is read before the first store, so
// the twelve streaming loads and the eight corner-column loads are in flight together (the arrays of one
// particle set could alias as far as the compiler knows, which would otherwise order them).  The
// particle streams are non-temporal, leaving L2 to the force-mesh lines that neighbouring
// particles share.
__global__ void __launch_bounds__(256) k_gather_kick_drift(ParticlePtrs P, uint32_t npr, LatticeGeom fg,
                                                           const float* F, KickDrift kd) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npr) return;
    const int r = blockIdx.y;
    const long gid = (long)r * npr + p;
    float x[3], pv[3], s1[3], s2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = __builtin_nontemporal_load(P.x[d] + gid);
    // x first: loads complete in order, so the gather, whose addresses need only x, does not wait
    // for the nine loads below
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pv[d] = __builtin_nontemporal_load(P.p[d] + gid);
        s1[d] = __builtin_nontemporal_load(P.psi1[d] + gid);
        s2[d] = __builtin_nontemporal_load(P.psi2[d] + gid);
    }
    int idx[3];
    lagr_index((uint32_t)p, fg.n_part, idx[0], idx[1], idx[2]);
    Cell c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = cell_of(idx[d], x[d], fg.n_part, fg.n_mesh, fg.inv_h, fg.qoff);
    float g[3];
    gather_interleaved(F + r * fg.mesh_bstride, fg.row, fg.n_mesh, c[0].m, c[1].m, c[2].m, c[0].f, c[1].f, c[2].f,
                       g);
    const bool move = kd.drift != 0.0f || kd.dd1 != 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float pp = pv[d] + kd.kick * bracket(g[d], kd.d1, kd.d2m, s1[d], s2[d]);
        __builtin_nontemporal_store(pp, P.p[d] + gid);
        if (move) __builtin_nontemporal_store(x[d] + pp * kd.drift + kd.dd1 * s1[d] + kd.dd2 * s2[d], P.x[d] + gid);
    }
}

hipError_t gather_kick_drift(const ParticlePtrs& P, long npr, int n_real, const LatticeGeom& fg, const float* F,
                             const KickDrift& kd, hipStream_t st) {
    ProfScope ps((kd.drift != 0.0f || kd.dd1 != 0.0f) ? PROF_GKD : PROF_KICK, st);
    hipLaunchKernelGGL(k_gather_kick_drift, dim3((unsigned)((npr + 255) / 256), n_real), dim3(256), 0, st, P,
                       (uint32_t)npr, fg, F, kd);
    return hipGetLastError();
}

__global__ void k_gather_force(ParticlePtrs P, long npr, int n_real, LatticeGeom fg, const float* F, float* ax,
                               float* ay, float* az) {
    long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= npr * n_real) return;
    long r = gid / npr, p = gid - r * npr;
    int idx[3];
    lagr_index((uint32_t)p, fg.n_part, idx[0], idx[1], idx[2]);
    Cell c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = cell_of(idx[d], P.x[d][gid], fg.n_part, fg.n_mesh, fg.inv_h, fg.qoff);
    float g[3];
    gather_interleaved(F + r * fg.mesh_bstride, fg.row, fg.n_mesh, c[0].m, c[1].m, c[2].m, c[0].f, c[1].f, c[2].f,
                       g);
    ax[gid] = g[0];
    ay[gid] = g[1];
    az[gid] = g[2];
}

hipError_t gather_force(const ParticlePtrs& P, long npr, int n_real, const LatticeGeom& fg, const float* F,
                        float* const acc[3], hipStream_t st) {
    long n = npr * n_real;
    ProfScope ps(PROF_GATHER, st);
    hipLaunchKernelGGL(k_gather_force, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, npr, n_real,
                       fg, F, acc[0], acc[1], acc[2]);
    return hipGetLastError();
}

}  // namespace cola
