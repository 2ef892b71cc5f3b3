// FFT pass kernels, written against a line engine (DynLine: host-built plan, any size;
// StatLine: plan fixed at compile time), and their launch helpers.  Included by fft.hip (the
// host logic and the dynamic instantiations) and by the fft_static_*.hip files (the static
// instantiations for the mesh sizes of the workloads).
//
// Layouts: real fields are [x][y][z] with rows of `row` floats (2 nzp in the workspace meshes, z
// contiguous); the half spectrum is transposed, [kz][x][y] of float2 with y contiguous, so that no
// pass walks an axis at the stride of a whole plane:
//   z: real rows in, one kz plane chunk of W consecutive y out per kz (and the reverse), through
//      an n/2-point complex FFT per row plus a split step; W lines of one x plane per block;
//   y: contiguous complex rows (kz, x) of n values;
//   x: columns at a stride of n values, a tile of TK adjacent y columns of one kz plane per block,
//      so that every row access moves TK * 8 contiguous bytes.
#pragma once

#include "cola_internal.h"

namespace cola {

// ------------------------------------------------------------------ column geometry

// x columns of a realization's transposed spectrum (offsets fit 32 bits: meshes up to 1536^3).
struct ColGeom {
    int es;           // element stride along x (n)
    int inner;        // columns per kz plane (n)
    int plane_stride; // float2 between kz planes (n^2 plus the plane pad)
    int tk;           // columns per tile
    int tiles;        // tiles per plane
};

// Block b runs on XCD b % 8 (round-robin dispatch); hand each XCD a contiguous run of tiles so
// that neighbouring tiles, which share 128-byte lines when a tile row is narrower than a line,
// meet in the same L2.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// TK > 0: columns per tile fixed at compile time (cg.tk is then equal to it).  c: the column (y),
// plane: the kz plane of the block's tile.
template <int TK>
__device__ __forceinline__ bool col_setup(const ColGeom& cg, int& t, uint32_t& base, int& c, int& plane) {
    const int tk = TK > 0 ? TK : cg.tk;
    const int ct = threadIdx.x % tk;
    t = threadIdx.x / tk;
    const int blk = xcd_block();
    plane = blk / cg.tiles;
    const int tile = blk - plane * cg.tiles;
    c = tile * tk + ct;
    base = (uint32_t)plane * (uint32_t)cg.plane_stride + (uint32_t)c;
    return c < cg.inner;
}

__device__ __forceinline__ int signed_mode(int e, int n) { return e < n / 2 ? e : e - n; }

// A column kernel's exchange base in LDS after TW staged twiddles: column ct of the tile at
// element ct (float2, or float when the engine splits its exchanges into real and imaginary parts).
template <class LE>
__device__ __forceinline__ float2* col_lds(float2* lds, int tw_entries, int ct) {
    if constexpr (LE::kSplit) return reinterpret_cast<float2*>(reinterpret_cast<float*>(lds + tw_entries) + ct);
    else return lds + tw_entries + ct;
}

// Launch bound of a column kernel: 512 threads, or 1024 for a compile-time plan whose tile needs
// them (wide tiles of many-thread lines, affordable with the split exchange's half-size LDS).
template <class LE, int TK>
constexpr int col_bound() {
    return (LE::kStatic && TK > 0 && TK * LE::kT > 512) ? 1024 : 512;
}

// ------------------------------------------------------------------ twiddles in LDS

// Table entries a kernel stages at the front of its LDS (0: it reads the global table).  The z
// passes' split steps also read entries 0..M-1.
template <class LE>
constexpr int z_tw_entries() {
    return LE::kTwN > 0 ? (LE::kTwN > LE::kN ? LE::kTwN : LE::kN) : 0;
}
template <class LF, class LI>
constexpr int pair_tw_entries() {
    return LF::kTwN > LI::kTwN ? LF::kTwN : LI::kTwN;
}
constexpr size_t tw_lds_bytes(int entries) { return (size_t)entries * sizeof(float2); }

// Copies the first CNT table entries to lds[0..CNT) and returns the table to read (the caller
// places a barrier before the first read); CNT = 0 returns the global table.
template <int CNT>
__device__ __forceinline__ const float2* stage_twiddles(const float2* tw, float2* lds) {
    if constexpr (CNT == 0) {
        return tw;
    } else {
        for (int i = threadIdx.x; i < CNT; i += blockDim.x) lds[i] = tw[i];
        return lds;
    }
}

// ------------------------------------------------------------------ streaming row access

// Non-temporal loads and stores for the row passes: a block moves data that no other block
// touches (the z c2r time fell by a tenth, 0.66 -> 0.59 ms on 768^3, with both).  The column
// passes keep cached access unless a tile row fills a whole 128-byte line: a 64-byte tile row
// shares its line with the neighbouring tile, which finds it in L2.
__device__ __forceinline__ float2 load_stream(const float2* p) {
    float2 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// Column passes: streaming access only when a tile row fills whole 128-byte lines (16 columns).
template <int TK>
__device__ __forceinline__ float2 load_col(const float2* p) {
    if constexpr (TK >= 16) return load_stream(p);
    else return *p;
}
template <int TK>
__device__ __forceinline__ void store_col(float2* p, float2 v) {
    if constexpr (TK >= 16) store_stream(p, v);
    else *p = v;
}

// ------------------------------------------------------------------ z pass: real -> half complex

// LDS stride of the lines of a z pass block: M + 1 complex values fit a line with its kz Nyquist
// value.  A wave's transposed LDS accesses cover W lines x 64 / W planes k at j stride + k; with M
// a multiple of 32 the stride M + 2 puts half as many of its lanes on one LDS bank pair as M + 1
// does at W = 8 and 16 (4 instead of 8, 2 instead of 4).
__device__ __forceinline__ constexpr int z_line_stride(int M) { return M + 2; }

// Rows of n = 2M reals; output M+1 complex per row.  Z = FFT_M(x_even + i x_odd);
// X_k = (Z_k + conj Z_{M-k})/2 - i W_n^k (Z_k - conj Z_{M-k})/2, k = 0..M.
// Block: W = 2^lw lines (x, y0 .. y0 + W - 1) of one x plane (W divides n); output X_k of line j
// at out[k plane + x n + y0 + j].
template <class LE>
__global__ void __launch_bounds__(512) k_fft_z_r2c(const float* in, long in_row, long in_bstride, float2* out,
                                                   long out_bstride, int n, long plane, int lw, LE eng,
                                                   const float2* tw, float pa, float pb) {
    constexpr int R = LE::kR;
    constexpr int TW = z_tw_entries<LE>();
    extern __shared__ float2 lds[];
    const int T = eng.T(), M = eng.n();
    const int W = 1 << lw;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const long first = (long)blockIdx.x * W;  // line index x n + y of the block's first line
    const int x = (int)(first / n), y0 = (int)(first - (long)x * n);
    in += (long)blockIdx.y * in_bstride;
    out += (long)blockIdx.y * out_bstride;
    float2* const Lb = lds + TW;
    const int LS = z_line_stride(M);
    float2* L = Lb + line * LS;
    float2 v[R];
    const float2* src = reinterpret_cast<const float2*>(in + (first + line) * in_row);
    eng.first(t, [&](int q, int e) {
        float2 z = load_stream(src + e);
        v[q] = make_float2(fmaf(z.x, pa, pb), fmaf(z.y, pa, pb));
    });
    const float2* twl = stage_twiddles<TW>(tw, lds);
    if constexpr (TW > 0) __syncthreads();
    eng.template run<false>(v, L, t, twl, true);
    eng.last(t, [&](int q, int e) { L[e] = v[q]; });
    __syncthreads();
    // split and transposed store: consecutive threads take consecutive lines of one k, so every
    // kz plane receives W contiguous values; R outputs per thread plus the k = M column
    float2* dst = out + (long)x * n + y0;
    const int bd = blockDim.x;
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int o = threadIdx.x + u * bd;
        const int k = o >> lw, j = o & (W - 1);
        const float2* Lj = Lb + j * LS;
        const float2 zk = Lj[k];
        const float2 zc = cconj(Lj[k == 0 ? 0 : M - k]);
        const float2 e = cscale(cadd(zk, zc), 0.5f);
        const float2 d = csub(zk, zc);
        const float2 od = make_float2(0.5f * d.y, -0.5f * d.x);  // -i d / 2
        store_stream(dst + (long)k * plane + j, cadd(e, cmul(twl[k], od)));
    }
    if (threadIdx.x < W) {
        const float2 z0 = Lb[threadIdx.x * LS];
        store_stream(dst + (long)M * plane + threadIdx.x, make_float2(z0.x - z0.y, 0.0f));
    }
}

// ------------------------------------------------------------------ z pass: half complex -> real

// Z_k = (X_k + conj X_{M-k}) + i conj(W_n^k) (X_k - conj X_{M-k}); x_{2j} + i x_{2j+1} = IFFT_M(Z)_j.
// Block: the W = 2^lw lines (x, y0 .. y0 + W - 1) of one x plane; line j reads
// in[k plane + x n + y0 + j] and writes the real row (x, y0 + j).  ghost: the row also gets x_0, x_1
// again at n, n + 1 (rows of at least n + 2 floats).
template <class LE>
__global__ void __launch_bounds__(512) k_fft_z_c2r(const float2* in, long in_bstride, float* out, long out_row,
                                                   long out_bstride, int n, long plane, int lw, int ghost, LE eng,
                                                   const float2* tw, float scale) {
    constexpr int R = LE::kR;
    constexpr int TW = z_tw_entries<LE>();
    extern __shared__ float2 lds[];
    const int T = eng.T(), M = eng.n();
    const int W = 1 << lw;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const long first = (long)blockIdx.x * W;
    const int x = (int)(first / n), y0 = (int)(first - (long)x * n);
    in += (long)blockIdx.y * in_bstride;
    out += (long)blockIdx.y * out_bstride;
    float2* const Lb = lds + TW;
    const int LS = z_line_stride(M);
    const float2* twl = stage_twiddles<TW>(tw, lds);  // visible after the barrier below
    {
        // every load of this thread is issued before the first LDS store
        const float2* src = in + (long)x * n + y0;
        const int bd = blockDim.x;
        float2 xv[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int o = threadIdx.x + u * bd;
            xv[u] = load_stream(src + (long)(o >> lw) * plane + (o & (W - 1)));
        }
        const float2 xm = threadIdx.x < W ? load_stream(src + (long)M * plane + threadIdx.x) : make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int o = threadIdx.x + u * bd;
            const int k = o >> lw, j = o & (W - 1);
            Lb[j * LS + k] = cscale(xv[u], scale);
        }
        if (threadIdx.x < W)  // kz Nyquist plane
            Lb[threadIdx.x * LS + M] = cscale(xm, scale);
    }
    __syncthreads();
    float2* L = Lb + line * LS;
    float2 v[R];
    eng.first(t, [&](int q, int k) {
        float2 xk = L[k];
        float2 xc = cconj(L[M - k]);
        float2 d = cmul(cconj(twl[k]), csub(xk, xc));
        v[q] = make_float2(xk.x + xc.x - d.y, xk.y + xc.y + d.x);  // (xk + xc) + i d
    });
    __syncthreads();
    eng.template run<true>(v, L, t, twl, true);
    float2* dst = reinterpret_cast<float2*>(out + (first + line) * out_row);
    eng.last(t, [&](int q, int e) {
        store_stream(dst + e, v[q]);
        if (ghost && e == 0) store_stream(dst + M, v[q]);
    });
}

// The three force components in one pass, written interleaved: the block's threads form three
// groups of W lines each; group c inverts, as the kernel above does for one spectrum, the spectrum
// of F_x (c = 0: in0), F_y (in1) or F_z (in2, multiplied by i k_z) of the rows (x, y0 .. y0 + W - 1),
// each group in its own LDS area.  Those areas together hold W rows of 3 (n + 2) floats, so after
// the transforms the same LDS is the staging area of the interleaved rows
//   out[(x n + y) out_row + 3 z + c],  z = 0 .. n + 1 (z = n, n + 1 repeat z = 0, 1),
// which the whole block then writes with contiguous stores.  A CIC gather finds the three
// components of a cell pair (z, z + 1) in 24 contiguous bytes instead of three lines of separate
// meshes.
template <class LE>
__global__ void __launch_bounds__(1024) k_fft_z_c2r3(const float2* in0, const float2* in1, const float2* in2,
                                                     long in_bstride, float* out, long out_row, long out_bstride,
                                                     int n, long plane, int lw, LE eng, const float2* tw, float kf,
                                                     float scale) {
    constexpr int R = LE::kR;
    constexpr int TW = z_tw_entries<LE>();
    extern __shared__ float2 lds[];
    const int T = eng.T(), M = eng.n();
    const int W = 1 << lw;
    const int gs = W * T;  // threads per group
    const int comp = threadIdx.x / gs, lt = threadIdx.x - comp * gs;
    const int line = lt / T, t = lt % T;
    // blocks of neighbouring lines meet in one XCD's L2: with W < 16 they share the 128-byte lines
    // of every kz plane
    const long first = (long)xcd_block() * W;
    const int x = (int)(first / n), y0 = (int)(first - (long)x * n);
    float2* const Lb = lds + TW;
    const int LS = z_line_stride(M);  // this group's lines
    float2* const Lg = Lb + (long)comp * W * LS;
    const float2* twl = stage_twiddles<TW>(tw, lds);  // visible after the barrier below
    {
        const float2* src = (comp == 0 ? in0 : (comp == 1 ? in1 : in2)) + (long)blockIdx.y * in_bstride +
                            (long)x * n + y0;
        const uint32_t pl = (uint32_t)plane;
        float2 xv[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {  // k plane + j < (n/2 + 1) plane < 2^31
            const uint32_t o = lt + u * gs;
            xv[u] = load_stream(src + ((o >> lw) * pl + (o & (W - 1))));
        }
        const float2 xm = lt < W ? load_stream(src + (long)M * plane + lt) : make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int o = lt + u * gs;
            const int k = o >> lw, j = o & (W - 1);
            float2 y = xv[u];
            if (comp == 2) {
                const float kz = kf * (float)k;
                y = make_float2(-kz * y.y, kz * y.x);
            }
            Lg[j * LS + k] = cscale(y, scale);
        }
        if (lt < W)  // kz Nyquist plane (0 for the i k_z component)
            Lg[lt * LS + M] = comp == 2 ? make_float2(0.0f, 0.0f) : cscale(xm, scale);
    }
    __syncthreads();
    float2* L = Lg + line * LS;
    float2 v[R];
    eng.first(t, [&](int q, int k) {
        float2 xk = L[k];
        float2 xc = cconj(L[M - k]);
        float2 d = cmul(cconj(twl[k]), csub(xk, xc));
        v[q] = make_float2(xk.x + xc.x - d.y, xk.y + xc.y + d.x);  // (xk + xc) + i d
    });
    __syncthreads();
    eng.template run<true>(v, L, t, twl, true);
    __syncthreads();  // every group's transform is done: the LDS becomes the staging rows
    const int rs = 3 * (2 * M + 2);  // floats per staged row: n + 2 cells of three components
    float* const S = reinterpret_cast<float*>(Lb);
    float* const Sl = S + line * rs + comp;
    eng.last(t, [&](int q, int e) {  // v[q]: cells 2e and 2e + 1 of this component
        Sl[6 * e] = v[q].x;
        Sl[6 * e + 3] = v[q].y;
        if (e == 0) {
            Sl[6 * M] = v[q].x;
            Sl[6 * M + 3] = v[q].y;
        }
    });
    __syncthreads();
    float* dst = out + (long)blockIdx.y * out_bstride + first * out_row;
    const int half = rs / 2;  // float2 per staged row (rs is even)
    for (int j = 0; j < W; ++j)
        for (int h = threadIdx.x; h < half; h += blockDim.x)
            store_stream(reinterpret_cast<float2*>(dst + j * out_row) + h, reinterpret_cast<const float2*>(S + j * rs)[h]);
}

// ------------------------------------------------------------------ y rows

// Complex rows of n contiguous values (the rows (kz, x) of the transposed spectrum), transformed
// in place, W lines per block: OPR 0 forward, 1 inverse, 2 the y inverse of the force: A <-
// IFFT_y[i k_y A] (the k_y Nyquist entry set to 0) and S <- IFFT_y[A].
template <class LE, int OPR>
__global__ void __launch_bounds__(512) k_fft_rows(float2* A, float2* S, long bstride, long nrows, long plane,
                                                  LE eng, const float2* tw, float kf) {
    constexpr int R = LE::kR;
    constexpr int TW = LE::kTwN;
    extern __shared__ float2 lds[];
    const int T = eng.T(), n = eng.n();
    const int W = blockDim.x / T;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const long row = (long)blockIdx.x * W + line;
    const bool active = row < nrows;
    const long kz = row / n;
    const long roff = kz * plane + (row - kz * n) * n;  // row (kz, x) of the transposed spectrum
    A += (long)blockIdx.y * bstride + roff;
    float2* L = lds + TW + line * n;
    float2 v[R], h[R];
    if (active) {
        eng.first(t, [&](int q, int e) {
            const float2 a = load_stream(A + e);
            if constexpr (OPR == 2) {
                h[q] = a;
                const int my = signed_mode(e, n);
                const float ky = (2 * my == -n) ? 0.0f : kf * (float)my;
                v[q] = make_float2(-ky * a.y, ky * a.x);
            } else {
                v[q] = a;
            }
        });
    }
    const float2* twl = stage_twiddles<TW>(tw, lds);
    if constexpr (TW > 0) __syncthreads();
    eng.template run<OPR != 0>(v, L, t, twl, active);
    if (active) eng.last(t, [&](int q, int e) { store_stream(A + e, v[q]); });
    if constexpr (OPR == 2) {
        eng.template run<true>(h, L, t, twl, active);
        if (active) {
            float2* Sd = S + (long)blockIdx.y * bstride + roff;
            eng.last(t, [&](int q, int e) { store_stream(Sd + e, h[q]); });
        }
    }
}

// ------------------------------------------------------------------ x columns

// Forward x transform of every (kz, y) column.
template <class LE, int TK>
__global__ void __launch_bounds__((col_bound<LE, TK>())) k_fft_cols(float2* data, long bstride, ColGeom cg, LE eng, const float2* tw) {
    constexpr int R = LE::kR;
    constexpr int TW = LE::kTwN;
    extern __shared__ float2 lds[];
    int t, c, plane;
    uint32_t base;
    const bool active = col_setup<TK>(cg, t, base, c, plane);
    data += (long)blockIdx.y * bstride;
    const uint32_t es = (uint32_t)cg.es;
    float2 v[R];
    if (active) eng.first(t, [&](int q, int e) { v[q] = load_col<TK>(data + base + (uint32_t)e * es); });
    const float2* twl = stage_twiddles<TW>(tw, lds);
    if constexpr (TW > 0) __syncthreads();
    eng.template run<false>(v, col_lds<LE>(lds, TW, threadIdx.x % (TK > 0 ? TK : cg.tk)), t, twl, active);
    if (!active) return;
    eng.last(t, [&](int q, int e) { store_col<TK>(data + base + (uint32_t)e * es, v[q]); });
}

// T(u) of a Green's-function filter: the cubic Hermite interpolant of its knots (u_j, t_j) with
// slopes m_0 = 0, m_j = (t_{j+1} - t_{j-1}) / (u_{j+1} - u_{j-1}) inside and the one-sided slope at
// the last knot; t_0 below the first knot, t_{n-1} beyond the last.  The slopes come with the
// filter (green_slopes, on the host).
// The piece is found by selects over the knots at fixed indices (the knots past the n-th are padded
// with u = 3e38 by green_slopes), so that the filter stays in scalar registers: indexing it with a
// lane value would copy it to scratch memory.
__device__ __forceinline__ float green_transfer(const GreenFilter& gf, float u) {
    if (u <= gf.u[0]) return gf.t[0];
    if (u >= gf.u_last) return gf.t_last;
    float ua = gf.u[0], ub = gf.u[1], ta = gf.t[0], tb = gf.t[1], ma = gf.m[0], mb = gf.m[1];
#pragma unroll
    for (int j = 2; j < 10; ++j) {
        const bool past = u > gf.u[j - 1];
        ua = past ? gf.u[j - 1] : ua;
        ub = past ? gf.u[j] : ub;
        ta = past ? gf.t[j - 1] : ta;
        tb = past ? gf.t[j] : tb;
        ma = past ? gf.m[j - 1] : ma;
        mb = past ? gf.m[j] : mb;
    }
    const float h = ub - ua;
    const float s = (u - ua) / h, s2 = s * s, s3 = s2 * s;
    return (2.0f * s3 - 3.0f * s2 + 1.0f) * ta + (s3 - 2.0f * s2 + s) * h * ma + (3.0f * s2 - 2.0f * s3) * tb +
           (s3 - s2) * h * mb;
}

// Fused x pass of the particle-mesh force on the (kz, y) columns: forward x FFT,
// V = S / (k^2 n^3) (k = 0 -> 0), then A = IFFT_x[V] and B = IFFT_x[i k_x V] (the k_x Nyquist plane
// of B set to 0).  ef: forward engine; ei: the same radices reversed, so the inverse starts from
// the forward's output pattern without an LDS round trip.
template <class LF, class LI, int TK, bool FILT = false>
__global__ void __launch_bounds__((col_bound<LF, TK>())) k_fft_x_green(const float2* S, float2* A, float2* B, long bstride,
                                                     ColGeom cg, LF ef, LI ei, const float2* tw, float kf,
                                                     float gscale, GreenFilter gf) {
    constexpr int R = LF::kR;
    constexpr int TW = pair_tw_entries<LF, LI>();
    extern __shared__ float2 lds[];
    int t, c, plane;
    uint32_t base;
    const bool active = col_setup<TK>(cg, t, base, c, plane);
    const long boff = (long)blockIdx.y * bstride;
    S += boff;
    A += boff;
    B += boff;
    const uint32_t es = (uint32_t)cg.es;
    const int n = ef.n();
    const int my = signed_mode(c, n), mz = plane;
    float2* L = col_lds<LF>(lds, TW, threadIdx.x % (TK > 0 ? TK : cg.tk));
    float2 v[R], h[R];
    if (active) ef.first(t, [&](int q, int e) { v[q] = load_col<TK>(S + base + (uint32_t)e * es); });
    const float2* twl = stage_twiddles<TW>(tw, lds);
    if constexpr (TW > 0) __syncthreads();
    ef.template run<false>(v, L, t, twl, active);
    const float kyz2 = (float)(my * my + mz * mz);
    const float g0 = gscale / (kf * kf);
    ef.last(t, [&](int q, int e) {
        int mx = signed_mode(e, n);
        float m2 = (float)(mx * mx) + kyz2;
        float gk = (m2 > 0.0f) ? g0 * __builtin_amdgcn_rcpf(m2) : 0.0f;  // hardware reciprocal, 1 ulp
        if constexpr (FILT) gk *= green_transfer(gf, sqrtf(m2) * (2.0f / (float)n));
        v[q] = cscale(v[q], gk);
        float kx = (2 * mx == -n) ? 0.0f : kf * (float)mx;
        h[q] = make_float2(-kx * v[q].y, kx * v[q].x);  // i k_x V
    });
    ei.template run<true>(v, L, t, twl, active);
    if (active) ei.last(t, [&](int q, int e) { store_col<TK>(A + base + (uint32_t)e * es, v[q]); });
    ei.template run<true>(h, L, t, twl, active);
    if (!active) return;
    ei.last(t, [&](int q, int e) { store_col<TK>(B + base + (uint32_t)e * es, h[q]); });
}

// x inverse with a multiplier taken from the full spectrum: W = IFFT_x[M(k) spec].
//   MUL_SCALE: M = scale;  MUL_IK: M = i k_a / k^2 * scale;  MUL_KK: M = k_a k_b / k^2 * scale.
// A factor k_d is zeroed on the Nyquist plane of axis d when it appears to an odd power.
template <class LE, int TK>
__global__ void __launch_bounds__((col_bound<LE, TK>())) k_fft_x_mult(const float2* spec, long spec_bstride, float2* W,
                                                    long w_bstride, ColGeom cg, LE eng, const float2* tw,
                                                    int mtype, int ax_a, int ax_b, float kf, float scale) {
    constexpr int R = LE::kR;
    constexpr int TW = LE::kTwN;
    extern __shared__ float2 lds[];
    int t, c, plane;
    uint32_t base;
    const bool active = col_setup<TK>(cg, t, base, c, plane);
    spec += (long)blockIdx.y * spec_bstride;
    W += (long)blockIdx.y * w_bstride;
    const uint32_t es = (uint32_t)cg.es;
    const int n = eng.n();
    const int my = signed_mode(c, n);
    const int mz = (2 * plane == n) ? -plane : plane;  // the kz = n/2 plane is the Nyquist plane
    float2 v[R];
    if (active) {
        eng.first(t, [&](int q, int e) {
            float2 x = load_col<TK>(spec + base + (uint32_t)e * es);
            const int mx = signed_mode(e, n);
            const int ma = ax_a == 0 ? mx : (ax_a == 1 ? my : mz);
            const int mb = ax_b == 0 ? mx : (ax_b == 1 ? my : mz);
            const float m2 = (float)(mx * mx + my * my + mz * mz);
            float f = scale;
            if (mtype == MUL_IK) {
                const bool nyq = (2 * ma == -n);
                f = (m2 > 0.0f && !nyq) ? scale * (float)ma / (kf * m2) : 0.0f;
                x = make_float2(-f * x.y, f * x.x);
            } else if (mtype == MUL_KK) {
                const bool nyq = (ax_a != ax_b) && ((2 * ma == -n) || (2 * mb == -n));
                f = (m2 > 0.0f && !nyq) ? scale * (float)ma * (float)mb / m2 : 0.0f;
                x = cscale(x, f);
            } else {
                x = cscale(x, f);
            }
            v[q] = x;
        });
    }
    const float2* twl = stage_twiddles<TW>(tw, lds);
    if constexpr (TW > 0) __syncthreads();
    eng.template run<true>(v, col_lds<LE>(lds, TW, threadIdx.x % (TK > 0 ? TK : cg.tk)), t, twl, active);
    if (!active) return;
    eng.last(t, [&](int q, int e) { store_col<TK>(W + base + (uint32_t)e * es, v[q]); });
}

// ------------------------------------------------------------------ launches

enum FftOp {
    OP_Z_R2C = 0, OP_Z_C2R, OP_Z_C2R3,                // z passes (line length n/2)
    OP_ROWS_FWD, OP_ROWS_INV, OP_ROWS_SPLIT,          // y rows
    OP_COLS_FWD, OP_X_GREEN, OP_X_MULT,               // x columns
    OP_X_GREEN_FILT                                   // x_green with a Green's-function filter
};
inline bool is_z_op(FftOp op) { return op <= OP_Z_C2R3; }
inline bool is_rows_op(FftOp op) { return op >= OP_ROWS_FWD && op <= OP_ROWS_SPLIT; }

// Everything one pass launch needs; each op reads its own subset.
struct FftLaunch {
    FftOp op;
    int n = 0;      // line length of the kernel's transform (n/2 for the z passes)
    int R = 0;      // values per thread
    int width = 0;  // lines per block (z, rows) or columns per tile (x)
    bool split = false;  // x columns: exchanges split into real and imaginary parts (static plans)
    bool probe = false;  // static launchers: only report whether the shape exists
    dim3 grid, block;
    size_t lds = 0;
    hipStream_t st = nullptr;
    // z passes
    const float* rin = nullptr;
    float* rout = nullptr;
    const float2* cin = nullptr;
    const float2* cin1 = nullptr;  // z_c2r3: the F_y and F_z spectra (cin: F_x)
    const float2* cin2 = nullptr;
    float2* cout = nullptr;
    long in_row = 0, in_bstride = 0, out_row = 0, out_bstride = 0;
    long plane = 0;  // kz-plane stride of the transposed spectrum (z passes, y rows)
    int mesh_n = 0, lw = 0, ghost = 0;
    float pa = 1.0f, pb = 0.0f;
    // rows: A = d0, S = d1, b0, nrows; columns: x_green (S = c0, A = d0, B = d1), cols (d0),
    // x_mult (spec = c0, W = d0)
    long nrows = 0;
    const float2* c0 = nullptr;
    float2* d0 = nullptr;
    float2* d1 = nullptr;
    long b0 = 0, b1 = 0;
    ColGeom cg{};
    GreenFilter gf{};
    const float2* tw = nullptr;
    float kf = 0.0f, scale = 1.0f;
    int mtype = 0, ax_a = 0, ax_b = 0;
};

template <class K>
inline hipError_t allow_lds_fft(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <class LE>
inline hipError_t go_z_r2c(const FftLaunch& L, LE e) {
    auto kern = k_fft_z_r2c<LE>;
    const size_t lds = L.lds + tw_lds_bytes(z_tw_entries<LE>());
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.rin, L.in_row, L.in_bstride, L.cout, L.out_bstride,
                       L.mesh_n, L.plane, L.lw, e, L.tw, L.pa, L.pb);
    return hipGetLastError();
}

template <class LE>
inline hipError_t go_z_c2r(const FftLaunch& L, LE e) {
    auto kern = k_fft_z_c2r<LE>;
    const size_t lds = L.lds + tw_lds_bytes(z_tw_entries<LE>());
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.cin, L.in_bstride, L.rout, L.out_row, L.out_bstride,
                       L.mesh_n, L.plane, L.lw, L.ghost, e, L.tw, L.scale);
    return hipGetLastError();
}

template <class LE>
inline hipError_t go_z_c2r3(const FftLaunch& L, LE e) {
    auto kern = k_fft_z_c2r3<LE>;
    const size_t lds = L.lds + tw_lds_bytes(z_tw_entries<LE>());
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.cin, L.cin1, L.cin2, L.in_bstride, L.rout, L.out_row,
                       L.out_bstride, L.mesh_n, L.plane, L.lw, e, L.tw, L.kf, L.scale);
    return hipGetLastError();
}

template <class LE, int OPR>
inline hipError_t go_rows(const FftLaunch& L, LE e) {
    auto kern = k_fft_rows<LE, OPR>;
    const size_t lds = L.lds + tw_lds_bytes(LE::kTwN);
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.d0, L.d1, L.b0, L.nrows, L.plane, e, L.tw, L.kf);
    return hipGetLastError();
}

template <class LE, int TK>
inline hipError_t go_cols(const FftLaunch& L, LE e) {
    auto kern = k_fft_cols<LE, TK>;
    const size_t lds = L.lds + tw_lds_bytes(LE::kTwN);
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.d0, L.b0, L.cg, e, L.tw);
    return hipGetLastError();
}

template <class LF, class LI, int TK, bool FILT = false>
inline hipError_t go_x_green(const FftLaunch& L, LF f, LI i) {
    auto kern = k_fft_x_green<LF, LI, TK, FILT>;
    const size_t lds = L.lds + tw_lds_bytes(pair_tw_entries<LF, LI>());
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.c0, L.d0, L.d1, L.b0, L.cg, f, i, L.tw, L.kf, L.scale,
                       L.gf);
    return hipGetLastError();
}

template <class LE, int TK>
inline hipError_t go_x_mult(const FftLaunch& L, LE e) {
    auto kern = k_fft_x_mult<LE, TK>;
    const size_t lds = L.lds + tw_lds_bytes(LE::kTwN);
    if (hipError_t ea = allow_lds_fft(kern, lds); ea != hipSuccess) return ea;
    hipLaunchKernelGGL(kern, L.grid, L.block, lds, L.st, L.c0, L.b0, L.d0, L.b1, L.cg, e, L.tw, L.mtype, L.ax_a,
                       L.ax_b, L.kf, L.scale);
    return hipGetLastError();
}

// Static-plan launchers: x columns of line length N with R values per thread and TK columns per
// tile, y rows of length N, z passes of line length M.
template <int N, int R, int TK, bool SPL = false>
inline hipError_t static_cols_ops(const FftLaunch& L) {
    using F = StatLine<N, R, TK, 1, false, SPL>;
    using I = StatLine<N, R, TK, 1, true, SPL>;
    if (L.probe) return hipSuccess;
    switch (L.op) {
        case OP_COLS_FWD: return go_cols<F, TK>(L, F{});
        case OP_X_GREEN: return go_x_green<F, I, TK>(L, F{}, I{});
        case OP_X_GREEN_FILT: return go_x_green<F, I, TK, true>(L, F{}, I{});
        case OP_X_MULT: return go_x_mult<F, TK>(L, F{});
        default: return hipErrorNotSupported;
    }
}

template <int N, int R>
inline hipError_t static_rows_ops(const FftLaunch& L) {
    using E = StatLine<N, R, 1, 1, false>;
    if (L.probe) return hipSuccess;
    switch (L.op) {
        case OP_ROWS_FWD: return go_rows<E, 0>(L, E{});
        case OP_ROWS_INV: return go_rows<E, 1>(L, E{});
        case OP_ROWS_SPLIT: return go_rows<E, 2>(L, E{});
        default: return hipErrorNotSupported;
    }
}

template <int M, int R>
inline hipError_t static_z_ops(const FftLaunch& L) {
    using E = StatLine<M, R, 1, 2, false>;
    if (L.probe) return hipSuccess;
    switch (L.op) {
        case OP_Z_R2C: return go_z_r2c<E>(L, E{});
        case OP_Z_C2R: return go_z_c2r<E>(L, E{});
        case OP_Z_C2R3: return go_z_c2r3<E>(L, E{});
        default: return hipErrorNotSupported;
    }
}

// Static kernels of the workload mesh sizes (fft_static_<n>.hip): hipErrorNotSupported when the
// file has no kernel of the launch's op, size and shape; with L.probe set nothing is launched.
hipError_t fft_static_1536(const FftLaunch& L);
hipError_t fft_static_768(const FftLaunch& L);
hipError_t fft_static_512(const FftLaunch& L);
hipError_t fft_static_384(const FftLaunch& L);
hipError_t fft_static_288(const FftLaunch& L);
hipError_t fft_static_256(const FftLaunch& L);

}  // namespace cola
