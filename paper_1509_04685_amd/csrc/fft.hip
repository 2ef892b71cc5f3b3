// 3D FFT passes for cubic meshes on gfx950 (Sec. 2.2: one forward and three inverse FFTs per
// particle-mesh force).  Layout: a half spectrum [x][y][kz] of float2 with kz rows padded to nzp
// (a multiple of 16, so rows start on 128-byte lines); the same memory holds the real field as
// [x][y][2 nzp] floats.
//
// Passes (each one HBM read and one write of the array):
//   z: contiguous rows, real <-> half complex via an n/2-point complex FFT plus a split step;
//   y, x: strided columns, a tile of TK adjacent columns per block so that every row access
//         moves TK * 8 contiguous bytes.
// The particle-mesh force fuses the forward x transform, the Green's function and the inverse x
// transform in one pass that writes two outputs, so the full spectrum never goes to HBM.

#include "cola_internal.h"

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

namespace cola {

// ------------------------------------------------------------------ host: plans and geometry

bool fft_size_ok(int n) {
    if (n < 4 || n % 2) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

Mesh3 make_mesh(int n) {
    Mesh3 g;
    g.n = n;
    g.m = n / 2;
    g.nzp = ((g.m + 1) + 15) / 16 * 16;
    return g;
}

FftPlan make_plan(int n, bool reverse) {
    FftPlan p{};
    p.n = n;
    int R;
    if (n % 3 == 0)
        R = (n % 24 == 0) ? 24 : (n % 12 == 0) ? 12 : (n % 6 == 0) ? 6 : 3;
    else
        R = (n % 16 == 0) ? 16 : (n % 8 == 0) ? 8 : (n % 4 == 0) ? 4 : 2;
    p.R = R;
    p.T = n / R;
    int m = n, k = 0;
    while (m % 3 == 0) { p.radix[k++] = 3; m /= 3; }
    while (R % 8 == 0 && m % 8 == 0) { p.radix[k++] = 8; m /= 8; }
    while (R % 4 == 0 && m % 4 == 0) { p.radix[k++] = 4; m /= 4; }
    while (m % 2 == 0) { p.radix[k++] = 2; m /= 2; }
    p.nst = k;
    if (reverse) std::reverse(p.radix, p.radix + k);
    finish_plan(p, 1);
    return p;
}

static int pick_tk(int n, int T) {
    int tk = 16;
    while (tk > 1 && (long)tk * n * 8 > 96 * 1024) tk /= 2;
    while ((long)tk * T > 512) tk /= 2;
    while (tk < 64 && tk * T < 256 && (long)(tk * 2) * n * 8 <= 64 * 1024) tk *= 2;
    return tk;
}

template <class K>
static hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ------------------------------------------------------------------ twiddles

__global__ void k_twiddles(float2* tw, int len) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s, c;
    sincospi(2.0 * (double)i / (double)len, &s, &c);
    tw[i] = make_float2((float)c, (float)(-s));
}

hipError_t launch_twiddles(float2* tw, int len, hipStream_t st) {
    ProfScope ps(PROF_OTHER, st);
    hipLaunchKernelGGL(k_twiddles, dim3((len + 255) / 256), dim3(256), 0, st, tw, len);
    return hipGetLastError();
}

// ------------------------------------------------------------------ z pass: real -> half complex

// Rows of n = 2M reals; output M+1 complex per row.  Z = FFT_M(x_even + i x_odd);
// X_k = (Z_k + conj Z_{M-k})/2 - i W_n^k (Z_k - conj Z_{M-k})/2, k = 0..M.
template <int R>
__global__ void __launch_bounds__(512) k_fft_z_r2c(const float* in, long in_row, long in_bstride,
                                                   float2* out, long out_row, long out_bstride,
                                                   long nrows, FftPlan pl, const float2* tw,
                                                   float pa, float pb) {
    extern __shared__ float2 lds[];
    const int T = pl.T, M = pl.n;
    const int lpb = blockDim.x / T;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const long row = (long)blockIdx.x * lpb + line;
    const bool active = row < nrows;
    in += (long)blockIdx.y * in_bstride;
    out += (long)blockIdx.y * out_bstride;
    float2* L = lds + line * (M + 1);
    float2 v[R];
    if (active) {
        const float2* src = reinterpret_cast<const float2*>(in + row * in_row);
        for_pattern<R>(pl.radix[0], t, T, pl.nr[0], [&](int q, int e) {
            float2 z = src[e];
            v[q] = make_float2(fmaf(z.x, pa, pb), fmaf(z.y, pa, pb));
        });
    }
    fft_line<R, false>(v, pl, L, 1, t, tw, active);
    if (active) for_pattern<R>(pl.radix[pl.nst - 1], t, T, pl.nr[pl.nst - 1], [&](int q, int e) { L[e] = v[q]; });
    __syncthreads();
    if (!active) return;
    float2* dst = out + row * out_row;
#pragma unroll
    for (int u = 0; u < R; ++u) {
        int k = t + u * T;
        float2 zk = L[k];
        float2 zc = cconj(L[k == 0 ? 0 : M - k]);
        float2 e = cscale(cadd(zk, zc), 0.5f);
        float2 d = csub(zk, zc);
        float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // -i d / 2
        dst[k] = cadd(e, cmul(tw[k], o));
    }
    if (t == 0) {
        float2 z0 = L[0];
        dst[M] = make_float2(z0.x - z0.y, 0.0f);
    }
}

// ------------------------------------------------------------------ z pass: half complex -> real

// Z_k = (X_k + conj X_{M-k}) + i conj(W_n^k) (X_k - conj X_{M-k}); x_{2j} + i x_{2j+1} = IFFT_M(Z)_j.
// MUL_IKZ multiplies X by i k_z first (the kz = M Nyquist column becomes 0).
template <int R, bool MUL_IKZ>
__global__ void __launch_bounds__(512) k_fft_z_c2r(const float2* in, long in_row, long in_bstride,
                                                   float* out, long out_row, long out_bstride,
                                                   long nrows, FftPlan pl, const float2* tw,
                                                   float kf, float scale) {
    extern __shared__ float2 lds[];
    const int T = pl.T, M = pl.n;
    const int lpb = blockDim.x / T;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const long row = (long)blockIdx.x * lpb + line;
    const bool active = row < nrows;
    in += (long)blockIdx.y * in_bstride;
    out += (long)blockIdx.y * out_bstride;
    float2* L = lds + line * (M + 1);
    if (active) {
        // issue all R loads of this thread before the first LDS store
        const float2* src = in + row * in_row;
        float2 x[R];
#pragma unroll
        for (int u = 0; u < R; ++u) x[u] = src[t + u * T];
        float2 xm = (t == 0) ? src[M] : make_float2(0.0f, 0.0f);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            int e = t + u * T;
            float2 y = x[u];
            if (MUL_IKZ) {
                float kz = kf * (float)e;
                y = make_float2(-kz * y.y, kz * y.x);
            }
            L[e] = cscale(y, scale);
        }
        if (t == 0) L[M] = MUL_IKZ ? make_float2(0.0f, 0.0f) : cscale(xm, scale);  // kz Nyquist
    }
    __syncthreads();
    float2 v[R];
    if (active) {
        for_pattern<R>(pl.radix[0], t, T, pl.nr[0], [&](int q, int k) {
            float2 xk = L[k];
            float2 xc = cconj(L[M - k]);
            float2 d = cmul(cconj(tw[k]), csub(xk, xc));
            v[q] = make_float2(xk.x + xc.x - d.y, xk.y + xc.y + d.x);  // (xk + xc) + i d
        });
    }
    __syncthreads();
    fft_line<R, true>(v, pl, L, 1, t, tw, active);
    if (!active) return;
    float2* dst = reinterpret_cast<float2*>(out + row * out_row);
    for_pattern<R>(pl.radix[pl.nst - 1], t, T, pl.nr[pl.nst - 1], [&](int q, int e) { dst[e] = v[q]; });
}

// ------------------------------------------------------------------ strided column passes

// Columns of a realization's padded spectrum (offsets fit 32 bits: meshes up to 1536^3).
struct ColGeom {
    int es;           // element stride along the transform axis (float2)
    int inner;        // contiguous columns per outer block
    int outer_stride;
    int nzp;          // columns c are valid when c % nzp < mvalid
    int mvalid;
    int tk;           // columns per tile
    int tiles;        // tiles per outer block
};

// Block b runs on XCD b % 8 (round-robin dispatch); hand each XCD a contiguous run of tiles so
// that neighbouring tiles, which share 128-byte lines when a tile row is narrower than a line,
// meet in the same L2.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ bool col_setup(const ColGeom& cg, int& t, uint32_t& base, int& c) {
    const int ct = threadIdx.x % cg.tk;
    t = threadIdx.x / cg.tk;
    const int blk = xcd_block();
    const int outer = blk / cg.tiles;
    const int tile = blk - outer * cg.tiles;
    c = tile * cg.tk + ct;
    base = (uint32_t)outer * (uint32_t)cg.outer_stride + (uint32_t)c;
    return c < cg.inner && (c % cg.nzp) < cg.mvalid;
}

template <int R, bool INV>
__global__ void __launch_bounds__(512) k_fft_cols(float2* data, long bstride, ColGeom cg, FftPlan pl,
                                                  const float2* tw) {
    extern __shared__ float2 lds[];
    int t, c;
    uint32_t base;
    const bool active = col_setup(cg, t, base, c);
    data += (long)blockIdx.y * bstride;
    const uint32_t es = (uint32_t)cg.es;
    float2 v[R];
    if (active)
        for_pattern<R>(pl.radix[0], t, pl.T, pl.nr[0], [&](int q, int e) { v[q] = data[base + (uint32_t)e * es]; });
    fft_line<R, INV>(v, pl, lds + threadIdx.x % cg.tk, cg.tk, t, tw, active);
    if (!active) return;
    for_pattern<R>(pl.radix[pl.nst - 1], t, pl.T, pl.nr[pl.nst - 1],
                   [&](int q, int e) { data[base + (uint32_t)e * es] = v[q]; });
}

__device__ __forceinline__ int signed_mode(int e, int n) { return e < n / 2 ? e : e - n; }

// Fused x pass of the particle-mesh force.  Columns are (y, kz); the transform axis is x.
// Forward x FFT, V = S / (k^2 n^3) (k = 0 -> 0), then A = IFFT_x[V] and B = IFFT_x[i k_x V]
// (the k_x Nyquist plane of B set to 0).  pf: forward plan; pi: the same radices reversed, so
// the inverse starts from the forward's output pattern without an LDS round trip.
template <int R>
__global__ void __launch_bounds__(512) k_fft_x_green(const float2* S, float2* A, float2* B, long bstride,
                                                     ColGeom cg, FftPlan pf, FftPlan pi,
                                                     const float2* tw, float kf, float gscale) {
    extern __shared__ float2 lds[];
    int t, c;
    uint32_t base;
    const bool active = col_setup(cg, t, base, c);
    const long boff = (long)blockIdx.y * bstride;
    S += boff;
    A += boff;
    B += boff;
    const uint32_t es = (uint32_t)cg.es;
    const int n = pf.n;
    const int yrow = c / cg.nzp;
    const int my = signed_mode(yrow, n), mz = c - yrow * cg.nzp;
    float2* L = lds + threadIdx.x % cg.tk;
    float2 v[R], h[R];
    if (active)
        for_pattern<R>(pf.radix[0], t, pf.T, pf.nr[0], [&](int q, int e) { v[q] = S[base + (uint32_t)e * es]; });
    fft_line<R, false>(v, pf, L, cg.tk, t, tw, active);
    const float kyz2 = (float)(my * my + mz * mz);
    for_pattern<R>(pf.radix[pf.nst - 1], t, pf.T, pf.nr[pf.nst - 1], [&](int q, int e) {
        int mx = signed_mode(e, n);
        float m2 = (float)(mx * mx) + kyz2;
        float gk = (m2 > 0.0f) ? gscale / (kf * kf * m2) : 0.0f;
        v[q] = cscale(v[q], gk);
        float kx = (2 * mx == -n) ? 0.0f : kf * (float)mx;
        h[q] = make_float2(-kx * v[q].y, kx * v[q].x);  // i k_x V
    });
    fft_line<R, true>(v, pi, L, cg.tk, t, tw, active);
    if (active)
        for_pattern<R>(pi.radix[pi.nst - 1], t, pi.T, pi.nr[pi.nst - 1],
                       [&](int q, int e) { A[base + (uint32_t)e * es] = v[q]; });
    fft_line<R, true>(h, pi, L, cg.tk, t, tw, active);
    if (!active) return;
    for_pattern<R>(pi.radix[pi.nst - 1], t, pi.T, pi.nr[pi.nst - 1],
                   [&](int q, int e) { B[base + (uint32_t)e * es] = h[q]; });
}

// y inverse of A giving two outputs: A <- IFFT_y[i k_y A] (Nyquist of k_y set to 0) and
// S <- IFFT_y[A].  Columns are kz within one x plane.
template <int R>
__global__ void __launch_bounds__(512) k_fft_y_split(float2* A, float2* S, long bstride, ColGeom cg,
                                                     FftPlan pl, const float2* tw, float kf) {
    extern __shared__ float2 lds[];
    int t, c;
    uint32_t base;
    const bool active = col_setup(cg, t, base, c);
    const long boff = (long)blockIdx.y * bstride;
    A += boff;
    S += boff;
    const uint32_t es = (uint32_t)cg.es;
    const int n = pl.n;
    float2* L = lds + threadIdx.x % cg.tk;
    float2 v[R], h[R];
    if (active) {
        for_pattern<R>(pl.radix[0], t, pl.T, pl.nr[0], [&](int q, int e) {
            float2 a = A[base + (uint32_t)e * es];
            h[q] = a;
            int my = signed_mode(e, n);
            float ky = (2 * my == -n) ? 0.0f : kf * (float)my;
            v[q] = make_float2(-ky * a.y, ky * a.x);
        });
    }
    fft_line<R, true>(v, pl, L, cg.tk, t, tw, active);
    if (active)
        for_pattern<R>(pl.radix[pl.nst - 1], t, pl.T, pl.nr[pl.nst - 1],
                       [&](int q, int e) { A[base + (uint32_t)e * es] = v[q]; });
    fft_line<R, true>(h, pl, L, cg.tk, t, tw, active);
    if (!active) return;
    for_pattern<R>(pl.radix[pl.nst - 1], t, pl.T, pl.nr[pl.nst - 1],
                   [&](int q, int e) { S[base + (uint32_t)e * es] = h[q]; });
}

// x inverse with a multiplier taken from the full spectrum: W = IFFT_x[M(k) spec].
//   MUL_SCALE: M = scale;  MUL_IK: M = i k_a / k^2 * scale;  MUL_KK: M = k_a k_b / k^2 * scale.
// A factor k_d is zeroed on the Nyquist plane of axis d when it appears to an odd power.
template <int R>
__global__ void __launch_bounds__(512) k_fft_x_mult(const float2* spec, long spec_bstride, float2* W,
                                                    long w_bstride, ColGeom cg, FftPlan pl,
                                                    const float2* tw, int mtype, int ax_a, int ax_b,
                                                    float kf, float scale) {
    extern __shared__ float2 lds[];
    int t, c;
    uint32_t base;
    const bool active = col_setup(cg, t, base, c);
    spec += (long)blockIdx.y * spec_bstride;
    W += (long)blockIdx.y * w_bstride;
    const uint32_t es = (uint32_t)cg.es;
    const int n = pl.n;
    const int yrow = c / cg.nzp;
    const int my = signed_mode(yrow, n);
    const int mzr = c - yrow * cg.nzp;
    const int mz = (2 * mzr == n) ? -mzr : mzr;  // the kz = n/2 column is the Nyquist plane
    float2 v[R];
    if (active) {
        for_pattern<R>(pl.radix[0], t, pl.T, pl.nr[0], [&](int q, int e) {
            float2 x = spec[base + (uint32_t)e * es];
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
    fft_line<R, true>(v, pl, lds + threadIdx.x % cg.tk, cg.tk, t, tw, active);
    if (!active) return;
    for_pattern<R>(pl.radix[pl.nst - 1], t, pl.T, pl.nr[pl.nst - 1],
                   [&](int q, int e) { W[base + (uint32_t)e * es] = v[q]; });
}

// ------------------------------------------------------------------ host launchers

template <int V>
using IntC = std::integral_constant<int, V>;

// Calls f(IntC<R>{}) for the per-thread register count R of a plan.
template <class F>
static hipError_t dispatch_r(int R, F&& f) {
    switch (R) {
        case 2: f(IntC<2>{}); break;
        case 3: f(IntC<3>{}); break;
        case 4: f(IntC<4>{}); break;
        case 6: f(IntC<6>{}); break;
        case 8: f(IntC<8>{}); break;
        case 12: f(IntC<12>{}); break;
        case 16: f(IntC<16>{}); break;
        case 24: f(IntC<24>{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ kernel shapes and autotuning

// Shape of one FFT kernel launch: R values per thread and `width` lines per block (z passes)
// or columns per tile (y/x passes).
struct FftShape {
    int R = 0;
    int width = 0;
};

enum FftKind { FK_Z_R2C = 0, FK_Z_C2R, FK_COLS_Y, FK_COLS_X, FK_X_GREEN, FK_Y_SPLIT, FK_X_MULT, FK_NUM };
static const char* const kFftKindName[FK_NUM] = {"z_r2c", "z_c2r", "cols_y", "cols_x", "x_green",
                                                 "y_split", "x_mult"};

static bool plan_ok(int n, int R) {
    if (R < 2 || n % R) return false;
    if (n % 3 == 0 && R % 3) return false;
    int m = n;
    while (m % 3 == 0) m /= 3;
    int p2 = 1;
    while (R % (p2 * 2) == 0 && p2 < 8) p2 *= 2;
    if (m > 1 && p2 < 2) return false;
    return true;
}

FftPlan make_plan_r(int n, int R, bool reverse) {
    FftPlan p{};
    p.n = n;
    p.R = R;
    p.T = n / R;
    int m = n, k = 0;
    while (m % 3 == 0) { p.radix[k++] = 3; m /= 3; }
    while (R % 8 == 0 && m % 8 == 0) { p.radix[k++] = 8; m /= 8; }
    while (R % 4 == 0 && m % 4 == 0) { p.radix[k++] = 4; m /= 4; }
    while (m % 2 == 0) { p.radix[k++] = 2; m /= 2; }
    p.nst = k;
    if (reverse) std::reverse(p.radix, p.radix + k);
    finish_plan(p, 1);
    return p;
}

static std::vector<int> valid_rs(int n) {
    std::vector<int> out;
    for (int R : {2, 3, 4, 6, 8, 12, 16, 24})
        if (plan_ok(n, R)) out.push_back(R);
    return out;
}

static bool is_z(FftKind k) { return k == FK_Z_R2C || k == FK_Z_C2R; }

// Line length the kernel transforms: n/2 for the z passes, n otherwise.
static int line_len(FftKind k, int n) { return is_z(k) ? n / 2 : n; }

static size_t shape_lds(FftKind k, int n, const FftShape& sh) {
    int L = line_len(k, n);
    return is_z(k) ? (size_t)sh.width * (L + 1) * sizeof(float2) : (size_t)sh.width * L * sizeof(float2);
}

static bool shape_ok(FftKind k, int n, const FftShape& sh) {
    int L = line_len(k, n);
    if (!plan_ok(L, sh.R)) return false;
    long threads = (long)sh.width * (L / sh.R);
    if (threads > 512 || threads < 1) return false;
    return shape_lds(k, n, sh) <= 128 * 1024;
}

static FftShape default_shape(FftKind k, int n) {
    int L = line_len(k, n);
    FftPlan pl = make_plan(L);
    FftShape sh;
    sh.R = pl.R;
    if (is_z(k)) {
        sh.width = std::max(1, 256 / pl.T);
        while ((long)sh.width * pl.T > 512) sh.width /= 2;
    } else {
        sh.width = pick_tk(n, pl.T);
    }
    return sh;
}

namespace {
struct ShapeCache {
    std::mutex mu;
    std::map<std::pair<int, int>, FftShape> tuned;  // (kind, n) -> shape
};
ShapeCache& shape_cache() {
    static ShapeCache c;
    return c;
}
}  // namespace

static FftShape shape_for(FftKind k, int n) {
    ShapeCache& c = shape_cache();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.tuned.find({(int)k, n});
    if (it != c.tuned.end()) return it->second;
    return default_shape(k, n);
}

static FftPlan plan_for(FftKind k, int n, bool reverse = false) {
    return make_plan_r(line_len(k, n), shape_for(k, n).R, reverse);
}

// ------------------------------------------------------------------ launchers

static ColGeom cols_y(const Mesh3& g, int tk) {
    ColGeom cg;
    cg.es = g.nzp;
    cg.inner = g.nzp;
    cg.outer_stride = g.n * g.nzp;
    cg.nzp = g.nzp;
    cg.mvalid = g.m + 1;
    cg.tk = tk;
    cg.tiles = (cg.inner + tk - 1) / tk;
    return cg;
}

static ColGeom cols_x(const Mesh3& g, int tk) {
    ColGeom cg;
    cg.es = g.n * g.nzp;
    cg.inner = g.n * g.nzp;
    cg.outer_stride = 0;
    cg.nzp = g.nzp;
    cg.mvalid = g.m + 1;
    cg.tk = tk;
    cg.tiles = (cg.inner + tk - 1) / tk;
    return cg;
}

static long col_blocks(const ColGeom& cg, const Mesh3& g, bool y_axis) {
    return (y_axis ? (long)g.n : 1L) * cg.tiles;
}

template <bool INV>
static hipError_t run_cols_shape(float2* data, long bstride, const Mesh3& g, bool y_axis, const float2* tw,
                                 int n_real, const FftShape& sh, hipStream_t st) {
    FftPlan pl = make_plan_r(g.n, sh.R, false);
    ColGeom cg = y_axis ? cols_y(g, sh.width) : cols_x(g, sh.width);
    size_t lds = (size_t)sh.width * g.n * sizeof(float2);
    dim3 grid((unsigned)col_blocks(cg, g, y_axis), n_real), block(sh.width * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_cols<decltype(rr)::value, INV>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(INV ? (y_axis ? PROF_Y_INV : PROF_OTHER) : (y_axis ? PROF_Y_FWD : PROF_X_FWD), st, g.n);
        hipLaunchKernelGGL(kern, grid, block, lds, st, data, bstride, cg, pl, tw);
    });
    if (err != hipSuccess) return err;
    return de;
}

template <bool INV>
static hipError_t run_cols(float2* data, long bstride, const Mesh3& g, bool y_axis, const float2* tw,
                           int n_real, hipStream_t st) {
    return run_cols_shape<INV>(data, bstride, g, y_axis, tw, n_real, shape_for(y_axis ? FK_COLS_Y : FK_COLS_X, g.n),
                               st);
}

static hipError_t run_z_r2c_shape(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                                  const Mesh3& g, const float2* tw, int n_real, float pa, float pb,
                                  const FftShape& sh, hipStream_t st) {
    FftPlan pl = make_plan_r(g.m, sh.R, false);
    finish_plan(pl, 2);
    int lpb = sh.width;
    long nrows = (long)g.n * g.n;
    size_t lds = (size_t)lpb * (g.m + 1) * sizeof(float2);
    dim3 grid((unsigned)((nrows + lpb - 1) / lpb), n_real), block(lpb * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_z_r2c<decltype(rr)::value>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_Z_R2C, st, g.n);
        hipLaunchKernelGGL(kern, grid, block, lds, st, in, in_row, in_bstride, out, (long)g.nzp,
                           out_bstride, nrows, pl, tw, pa, pb);
    });
    if (err != hipSuccess) return err;
    return de;
}

static hipError_t run_z_r2c(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                            const Mesh3& g, const float2* tw, int n_real, float pa, float pb, hipStream_t st) {
    return run_z_r2c_shape(in, in_row, in_bstride, out, out_bstride, g, tw, n_real, pa, pb,
                           shape_for(FK_Z_R2C, g.n), st);
}

template <bool MUL>
static hipError_t run_z_c2r_shape(const float2* in, long in_bstride, float* out, long out_row, long out_bstride,
                                  const Mesh3& g, const float2* tw, int n_real, float kf, float scale,
                                  const FftShape& sh, hipStream_t st) {
    FftPlan pl = make_plan_r(g.m, sh.R, false);
    finish_plan(pl, 2);
    int lpb = sh.width;
    long nrows = (long)g.n * g.n;
    size_t lds = (size_t)lpb * (g.m + 1) * sizeof(float2);
    dim3 grid((unsigned)((nrows + lpb - 1) / lpb), n_real), block(lpb * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_z_c2r<decltype(rr)::value, MUL>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_Z_C2R, st, g.n);
        hipLaunchKernelGGL(kern, grid, block, lds, st, in, (long)g.nzp, in_bstride, out, out_row,
                           out_bstride, nrows, pl, tw, kf, scale);
    });
    if (err != hipSuccess) return err;
    return de;
}

template <bool MUL>
static hipError_t run_z_c2r(const float2* in, long in_bstride, float* out, long out_row, long out_bstride,
                            const Mesh3& g, const float2* tw, int n_real, float kf, float scale,
                            hipStream_t st) {
    return run_z_c2r_shape<MUL>(in, in_bstride, out, out_row, out_bstride, g, tw, n_real, kf, scale,
                                shape_for(FK_Z_C2R, g.n), st);
}

static hipError_t run_x_green_shape(float2* S, float2* A, float2* B, long bstride, const Mesh3& g,
                                    const float2* tw, float kf, int n_real, const FftShape& sh, hipStream_t st) {
    FftPlan pf = make_plan_r(g.n, sh.R, false), pi = make_plan_r(g.n, sh.R, true);
    size_t lds = (size_t)sh.width * g.n * sizeof(float2);
    ColGeom cg = cols_x(g, sh.width);
    dim3 grid((unsigned)col_blocks(cg, g, false), n_real), block(sh.width * pf.T);
    float gscale = 1.0f / ((float)g.n * (float)g.n * (float)g.n);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pf.R, [&](auto rr) {
        auto kern = k_fft_x_green<decltype(rr)::value>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_X_GREEN, st, g.n);
        hipLaunchKernelGGL(kern, grid, block, lds, st, S, A, B, bstride, cg, pf, pi, tw, kf, gscale);
    });
    if (err != hipSuccess) return err;
    return de;
}

static hipError_t run_y_split_shape(float2* A, float2* S, long bstride, const Mesh3& g, const float2* tw,
                                    float kf, int n_real, const FftShape& sh, hipStream_t st) {
    FftPlan pl = make_plan_r(g.n, sh.R, false);
    size_t lds = (size_t)sh.width * g.n * sizeof(float2);
    ColGeom cg = cols_y(g, sh.width);
    dim3 grid((unsigned)col_blocks(cg, g, true), n_real), block(sh.width * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_y_split<decltype(rr)::value>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_Y_SPLIT, st, g.n);
        hipLaunchKernelGGL(kern, grid, block, lds, st, A, S, bstride, cg, pl, tw, kf);
    });
    if (err != hipSuccess) return err;
    return de;
}

static hipError_t run_x_mult_shape(const float2* spec, long spec_bstride, float2* work, long work_bstride,
                                   const Mesh3& g, const float2* tw, int n_real, int mtype, int axis_a,
                                   int axis_b, float kf, float scale, const FftShape& sh, hipStream_t st) {
    FftPlan pl = make_plan_r(g.n, sh.R, false);
    size_t lds = (size_t)sh.width * g.n * sizeof(float2);
    ColGeom cg = cols_x(g, sh.width);
    dim3 grid((unsigned)col_blocks(cg, g, false), n_real), block(sh.width * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_x_mult<decltype(rr)::value>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_X_INV_MULT, st, g.n);
        hipLaunchKernelGGL(kern, grid, block, lds, st, spec, spec_bstride, work, work_bstride, cg, pl, tw,
                           mtype, axis_a, axis_b, kf, scale);
    });
    if (err != hipSuccess) return err;
    return de;
}

hipError_t fft_zy_forward(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                          const Mesh3& g, const float2* tw, int n_real, float pa, float pb,
                          hipStream_t st) {
    hipError_t e = run_z_r2c(in, in_row, in_bstride, out, out_bstride, g, tw, n_real, pa, pb, st);
    if (e != hipSuccess) return e;
    return run_cols<false>(out, out_bstride, g, true, tw, n_real, st);
}

hipError_t fft3d_r2c(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                     const Mesh3& g, const float2* tw, int n_real, float pa, float pb, hipStream_t st) {
    hipError_t e = fft_zy_forward(in, in_row, in_bstride, out, out_bstride, g, tw, n_real, pa, pb, st);
    if (e != hipSuccess) return e;
    return run_cols<false>(out, out_bstride, g, false, tw, n_real, st);
}

hipError_t pm_force_from_spectrum(float2* S, float2* A, float2* B, long bstride, const Mesh3& g,
                                  const float2* tw, float kf, int n_real, hipStream_t st) {
    hipError_t e = run_x_green_shape(S, A, B, bstride, g, tw, kf, n_real, shape_for(FK_X_GREEN, g.n), st);
    if (e != hipSuccess) return e;
    e = run_y_split_shape(A, S, bstride, g, tw, kf, n_real, shape_for(FK_Y_SPLIT, g.n), st);
    if (e != hipSuccess) return e;
    e = run_cols<true>(B, bstride, g, true, tw, n_real, st);
    if (e != hipSuccess) return e;
    const long rowf = 2L * g.nzp;
    e = run_z_c2r<false>(B, bstride, reinterpret_cast<float*>(B), rowf, 2 * bstride, g, tw, n_real, kf, 1.0f, st);
    if (e != hipSuccess) return e;
    e = run_z_c2r<false>(A, bstride, reinterpret_cast<float*>(A), rowf, 2 * bstride, g, tw, n_real, kf, 1.0f, st);
    if (e != hipSuccess) return e;
    return run_z_c2r<true>(S, bstride, reinterpret_cast<float*>(S), rowf, 2 * bstride, g, tw, n_real, kf, 1.0f, st);
}

hipError_t fft3d_c2r_mult(const float2* spec, long spec_bstride, float2* work, long work_bstride,
                          float* out, long out_row, long out_bstride, const Mesh3& g, const float2* tw,
                          int n_real, int mtype, int axis_a, int axis_b, float kf, float scale,
                          hipStream_t st) {
    hipError_t e = run_x_mult_shape(spec, spec_bstride, work, work_bstride, g, tw, n_real, mtype, axis_a, axis_b,
                                    kf, scale, shape_for(FK_X_MULT, g.n), st);
    if (e != hipSuccess) return e;
    e = run_cols<true>(work, work_bstride, g, true, tw, n_real, st);
    if (e != hipSuccess) return e;
    return run_z_c2r<false>(work, work_bstride, out, out_row, out_bstride, g, tw, n_real, kf, 1.0f, st);
}

// Times every admissible shape of each FFT kernel at mesh size n on the buffers S, A, B (each at
// least one padded half spectrum of size n; their contents are overwritten) and keeps the fastest
// per kind for the rest of the process.  `report` gets one line per kind.
hipError_t autotune_fft(int n, float2* S, float2* A, float2* B, const float2* tw, hipStream_t st,
                        std::string* report) {
    Mesh3 g = make_mesh(n);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return hipErrorUnknown;
    const float kf = 0.01f;
    hipError_t status = hipSuccess;
    for (int k = 0; k < FK_NUM && status == hipSuccess; ++k) {
        FftKind kind = (FftKind)k;
        int L = line_len(kind, n);
        std::vector<FftShape> cands;
        for (int R : valid_rs(L))
            for (int w : {1, 2, 4, 8, 16, 32, 64}) {
                FftShape sh{R, w};
                if (!shape_ok(kind, n, sh)) continue;
                long threads = (long)w * (L / R);
                if (threads < 64 && w < 64) continue;
                cands.push_back(sh);
            }
        if (cands.empty()) continue;
        auto launch = [&](const FftShape& sh) -> hipError_t {
            switch (kind) {
                case FK_Z_R2C:
                    return run_z_r2c_shape(reinterpret_cast<const float*>(S), 2L * g.nzp, 0, S, 0, g, tw, 1, 1.0f,
                                           0.0f, sh, st);
                case FK_Z_C2R:
                    return run_z_c2r_shape<false>(A, 0, reinterpret_cast<float*>(A), 2L * g.nzp, 0, g, tw, 1, kf,
                                                  1.0f, sh, st);
                case FK_COLS_Y: return run_cols_shape<false>(S, 0, g, true, tw, 1, sh, st);
                case FK_COLS_X: return run_cols_shape<false>(S, 0, g, false, tw, 1, sh, st);
                case FK_X_GREEN: return run_x_green_shape(S, A, B, 0, g, tw, kf, 1, sh, st);
                case FK_Y_SPLIT: return run_y_split_shape(A, S, 0, g, tw, kf, 1, sh, st);
                case FK_X_MULT: return run_x_mult_shape(S, 0, A, 0, g, tw, 1, MUL_IK, 0, 0, kf, 1.0f, sh, st);
                default: return hipErrorInvalidValue;
            }
        };
        float best = 1e30f;
        FftShape best_sh = default_shape(kind, n);
        for (const FftShape& sh : cands) {
            if ((status = launch(sh)) != hipSuccess) break;  // warm-up (and code-object load)
            float tmin = 1e30f;
            for (int rep = 0; rep < 3 && status == hipSuccess; ++rep) {
                (void)hipEventRecord(e0, st);
                status = launch(sh);
                (void)hipEventRecord(e1, st);
                if (hipEventSynchronize(e1) != hipSuccess) status = hipErrorUnknown;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                tmin = std::min(tmin, ms);
            }
            if (status != hipSuccess) break;
            if (tmin < best) {
                best = tmin;
                best_sh = sh;
            }
        }
        if (status != hipSuccess) break;
        {
            ShapeCache& c = shape_cache();
            std::lock_guard<std::mutex> gl(c.mu);
            c.tuned[{k, n}] = best_sh;
        }
        if (report) {
            char line[160];
            std::snprintf(line, sizeof(line), "n=%d %s: R=%d width=%d %.3f ms (%zu shapes)\n", n,
                          kFftKindName[k], best_sh.R, best_sh.width, best, cands.size());
            *report += line;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

// ------------------------------------------------------------------ layout copies

__global__ void k_copy_rows(const float2* src, long src_row, float2* dst, long dst_row, long nrows, int len) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = nrows * len;
    if (i >= total) return;
    long r = i / len;
    int c = (int)(i % len);
    dst[r * dst_row + c] = src[r * src_row + c];
}

hipError_t copy_unpad_to_pad(const float2* src, float2* dst, const Mesh3& g, hipStream_t st) {
    long nrows = (long)g.n * g.n;
    long total = nrows * (g.m + 1);
    ProfScope ps(PROF_COPY, st);
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src,
                       (long)(g.m + 1), dst, (long)g.nzp, nrows, g.m + 1);
    return hipGetLastError();
}

hipError_t copy_pad_to_unpad(const float2* src, float2* dst, const Mesh3& g, hipStream_t st) {
    long nrows = (long)g.n * g.n;
    long total = nrows * (g.m + 1);
    ProfScope ps(PROF_COPY, st);
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src,
                       (long)g.nzp, dst, (long)(g.m + 1), nrows, g.m + 1);
    return hipGetLastError();
}

}  // namespace cola
