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
#include <type_traits>

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
    const bool active = line < lpb && row < nrows;
    in += (long)blockIdx.y * in_bstride;
    out += (long)blockIdx.y * out_bstride;
    float2* L = lds + line * (M + 1);
    float2 v[R];
    const int r0 = pl.radix[0];
    if (active) {
        const float2* src = reinterpret_cast<const float2*>(in + row * in_row);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            int s = q / r0, i = q % r0;
            float2 z = src[pattern_index(s, i, r0, t, T, M)];
            v[q] = make_float2(fmaf(z.x, pa, pb), fmaf(z.y, pa, pb));
        }
    }
    fft_line<R, false>(v, pl, L, 1, t, tw, 2, active);
    const int rl = pl.radix[pl.nst - 1];
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) L[pattern_index(q / rl, q % rl, rl, t, T, M)] = v[q];
    }
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
    const bool active = line < lpb && row < nrows;
    in += (long)blockIdx.y * in_bstride;
    out += (long)blockIdx.y * out_bstride;
    float2* L = lds + line * (M + 1);
    if (active) {
        const float2* src = in + row * in_row;
        for (int e = t; e <= M; e += T) {
            float2 x = src[e];
            if (MUL_IKZ) {
                float kz = (e == M) ? 0.0f : kf * (float)e;
                x = make_float2(-kz * x.y, kz * x.x);
            }
            L[e] = cscale(x, scale);
        }
    }
    __syncthreads();
    float2 v[R];
    const int r0 = pl.radix[0];
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            int k = pattern_index(q / r0, q % r0, r0, t, T, M);
            float2 xk = L[k];
            float2 xc = cconj(L[M - k]);
            float2 d = cmul(cconj(tw[k]), csub(xk, xc));
            v[q] = make_float2(xk.x + xc.x - d.y, xk.y + xc.y + d.x);  // (xk + xc) + i d
        }
    }
    __syncthreads();
    fft_line<R, true>(v, pl, L, 1, t, tw, 2, active);
    if (!active) return;
    const int rl = pl.radix[pl.nst - 1];
    float2* dst = reinterpret_cast<float2*>(out + row * out_row);
#pragma unroll
    for (int q = 0; q < R; ++q) dst[pattern_index(q / rl, q % rl, rl, t, T, M)] = v[q];
}

// ------------------------------------------------------------------ strided column passes

struct ColGeom {
    long es;          // element stride along the transform axis (float2)
    long inner;       // contiguous columns per outer block
    long outer_stride;
    int nzp;          // columns c are valid when c % nzp < mvalid
    int mvalid;
    int tk;           // columns per tile
    long tiles;       // tiles per outer block
};

__device__ __forceinline__ bool col_setup(const ColGeom& cg, int& t, long& base, long& c) {
    const int ct = threadIdx.x % cg.tk;
    t = threadIdx.x / cg.tk;
    const long outer = blockIdx.x / cg.tiles;
    const long tile = blockIdx.x % cg.tiles;
    c = tile * cg.tk + ct;
    base = outer * cg.outer_stride + c;
    return c < cg.inner && (c % cg.nzp) < cg.mvalid;
}

template <int R, bool INV>
__global__ void __launch_bounds__(512) k_fft_cols(float2* data, long bstride, ColGeom cg, FftPlan pl,
                                                   const float2* tw) {
    extern __shared__ float2 lds[];
    int t;
    long base, c;
    const bool active = col_setup(cg, t, base, c);
    data += (long)blockIdx.y * bstride;
    const int T = pl.T, n = pl.n, r0 = pl.radix[0], rl = pl.radix[pl.nst - 1];
    float2 v[R];
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = data[base + (long)pattern_index(q / r0, q % r0, r0, t, T, n) * cg.es];
    }
    fft_line<R, INV>(v, pl, lds + threadIdx.x % cg.tk, cg.tk, t, tw, 1, active);
    if (!active) return;
#pragma unroll
    for (int q = 0; q < R; ++q) data[base + (long)pattern_index(q / rl, q % rl, rl, t, T, n) * cg.es] = v[q];
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
    int t;
    long base, c;
    const bool active = col_setup(cg, t, base, c);
    const long boff = (long)blockIdx.y * bstride;
    S += boff;
    A += boff;
    B += boff;
    const int T = pf.T, n = pf.n, r0 = pf.radix[0], rl = pf.radix[pf.nst - 1];
    const int my = signed_mode((int)(c / cg.nzp), n), mz = (int)(c % cg.nzp);
    float2* L = lds + threadIdx.x % cg.tk;
    float2 v[R], h[R];
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = S[base + (long)pattern_index(q / r0, q % r0, r0, t, T, n) * cg.es];
    }
    fft_line<R, false>(v, pf, L, cg.tk, t, tw, 1, active);
    const float kyz2 = (float)(my * my + mz * mz);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        int mx = signed_mode(pattern_index(q / rl, q % rl, rl, t, T, n), n);
        float m2 = (float)(mx * mx) + kyz2;
        float gk = (m2 > 0.0f) ? gscale / (kf * kf * m2) : 0.0f;
        v[q] = cscale(v[q], gk);
        float kx = (2 * mx == -n) ? 0.0f : kf * (float)mx;
        h[q] = make_float2(-kx * v[q].y, kx * v[q].x);  // i k_x V
    }
    fft_line<R, true>(v, pi, L, cg.tk, t, tw, 1, active);
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) A[base + (long)pattern_index(q / r0, q % r0, r0, t, T, n) * cg.es] = v[q];
    }
    fft_line<R, true>(h, pi, L, cg.tk, t, tw, 1, active);
    if (!active) return;
#pragma unroll
    for (int q = 0; q < R; ++q) B[base + (long)pattern_index(q / r0, q % r0, r0, t, T, n) * cg.es] = h[q];
}

// y inverse of A giving two outputs: A <- IFFT_y[i k_y A] (Nyquist of k_y set to 0) and
// S <- IFFT_y[A].  Columns are kz within one x plane.
template <int R>
__global__ void __launch_bounds__(512) k_fft_y_split(float2* A, float2* S, long bstride, ColGeom cg,
                                                      FftPlan pl, const float2* tw, float kf) {
    extern __shared__ float2 lds[];
    int t;
    long base, c;
    const bool active = col_setup(cg, t, base, c);
    const long boff = (long)blockIdx.y * bstride;
    A += boff;
    S += boff;
    const int T = pl.T, n = pl.n, r0 = pl.radix[0], rl = pl.radix[pl.nst - 1];
    float2* L = lds + threadIdx.x % cg.tk;
    float2 v[R], h[R];
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            int e = pattern_index(q / r0, q % r0, r0, t, T, n);
            float2 a = A[base + (long)e * cg.es];
            h[q] = a;
            int my = signed_mode(e, n);
            float ky = (2 * my == -n) ? 0.0f : kf * (float)my;
            v[q] = make_float2(-ky * a.y, ky * a.x);
        }
    }
    fft_line<R, true>(v, pl, L, cg.tk, t, tw, 1, active);
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) A[base + (long)pattern_index(q / rl, q % rl, rl, t, T, n) * cg.es] = v[q];
    }
    fft_line<R, true>(h, pl, L, cg.tk, t, tw, 1, active);
    if (!active) return;
#pragma unroll
    for (int q = 0; q < R; ++q) S[base + (long)pattern_index(q / rl, q % rl, rl, t, T, n) * cg.es] = h[q];
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
    int t;
    long base, c;
    const bool active = col_setup(cg, t, base, c);
    spec += (long)blockIdx.y * spec_bstride;
    W += (long)blockIdx.y * w_bstride;
    const int T = pl.T, n = pl.n, r0 = pl.radix[0], rl = pl.radix[pl.nst - 1];
    const int my = signed_mode((int)(c / cg.nzp), n);
    const int mzr = (int)(c % cg.nzp);
    const int mz = (2 * mzr == n) ? -mzr : mzr;  // the kz = n/2 column is the Nyquist plane
    float2 v[R];
    if (active) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            int e = pattern_index(q / r0, q % r0, r0, t, T, n);
            float2 x = spec[base + (long)e * cg.es];
            int m[3] = {signed_mode(e, n), my, mz};
            float m2 = (float)(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            float f = scale;
            if (mtype == MUL_IK) {
                bool nyq = (2 * m[ax_a] == -n);
                f = (m2 > 0.0f && !nyq) ? scale * (float)m[ax_a] / (kf * m2) : 0.0f;
                x = make_float2(-f * x.y, f * x.x);
            } else if (mtype == MUL_KK) {
                bool nyq = (ax_a != ax_b) && ((2 * m[ax_a] == -n) || (2 * m[ax_b] == -n));
                f = (m2 > 0.0f && !nyq) ? scale * (float)m[ax_a] * (float)m[ax_b] / m2 : 0.0f;
                x = cscale(x, f);
            } else {
                x = cscale(x, f);
            }
            v[q] = x;
        }
    }
    fft_line<R, true>(v, pl, lds + threadIdx.x % cg.tk, cg.tk, t, tw, 1, active);
    if (!active) return;
#pragma unroll
    for (int q = 0; q < R; ++q) W[base + (long)pattern_index(q / rl, q % rl, rl, t, T, n) * cg.es] = v[q];
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

static ColGeom cols_y(const Mesh3& g, int tk) {
    ColGeom cg;
    cg.es = g.nzp;
    cg.inner = g.nzp;
    cg.outer_stride = (long)g.n * g.nzp;
    cg.nzp = g.nzp;
    cg.mvalid = g.m + 1;
    cg.tk = tk;
    cg.tiles = (cg.inner + tk - 1) / tk;
    return cg;
}

static ColGeom cols_x(const Mesh3& g, int tk) {
    ColGeom cg;
    cg.es = (long)g.n * g.nzp;
    cg.inner = (long)g.n * g.nzp;
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
static hipError_t run_cols(float2* data, long bstride, const Mesh3& g, bool y_axis, const float2* tw,
                           int n_real, hipStream_t st) {
    FftPlan pl = make_plan(g.n);
    int tk = pick_tk(g.n, pl.T);
    ColGeom cg = y_axis ? cols_y(g, tk) : cols_x(g, tk);
    size_t lds = (size_t)tk * g.n * sizeof(float2);
    dim3 grid((unsigned)col_blocks(cg, g, y_axis), n_real), block(tk * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_cols<decltype(rr)::value, INV>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(INV ? (y_axis ? PROF_Y_INV : PROF_OTHER) : (y_axis ? PROF_Y_FWD : PROF_X_FWD), st);
        hipLaunchKernelGGL(kern, grid, block, lds, st, data, bstride, cg, pl, tw);
    });
    if (err != hipSuccess) return err;
    if (de != hipSuccess) return de;
    return hipGetLastError();
}

static hipError_t run_z_r2c(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                            const Mesh3& g, const float2* tw, int n_real, float pa, float pb,
                            hipStream_t st) {
    FftPlan pl = make_plan(g.m);
    int lpb = std::max(1, 256 / pl.T);
    long nrows = (long)g.n * g.n;
    size_t lds = (size_t)lpb * (g.m + 1) * sizeof(float2);
    dim3 grid((unsigned)((nrows + lpb - 1) / lpb), n_real), block(lpb * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_z_r2c<decltype(rr)::value>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_Z_R2C, st);
        hipLaunchKernelGGL(kern, grid, block, lds, st, in, in_row, in_bstride, out, (long)g.nzp,
                           out_bstride, nrows, pl, tw, pa, pb);
    });
    if (err != hipSuccess) return err;
    if (de != hipSuccess) return de;
    return hipGetLastError();
}

template <bool MUL>
static hipError_t run_z_c2r(const float2* in, long in_bstride, float* out, long out_row, long out_bstride,
                            const Mesh3& g, const float2* tw, int n_real, float kf, float scale,
                            hipStream_t st) {
    FftPlan pl = make_plan(g.m);
    int lpb = std::max(1, 256 / pl.T);
    long nrows = (long)g.n * g.n;
    size_t lds = (size_t)lpb * (g.m + 1) * sizeof(float2);
    dim3 grid((unsigned)((nrows + lpb - 1) / lpb), n_real), block(lpb * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_z_c2r<decltype(rr)::value, MUL>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_Z_C2R, st);
        hipLaunchKernelGGL(kern, grid, block, lds, st, in, (long)g.nzp, in_bstride, out, out_row,
                           out_bstride, nrows, pl, tw, kf, scale);
    });
    if (err != hipSuccess) return err;
    if (de != hipSuccess) return de;
    return hipGetLastError();
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
    FftPlan pf = make_plan(g.n), pi = make_plan(g.n, true);
    int tk = pick_tk(g.n, pf.T);
    size_t lds = (size_t)tk * g.n * sizeof(float2);
    {
        ColGeom cg = cols_x(g, tk);
        dim3 grid((unsigned)col_blocks(cg, g, false), n_real), block(tk * pf.T);
        float gscale = 1.0f / ((float)g.n * (float)g.n * (float)g.n);
        hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pf.R, [&](auto rr) {
            auto kern = k_fft_x_green<decltype(rr)::value>;
            if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
            ProfScope ps(PROF_X_GREEN, st);
            hipLaunchKernelGGL(kern, grid, block, lds, st, S, A, B, bstride, cg, pf, pi, tw, kf, gscale);
        });
    if (err != hipSuccess) return err;
    if (de != hipSuccess) return de;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        ColGeom cg = cols_y(g, tk);
        dim3 grid((unsigned)col_blocks(cg, g, true), n_real), block(tk * pf.T);
        hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pf.R, [&](auto rr) {
            auto kern = k_fft_y_split<decltype(rr)::value>;
            if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
            ProfScope ps(PROF_Y_SPLIT, st);
            hipLaunchKernelGGL(kern, grid, block, lds, st, A, S, bstride, cg, pf, tw, kf);
        });
    if (err != hipSuccess) return err;
    if (de != hipSuccess) return de;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e = run_cols<true>(B, bstride, g, true, tw, n_real, st);
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
    FftPlan pl = make_plan(g.n);
    int tk = pick_tk(g.n, pl.T);
    size_t lds = (size_t)tk * g.n * sizeof(float2);
    ColGeom cg = cols_x(g, tk);
    dim3 grid((unsigned)col_blocks(cg, g, false), n_real), block(tk * pl.T);
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(pl.R, [&](auto rr) {
        auto kern = k_fft_x_mult<decltype(rr)::value>;
        if (hipError_t ea = allow_lds(kern, lds); ea != hipSuccess) { err = ea; return; }
        ProfScope ps(PROF_X_INV_MULT, st);
        hipLaunchKernelGGL(kern, grid, block, lds, st, spec, spec_bstride, work, work_bstride, cg, pl, tw,
                           mtype, axis_a, axis_b, kf, scale);
    });
    if (err != hipSuccess) return err;
    if (de != hipSuccess) return de;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = run_cols<true>(work, work_bstride, g, true, tw, n_real, st);
    if (e != hipSuccess) return e;
    return run_z_c2r<false>(work, work_bstride, out, out_row, out_bstride, g, tw, n_real, kf, 1.0f, st);
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
