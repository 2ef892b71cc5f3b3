// Kernels of the 2LPT initial conditions (Sec. 2.2, after Crocce, Pueblas & Scoccimarro 2006):
// seeded white noise, the Gaussian field's spectrum, the second-order source and the initial state.
//
// White noise: Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw 2011), key (seed, 0),
// counter (cell index, 0, 0, 0).  The top 24 bits of the first two outputs give the uniforms
// u1 = (r0 >> 40 + 1) 2^-24 in (0, 1] and u2 = (r1 >> 40) 2^-24 in [0, 1), exact in float;
// Box-Muller gives w = sqrt(-2 ln u1) cos(2 pi u2).  Runs sharing a seed share the field
// (Sec. 2.3).

#include "cola_internal.h"

namespace cola {

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__global__ void k_noise(float* w, long n, uint64_t seed) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t c[4] = {(uint64_t)i, 0, 0, 0};
    philox4x64_10(c, seed, 0);
    float u1 = (float)((c[0] >> 40) + 1) * 5.9604644775390625e-8f;  // 2^-24
    float u2 = (float)(c[1] >> 40) * 5.9604644775390625e-8f;
    w[i] = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

hipError_t ic_noise(float* w, int n_part, const uint64_t* seeds, int n_real, long bstride, hipStream_t st) {
    long n = (long)n_part * n_part * n_part;
    for (int r = 0; r < n_real; ++r) {
        ProfScope ps(PROF_IC, st);
        hipLaunchKernelGGL(k_noise, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w + r * bstride, n,
                           seeds[r]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// delta_k = W_k sqrt(P(|k|) N^3 / L^3), P = A k^n_s T_BBKS(k)^2, k = 0 removed.  The spectrum is
// evaluated in float64 per mode and rounded once.
__device__ double bbks_t(double k, double gamma) {
    double q = k / gamma;
    if (q <= 0.0) return 1.0;
    double a = 16.1 * q, b = 5.46 * q, c = 6.71 * q;
    double poly = 1.0 + 3.89 * q + a * a + b * b * b + (c * c) * (c * c);
    return log1p(2.34 * q) / (2.34 * q) * pow(poly, -0.25);
}

// Over the transposed half spectrum [kz][x][y] (kz planes `plane` apart), kz < mvalid = n/2 + 1.
__global__ void k_ic_scale(float2* spec, long bstride, int n, long plane, int mvalid, float kf, double amp,
                           double gamma, double n_s, double norm) {
    const long nn = (long)n * n;
    const long total = nn * mvalid;
    spec += (long)blockIdx.y * bstride;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(i / nn);
        const long rr = i - kz * nn;
        int ky = (int)(rr % n), kx = (int)(rr / n);
        int mx = kx < n / 2 ? kx : kx - n, my = ky < n / 2 ? ky : ky - n;
        double m2 = (double)mx * mx + (double)my * my + (double)kz * kz;
        float2* sp = spec + (long)kz * plane + rr;
        float2 v = *sp;
        if (m2 == 0.0) {
            *sp = make_float2(0.0f, 0.0f);
            continue;
        }
        double k = (double)kf * sqrt(m2);
        double t = bbks_t(k, gamma);
        double pk = amp * pow(k, n_s) * t * t;
        float f = (float)sqrt(pk * norm);
        *sp = make_float2(v.x * f, v.y * f);
    }
}

hipError_t ic_scale_spectrum(float2* spec, long bstride, const Mesh3& g, int n_real, float kf, double amp,
                             double gamma, double n_s, double norm, hipStream_t st) {
    long total = g.total_c();
    long blocks = (total + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    ProfScope ps(PROF_IC, st);
    hipLaunchKernelGGL(k_ic_scale, dim3((unsigned)blocks, n_real), dim3(256), 0, st, spec, bstride, g.n, g.plane,
                       g.m + 1, kf, amp, gamma, n_s, norm);
    return hipGetLastError();
}

// mode 0: s = a b + a c + b c;  mode 1: s -= a^2
__global__ void k_lpt2(float* s, const float* a, const float* b, const float* c, long n, int mode) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        if (mode == 0) {
            float x = a[i], y = b[i], z = c[i];
            s[i] = x * y + x * z + y * z;
        } else {
            float x = a[i];
            s[i] -= x * x;
        }
    }
}

hipError_t lpt2_source(float* s, const float* a, const float* b, const float* c, long n, int mode,
                       hipStream_t st) {
    long blocks = (n + 255) / 256;
    if (blocks > 65535L * 4) blocks = 65535L * 4;
    ProfScope ps(PROF_IC, st);
    hipLaunchKernelGGL(k_lpt2, dim3((unsigned)blocks), dim3(256), 0, st, s, a, b, c, n, mode);
    return hipGetLastError();
}

// x = D1 psi1 + D2 psi2 (displacement from q), p = c1 psi1 + c2 psi2: the particle starts on the
// 2LPT path (c = 0 for the residual momentum of the COLA frame, c = a^2 dD/dt for the full one).
__global__ void k_ic_state(ParticlePtrs P, long n, float d1, float d2, float c1, float c2) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float s1 = P.psi1[d][i], s2 = P.psi2[d][i];
        P.x[d][i] = d1 * s1 + d2 * s2;
        P.p[d][i] = c1 * s1 + c2 * s2;
    }
}

hipError_t ic_set_state(const ParticlePtrs& P, long n, float d1, float d2, float c1, float c2, hipStream_t st) {
    ProfScope ps(PROF_IC, st);
    hipLaunchKernelGGL(k_ic_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, n, d1, d2, c1, c2);
    return hipGetLastError();
}

}  // namespace cola
