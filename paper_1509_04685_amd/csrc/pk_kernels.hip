// Matter power-spectrum binning (Sec. 2.5): |delta_k|^2 with the CIC window divided out,
// averaged over integer |m| shells; float64 sums.
//
// Bin b >= 1 holds the modes with b^2 <= |m|^2 < (b+1)^2, decided on integers so that every
// implementation bins a mode identically; k = 0 is excluded.  Each half-spectrum mode counts
// twice (itself and its mirror) except on the kz = 0 and kz = n/2 planes.  The spectrum is the
// transposed half spectrum [kz][x][y] of the FFT passes.

#include "cola_internal.h"

namespace cola {

constexpr int kMaxBinsLds = 1024;

__device__ __forceinline__ int isqrt_floor(long v) {
    int b = (int)sqrtf((float)v);
    while ((long)b * b > v) --b;
    while ((long)(b + 1) * (b + 1) <= v) ++b;
    return b;
}

__device__ __forceinline__ float sinc_pi(float x) {  // sin(pi x) / (pi x)
    return x == 0.0f ? 1.0f : sinpif(x) / (3.14159265358979323846f * x);
}

__global__ void k_pk_bin(const float2* spec, long bstride, int n, long plane, int n_bins, double* ksum,
                         double* psum, double* cnt, double kf) {
    __shared__ double sk[kMaxBinsLds], sp[kMaxBinsLds], sc[kMaxBinsLds];
    const bool use_lds = n_bins <= kMaxBinsLds;
    if (use_lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) sk[b] = sp[b] = sc[b] = 0.0;
    __syncthreads();
    const int r = blockIdx.y;
    spec += (long)r * bstride;
    ksum += (long)r * n_bins;
    psum += (long)r * n_bins;
    cnt += (long)r * n_bins;
    const int m = n / 2;
    const long total = (long)n * n * (m + 1);
    const float inv_n = 1.0f / (float)n;
    const long nn = (long)n * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(i / nn);  // transposed spectrum [kz][x][y], planes `plane` apart
        const long rr = i - kz * nn;
        int ky = (int)(rr % n), kx = (int)(rr / n);
        int mx = kx < m ? kx : kx - n, my = ky < m ? ky : ky - n;
        long m2 = (long)mx * mx + (long)my * my + (long)kz * kz;
        if (m2 == 0) continue;
        int b = isqrt_floor(m2);
        if (b >= n_bins) continue;
        float2 d = spec[(long)kz * plane + rr];
        float w1 = sinc_pi(mx * inv_n) * sinc_pi(my * inv_n) * sinc_pi(kz * inv_n);
        float w2 = w1 * w1;
        float pw = (d.x * d.x + d.y * d.y) / (w2 * w2);
        double wt = (kz == 0 || kz == m) ? 1.0 : 2.0;
        double kk = kf * sqrt((double)m2);
        if (use_lds) {
            atomicAdd(&sk[b], wt * kk);
            atomicAdd(&sp[b], wt * (double)pw);
            atomicAdd(&sc[b], wt);
        } else {
            atomicAdd(&ksum[b], wt * kk);
            atomicAdd(&psum[b], wt * (double)pw);
            atomicAdd(&cnt[b], wt);
        }
    }
    __syncthreads();
    if (use_lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) {
            if (sc[b] != 0.0) {
                atomicAdd(&ksum[b], sk[b]);
                atomicAdd(&psum[b], sp[b]);
                atomicAdd(&cnt[b], sc[b]);
            }
        }
}

hipError_t pk_bin(const float2* spec, long bstride, const Mesh3& g, int n_real, int n_bins, double* ksum,
                  double* psum, double* cnt, double kf, hipStream_t st) {
    long total = (long)g.n * g.n * (g.m + 1);
    long blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    ProfScope ps(PROF_PK, st);
    hipLaunchKernelGGL(k_pk_bin, dim3((unsigned)blocks, n_real), dim3(256), 0, st, spec, bstride, g.n, g.plane,
                       n_bins, ksum, psum, cnt, kf);
    return hipGetLastError();
}

// Multipoles about the line of sight `los` (Sec. 6): the same shells, each mode weighted by the
// Legendre polynomials L_2(mu) = (3 mu^2 - 1) / 2 and L_4(mu) = (35 mu^4 - 30 mu^2 + 3) / 8 of
// mu = m_los / |m| (mu^2 from integers, so it is exact up to one division).
__global__ void k_pk_bin_ell(const float2* spec, long bstride, int n, long plane, int n_bins, int los, double* ksum,
                             double* p0, double* p2, double* p4, double* cnt, double kf) {
    __shared__ double sk[kMaxBinsLds], s0[kMaxBinsLds], s2[kMaxBinsLds], s4[kMaxBinsLds], sc[kMaxBinsLds];
    const bool use_lds = n_bins <= kMaxBinsLds;
    if (use_lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) sk[b] = s0[b] = s2[b] = s4[b] = sc[b] = 0.0;
    __syncthreads();
    const int r = blockIdx.y;
    spec += (long)r * bstride;
    ksum += (long)r * n_bins;
    p0 += (long)r * n_bins;
    p2 += (long)r * n_bins;
    p4 += (long)r * n_bins;
    cnt += (long)r * n_bins;
    const int m = n / 2;
    const long total = (long)n * n * (m + 1);
    const float inv_n = 1.0f / (float)n;
    const long nn = (long)n * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(i / nn);  // transposed spectrum [kz][x][y], planes `plane` apart
        const long rr = i - kz * nn;
        int ky = (int)(rr % n), kx = (int)(rr / n);
        int mx = kx < m ? kx : kx - n, my = ky < m ? ky : ky - n;
        long m2 = (long)mx * mx + (long)my * my + (long)kz * kz;
        if (m2 == 0) continue;
        int b = isqrt_floor(m2);
        if (b >= n_bins) continue;
        float2 d = spec[(long)kz * plane + rr];
        float w1 = sinc_pi(mx * inv_n) * sinc_pi(my * inv_n) * sinc_pi(kz * inv_n);
        float w2 = w1 * w1;
        const double pw = (double)((d.x * d.x + d.y * d.y) / (w2 * w2));
        const int ml = los == 0 ? mx : (los == 1 ? my : kz);
        const double mu2 = (double)((long)ml * ml) / (double)m2;
        const double l2 = 1.5 * mu2 - 0.5, l4 = (35.0 * mu2 * mu2 - 30.0 * mu2 + 3.0) * 0.125;
        double wt = (kz == 0 || kz == m) ? 1.0 : 2.0;
        double kk = kf * sqrt((double)m2);
        if (use_lds) {
            atomicAdd(&sk[b], wt * kk);
            atomicAdd(&s0[b], wt * pw);
            atomicAdd(&s2[b], wt * pw * l2);
            atomicAdd(&s4[b], wt * pw * l4);
            atomicAdd(&sc[b], wt);
        } else {
            atomicAdd(&ksum[b], wt * kk);
            atomicAdd(&p0[b], wt * pw);
            atomicAdd(&p2[b], wt * pw * l2);
            atomicAdd(&p4[b], wt * pw * l4);
            atomicAdd(&cnt[b], wt);
        }
    }
    __syncthreads();
    if (use_lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) {
            if (sc[b] != 0.0) {
                atomicAdd(&ksum[b], sk[b]);
                atomicAdd(&p0[b], s0[b]);
                atomicAdd(&p2[b], s2[b]);
                atomicAdd(&p4[b], s4[b]);
                atomicAdd(&cnt[b], sc[b]);
            }
        }
}

hipError_t pk_bin_multipoles(const float2* spec, long bstride, const Mesh3& g, int n_real, int n_bins, int los,
                             double* ksum, double* p0, double* p2, double* p4, double* cnt, double kf,
                             hipStream_t st) {
    long total = (long)g.n * g.n * (g.m + 1);
    long blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    ProfScope ps(PROF_PK, st);
    hipLaunchKernelGGL(k_pk_bin_ell, dim3((unsigned)blocks, n_real), dim3(256), 0, st, spec, bstride, g.n, g.plane,
                       n_bins, los, ksum, p0, p2, p4, cnt, kf);
    return hipGetLastError();
}

__global__ void k_pk_finish_ell(double* kmean, double* p0, double* p2, double* p4, const double* cnt, long n,
                                double pnorm) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = cnt[i];
    const double s = c > 0.0 ? pnorm / c : 0.0;
    kmean[i] = c > 0.0 ? kmean[i] / c : 0.0;
    p0[i] = p0[i] * s;
    p2[i] = 5.0 * p2[i] * s;
    p4[i] = 9.0 * p4[i] * s;
}

hipError_t pk_finish_multipoles(double* kmean, double* p0, double* p2, double* p4, const double* cnt, long n,
                                double pnorm, hipStream_t st) {
    ProfScope ps(PROF_PK, st);
    hipLaunchKernelGGL(k_pk_finish_ell, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kmean, p0, p2, p4, cnt,
                       n, pnorm);
    return hipGetLastError();
}

// k_mean = ksum / cnt, pk = psum / cnt * pnorm (pnorm = L^3 / n^6), zero for empty bins.
__global__ void k_pk_finish(double* kmean, double* pk, const double* cnt, long n, double pnorm) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double c = cnt[i];
    kmean[i] = c > 0.0 ? kmean[i] / c : 0.0;
    pk[i] = c > 0.0 ? pk[i] / c * pnorm : 0.0;
}

hipError_t pk_finish(double* kmean, double* pk, double* cnt, long n, double pnorm, hipStream_t st) {
    ProfScope ps(PROF_PK, st);
    hipLaunchKernelGGL(k_pk_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kmean, pk, cnt, n, pnorm);
    return hipGetLastError();
}

}  // namespace cola
