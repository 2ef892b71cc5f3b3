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

// Each thread takes runs of kPkRun consecutive y of one (kz, x) row: |m| changes slowly along a
// row, so a run's modes mostly share a shell, and a thread adds a shell's sums to LDS only when
// the shell changes (one set of atomics per shell and run instead of per mode).
constexpr int kPkRun = 8;

// LDS: the bins are summed in LDS first (n_bins <= kMaxBinsLds).  A compile-time choice: with the
// target picked at run time the sums went through generic-address (flat) atomics even for LDS.
template <bool LDS>
__global__ void k_pk_bin(const float2* spec, long bstride, int n, long plane, int n_bins, double* ksum,
                         double* psum, double* cnt, double kf) {
    __shared__ double sk[LDS ? kMaxBinsLds : 1], sp[LDS ? kMaxBinsLds : 1], sc[LDS ? kMaxBinsLds : 1];
    if (LDS)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) sk[b] = sp[b] = sc[b] = 0.0;
    __syncthreads();
    const int r = blockIdx.y;
    spec += (long)r * bstride;
    ksum += (long)r * n_bins;
    psum += (long)r * n_bins;
    cnt += (long)r * n_bins;
    double* dk = LDS ? sk : ksum;
    double* dp = LDS ? sp : psum;
    double* dc = LDS ? sc : cnt;
    const int m = n / 2;
    const int runs = (n + kPkRun - 1) / kPkRun;  // runs per row
    const long total = (long)(m + 1) * n * runs;
    const float inv_n = 1.0f / (float)n;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (long)gridDim.x * blockDim.x) {
        const long row = c / runs;  // (kz, x): transposed spectrum [kz][x][y], planes `plane` apart
        const int y0 = (int)(c - row * runs) * kPkRun;
        const int kz = (int)(row / n), kx = (int)(row - (long)kz * n);
        const int mx = kx < m ? kx : kx - n;
        const long mxz = (long)mx * mx + (long)kz * kz;
        const float wxz = sinc_pi(mx * inv_n) * sinc_pi(kz * inv_n);
        const double wt = (kz == 0 || kz == m) ? 1.0 : 2.0;
        const float2* src = spec + (long)kz * plane + (long)kx * n;
        int cur = -1;
        double ak = 0.0, ap = 0.0, ac = 0.0;
        for (int q = 0; q < kPkRun; ++q) {
            const int ky = y0 + q;
            if (ky >= n) break;
            const int my = ky < m ? ky : ky - n;
            const long m2 = mxz + (long)my * my;
            const int b = m2 == 0 ? n_bins : isqrt_floor(m2);
            if (b != cur) {
                if (cur >= 0 && cur < n_bins) {
                    atomicAdd(&dk[cur], ak);
                    atomicAdd(&dp[cur], ap);
                    atomicAdd(&dc[cur], ac);
                }
                cur = b;
                ak = ap = ac = 0.0;
            }
            if (b >= n_bins) continue;
            const float2 d = src[ky];
            const float w1 = wxz * sinc_pi(my * inv_n);
            const float w2 = w1 * w1;
            const float pw = (d.x * d.x + d.y * d.y) / (w2 * w2);
            ak += wt * (kf * sqrt((double)m2));
            ap += wt * (double)pw;
            ac += wt;
        }
        if (cur >= 0 && cur < n_bins) {
            atomicAdd(&dk[cur], ak);
            atomicAdd(&dp[cur], ap);
            atomicAdd(&dc[cur], ac);
        }
    }
    __syncthreads();
    if (LDS)
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
    long total = (long)g.n * (g.m + 1) * ((g.n + kPkRun - 1) / kPkRun);
    long blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    ProfScope ps(PROF_PK, st);
    if (n_bins <= kMaxBinsLds)
        hipLaunchKernelGGL(k_pk_bin<true>, dim3((unsigned)blocks, n_real), dim3(256), 0, st, spec, bstride, g.n,
                           g.plane, n_bins, ksum, psum, cnt, kf);
    else
        hipLaunchKernelGGL(k_pk_bin<false>, dim3((unsigned)blocks, n_real), dim3(256), 0, st, spec, bstride, g.n,
                           g.plane, n_bins, ksum, psum, cnt, kf);
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
        // same product order as k_pk_bin (x and z first), so the real-space monopole is P(k)
        float w1 = (sinc_pi(mx * inv_n) * sinc_pi(kz * inv_n)) * sinc_pi(my * inv_n);
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
    ProfScope ps(PROF_OTHER, st);  // a few hundred bins: kept out of the binning kind's per-launch figure
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
    ProfScope ps(PROF_OTHER, st);  // a few hundred bins: kept out of the binning kind's per-launch figure
    hipLaunchKernelGGL(k_pk_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kmean, pk, cnt, n, pnorm);
    return hipGetLastError();
}

// ------------------------------------------------------------------ aliasing correction
//
// Jing (2005), named in Sec. 2.5: for a spectrum that is a power law P ~ k^n_eff near |m|, the
// measured <|delta_m|^2> is C(m) P(|m|) with the CIC aliasing sum
//   C(m) = sum_{|j_d| <= 2} W^2(u) (|u| / |m|)^n_eff,  u = |m| + j n,  W(u) = prod_d sinc^2(pi u_d / n),
// |m| = (|m_x|, |m_y|, |m_z|).  The corrected estimate divides each mode by C instead of W^2, with
// n_eff the bin's local slope, and is iterated from the deconvolved estimate.
//
// C depends on the sorted absolute mode integers (a >= b >= c) only, so it is evaluated once per
// class, (n/2 + 1)(n/2 + 2)(n/2 + 3) / 6 of them (1/24 of the half spectrum), into a table that the
// binning pass reads: 125 images with a log2 and an exp2 each make C an ALU-bound evaluation.

constexpr int kAliasImages = 2;
constexpr double kSlopeWindow = 1.35;  // the slope of bin b fits the bins with k_b / 1.35 <= k <= 1.35 k_b

__host__ __device__ __forceinline__ long tet_index(long a, long b, long c) {  // a >= b >= c >= 0
    return a * (a + 1) * (a + 2) / 6 + b * (b + 1) / 2 + c;
}

__device__ __forceinline__ void sort3_desc(int& a, int& b, int& c) {
    int t;
    if (a < b) { t = a; a = b; b = t; }
    if (b < c) { t = b; b = c; c = t; }
    if (a < b) { t = a; a = b; b = t; }
}

long pk_alias_scratch_floats(int n, int n_bins) {
    const long h = n / 2;
    const long classes = tet_index(h + 1, 0, 0);
    long bmax = 0;
    while ((bmax + 1) * (bmax + 1) <= 3 * h * h) ++bmax;
    const long nsl = n_bins < bmax + 1 ? n_bins : bmax + 1;
    return ((classes + 63) / 64) * 64 + nsl;
}

// Mode-weighted least-squares slope of ln P on ln k over the non-empty bins within a factor
// kSlopeWindow of k_b, clamped to [-4, 4]; 0 for an empty bin or a window of one bin.  Bins of
// integer shells have k_j in [j kf, (j + 1) kf), which bounds the scan.
__global__ void k_pk_slopes(const double* kmean, const double* pk, const double* cnt, int n_bins, int nsl, double kf,
                            float* scratch, long sstride, long slope_off) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (b >= nsl) return;
    kmean += (long)r * n_bins;
    pk += (long)r * n_bins;
    cnt += (long)r * n_bins;
    float* slope = scratch + r * sstride + slope_off;
    const double kb = kmean[b];
    if (!(kb > 0.0 && pk[b] > 0.0)) {
        slope[b] = 0.0f;
        return;
    }
    const double lo = kb / kSlopeWindow, hi = kb * kSlopeWindow;
    int j0 = (int)floor(lo / kf) - 2, j1 = (int)floor(hi / kf) + 2;
    if (j0 < 0) j0 = 0;
    if (j1 > n_bins - 1) j1 = n_bins - 1;
    double sw = 0.0, sx = 0.0, sy = 0.0;
    int used = 0;
    for (int j = j0; j <= j1; ++j) {
        const double k = kmean[j], p = pk[j];
        if (!(k > 0.0 && p > 0.0) || k < lo || k > hi) continue;
        sw += cnt[j];
        sx += cnt[j] * log(k);
        sy += cnt[j] * log(p);
        ++used;
    }
    if (used < 2) {
        slope[b] = 0.0f;
        return;
    }
    const double xm = sx / sw, ym = sy / sw;
    double sxy = 0.0, sxx = 0.0;
    for (int j = j0; j <= j1; ++j) {
        const double k = kmean[j], p = pk[j];
        if (!(k > 0.0 && p > 0.0) || k < lo || k > hi) continue;
        const double dx = log(k) - xm;
        sxy += cnt[j] * dx * (log(p) - ym);
        sxx += cnt[j] * dx * dx;
    }
    double s = sxy / sxx;
    s = s < -4.0 ? -4.0 : (s > 4.0 ? 4.0 : s);
    slope[b] = (float)s;
}

// One thread per class (a, b, c), a >= b >= c, of realization blockIdx.y: C for its bin's slope.
__global__ void k_alias_table(int n, int n_bins, int nsl, float* scratch, long sstride, long slope_off) {
    const int h = n / 2;
    const long total = tet_index(h + 1, 0, 0);
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    float* table = scratch + blockIdx.y * sstride;
    const float* slope = table + slope_off;
    // invert t = tet(a) + tri(b) + c
    int a = (int)cbrtf(6.0f * (float)t);
    while (a > 0 && tet_index(a, 0, 0) > t) --a;
    while (tet_index(a + 1, 0, 0) <= t) ++a;
    long rem = t - tet_index(a, 0, 0);
    int b = (int)sqrtf(2.0f * (float)rem);
    while (b > 0 && (long)b * (b + 1) / 2 > rem) --b;
    while ((long)(b + 1) * (b + 2) / 2 <= rem) ++b;
    const int c = (int)(rem - (long)b * (b + 1) / 2);
    const long m2 = (long)a * a + (long)b * b + (long)c * c;
    const int bin = m2 > 0 ? isqrt_floor(m2) : 0;
    if (m2 == 0 || bin >= nsl) {
        table[t] = 1.0f;
        return;
    }
    const float half = 0.5f * slope[bin];
    const float inv_n = 1.0f / (float)n;
    const float pi = 3.14159265358979323846f;
    float s4[3][2 * kAliasImages + 1], u2[3][2 * kAliasImages + 1];
    const int v[3] = {a, b, c};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float sn = sinpif((float)v[d] * inv_n);
        const float s2 = sn * sn;
#pragma unroll
        for (int j = 0; j < 2 * kAliasImages + 1; ++j) {
            const int u = v[d] + (j - kAliasImages) * n;
            const float x = pi * (float)u * inv_n;
            const float q = u == 0 ? 1.0f : s2 / (x * x);
            s4[d][j] = q * q;
            u2[d][j] = (float)u * (float)u;
        }
    }
    const float lm = log2f((float)m2);
    float sum = 0.0f;
#pragma unroll
    for (int jx = 0; jx < 2 * kAliasImages + 1; ++jx)
#pragma unroll
        for (int jy = 0; jy < 2 * kAliasImages + 1; ++jy) {
            const float wxy = s4[0][jx] * s4[1][jy];
            const float axy = u2[0][jx] + u2[1][jy];
#pragma unroll
            for (int jz = 0; jz < 2 * kAliasImages + 1; ++jz) {
                const float a2 = axy + u2[2][jz];
                sum += wxy * s4[2][jz] * exp2f(half * (log2f(a2) - lm));
            }
        }
    table[t] = sum;
}

// The pass of k_pk_bin with |delta|^2 / C(class) per mode; only the power sums (k_mean and the
// mode counts are final from the first estimate).  One mode per thread and step: neighbouring
// lanes take neighbouring y, whose classes sit close together in the table (with k_pk_bin's runs
// of y per thread the table gathers spread over more lines: 1.06 -> 1.37 ms per pass at 768^3).
__global__ void k_pk_bin_alias(const float2* spec, long bstride, int n, long plane, int n_bins, const float* scratch,
                               long sstride, double* psum) {
    __shared__ double sp[kMaxBinsLds];
    const bool use_lds = n_bins <= kMaxBinsLds;
    if (use_lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x) sp[b] = 0.0;
    __syncthreads();
    const int r = blockIdx.y;
    spec += (long)r * bstride;
    psum += (long)r * n_bins;
    const float* table = scratch + r * sstride;
    const int m = n / 2;
    const long total = (long)n * n * (m + 1);
    const long nn = (long)n * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int kz = (int)(i / nn);
        const long rr = i - kz * nn;
        const int ky = (int)(rr % n), kx = (int)(rr / n);
        int ax = kx <= m ? kx : n - kx, ay = ky <= m ? ky : n - ky, az = kz;
        const long m2 = (long)ax * ax + (long)ay * ay + (long)az * az;
        if (m2 == 0) continue;
        const int b = isqrt_floor(m2);
        if (b >= n_bins) continue;
        sort3_desc(ax, ay, az);
        const float2 d = spec[(long)kz * plane + rr];
        const float pw = (d.x * d.x + d.y * d.y) / table[tet_index(ax, ay, az)];
        const double wt = (kz == 0 || kz == m) ? 1.0 : 2.0;
        if (use_lds)
            atomicAdd(&sp[b], wt * (double)pw);
        else
            atomicAdd(&psum[b], wt * (double)pw);
    }
    __syncthreads();
    if (use_lds)
        for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
            if (sp[b] != 0.0) atomicAdd(&psum[b], sp[b]);
}

__global__ void k_pk_finish_p(double* pk, const double* cnt, long n, double pnorm) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = cnt[i];
    pk[i] = c > 0.0 ? pk[i] / c * pnorm : 0.0;
}

hipError_t pk_alias_pass(const float2* spec, long bstride, const Mesh3& g, int n_real, int n_bins,
                         const double* k_mean, double* pk, const double* n_modes, double pnorm, double kf,
                         float* scratch, long sstride, hipStream_t st) {
    const int n = g.n, h = n / 2;
    const long classes = tet_index(h + 1, 0, 0);
    const long slope_off = ((classes + 63) / 64) * 64;
    const int nsl = (int)(pk_alias_scratch_floats(n, n_bins) - slope_off);
    const long nb = (long)n_bins * n_real;
    {
        ProfScope ps(PROF_PK_ALIAS, st, 1);
        hipLaunchKernelGGL(k_pk_slopes, dim3((unsigned)((nsl + 63) / 64), n_real), dim3(64), 0, st, k_mean, pk,
                           n_modes, n_bins, nsl, kf, scratch, sstride, slope_off);
        hipLaunchKernelGGL(k_alias_table, dim3((unsigned)((classes + 255) / 256), n_real), dim3(256), 0, st, n,
                           n_bins, nsl, scratch, sstride, slope_off);
    }
    hipError_t e = launch_fill_d(pk, nb, 0.0, st);
    if (e != hipSuccess) return e;
    const long total = (long)n * n * (h + 1);
    long blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    ProfScope ps(PROF_PK_ALIAS, st, 2);
    hipLaunchKernelGGL(k_pk_bin_alias, dim3((unsigned)blocks, n_real), dim3(256), 0, st, spec, bstride, n, g.plane,
                       n_bins, scratch, sstride, pk);
    hipLaunchKernelGGL(k_pk_finish_p, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, pk, n_modes, nb, pnorm);
    return hipGetLastError();
}

}  // namespace cola
