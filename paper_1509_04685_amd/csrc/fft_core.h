// Register/LDS Stockham FFT engine for gfx950 (64-wide wavefronts).
//
// A line of n complex values (n = 2^a 3^b) is transformed by T = n / R threads, each owning
// R values in registers.  Radix-r stages (r in {2,3,4,8}, and 6 and 12 in static plans; r | R)
// follow the Stockham autosort recursion: with ns the product of the radices already applied,
// butterfly j (0 <= j < n/r) reads elements j + i n/r (i < r), multiplies element i by W_{ns r}^{i (j mod ns)},
// applies an r-point DFT and writes element i to (j / ns) ns r + (j mod ns) + i ns.  Thread t
// owns butterflies j = t + s T, s < R/r.  Between stages the values go through LDS (write,
// barrier, read, barrier).  The first stage's inputs and the last stage's outputs use the same
// pattern -- element (t + s T) + i n / r -- so a caller loads and stores straight from and to
// global memory, and a forward and an inverse transform can be chained in registers when the
// inverse plan starts with the forward plan's last radix.
//
// Twiddles come from a table tw[m] = exp(-2 pi i m / (n * tw_stride)) built in float64 on the
// device; the inverse uses conjugates.  Transforms are unnormalised.  Kernels built on a static
// plan read the table from a copy in LDS (kTwN entries): read from global memory, the twiddles
// cost a quarter of a pass's time on the 768-point lines.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace cola {

constexpr int kMaxStages = 12;

struct FftPlan {
    int n;        // complex line length
    int R;        // values per thread
    int T;        // threads per line, n / R
    int nst;      // number of stages
    int radix[kMaxStages];
    // per-stage constants, filled on the host by finish_plan():
    int ns[kMaxStages];        // product of the radices before the stage
    uint32_t nsm[kMaxStages];  // magic multiplier: j / ns == umulhi(j, nsm) for j < 2^16
    int nr[kMaxStages];        // n / radix: distance between a butterfly's inputs
    int tstep[kMaxStages];     // twiddle table step per unit of (j mod ns)
};

// Fills the per-stage constants of a plan whose radices are set (host side).
inline void finish_plan(FftPlan& p, int tw_stride) {
    int ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        int r = p.radix[s];
        p.ns[s] = ns;
        p.nsm[s] = ns > 1 ? (uint32_t)(0x100000000ull / (uint64_t)ns + 1ull) : 0u;  // ns = 1 special-cased
        p.nr[s] = p.n / r;
        p.tstep[s] = (p.n / (ns * r)) * tw_stride;
        ns *= r;
    }
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by the forward twiddle w = e^{-i theta} (or its conjugate for the inverse)
template <bool INV>
__device__ __forceinline__ float2 twiddle(float2 a, float2 w) {
    return INV ? make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y)
               : make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
    const float c = -0.5f;
    const float s = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 t = cadd(a1, a2);
    float2 u = csub(a1, a2);
    float2 m = make_float2(a0.x + c * t.x, a0.y + c * t.y);
    // forward: X1 = m - i s u, X2 = m + i s u
    float2 isu = INV ? make_float2(-s * u.y, s * u.x) : make_float2(s * u.y, -s * u.x);  // (-+ i) s u
    a0 = cadd(a0, t);
    a1 = cadd(m, isu);
    a2 = csub(m, isu);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* a) {
    const float h = 0.70710678118654752440f;
    float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    // W8^1 = (1 - i)/sqrt2, W8^2 = -i, W8^3 = (-1 - i)/sqrt2 (forward); conjugates inverse
    float2 w1 = INV ? make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y))
                    : make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
    float2 w2 = mul_mi<INV>(o2);
    float2 w3 = INV ? make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y))
                    : make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, w1);
    a[5] = csub(e1, w1);
    a[2] = cadd(e2, w2);
    a[6] = csub(e2, w2);
    a[3] = cadd(e3, w3);
    a[7] = csub(e3, w3);
}

// k in [0, N1 N2) with k = k1 (mod N1) and k = k2 (mod N2) (N1, N2 coprime).
constexpr int crt_index(int k1, int k2, int n1, int n2) {
    for (int k = 0; k < n1 * n2; ++k)
        if (k % n1 == k1 && k % n2 == k2) return k;
    return 0;
}

// 6- and 12-point DFTs (N1 = 2 or 4 times N2 = 3) by the prime-factor (Good-Thomas) mapping:
// input n = (n1 N2 + n2 N1) mod N, output k = CRT(k1, k2); the two factors need no twiddles
// between them, so a radix-6 or -12 stage costs a radix-3 stage's butterflies without its own
// pass through LDS.
template <int N1, bool INV>
__device__ __forceinline__ void dft_pfa3(float2* a) {
    constexpr int N2 = 3, N = N1 * N2;
    float2 y[N];  // y[k1 N2 + n2]
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
        float2 t[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) t[n1] = a[(n1 * N2 + n2 * N1) % N];
        if constexpr (N1 == 2) dft2<INV>(t[0], t[1]);
        if constexpr (N1 == 4) dft4<INV>(t[0], t[1], t[2], t[3]);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) y[k1 * N2 + n2] = t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
        float2 u0 = y[k1 * N2], u1 = y[k1 * N2 + 1], u2 = y[k1 * N2 + 2];
        dft3<INV>(u0, u1, u2);
        a[crt_index(k1, 0, N1, N2)] = u0;
        a[crt_index(k1, 1, N1, N2)] = u1;
        a[crt_index(k1, 2, N1, N2)] = u2;
    }
}

__device__ __forceinline__ int div_ns(int j, uint32_t nsm) { return (int)__umulhi((uint32_t)j, nsm); }

// One radix-r stage on the registers of one thread: twiddle then butterfly.
template <int r, int R, bool INV>
__device__ __forceinline__ void stage_compute(float2 (&v)[R], int t, int T, int ns, uint32_t nsm, int tstep,
                                              const float2* tw) {
#pragma unroll
    for (int s = 0; s < R / r; ++s) {
        float2* a = &v[s * r];
        if (ns > 1) {
            int j = t + s * T;
            int k = j - div_ns(j, nsm) * ns;
            int step = tstep * k;
#pragma unroll
            for (int i = 1; i < r; ++i) a[i] = twiddle<INV>(a[i], tw[i * step]);
        }
        if constexpr (r == 2) dft2<INV>(a[0], a[1]);
        if constexpr (r == 3) dft3<INV>(a[0], a[1], a[2]);
        if constexpr (r == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
        if constexpr (r == 8) dft8<INV>(a);
    }
}

template <int R, bool INV>
__device__ __forceinline__ void stage_dispatch(int r, float2 (&v)[R], int t, int T, int ns, uint32_t nsm, int tstep,
                                               const float2* tw) {
    if constexpr (R % 8 == 0) { if (r == 8) { stage_compute<8, R, INV>(v, t, T, ns, nsm, tstep, tw); return; } }
    if constexpr (R % 4 == 0) { if (r == 4) { stage_compute<4, R, INV>(v, t, T, ns, nsm, tstep, tw); return; } }
    if constexpr (R % 3 == 0) { if (r == 3) { stage_compute<3, R, INV>(v, t, T, ns, nsm, tstep, tw); return; } }
    if constexpr (R % 2 == 0) { if (r == 2) { stage_compute<2, R, INV>(v, t, T, ns, nsm, tstep, tw); return; } }
}

// Scatter a stage's outputs to LDS: value v[s r + i] goes to element (j/ns) ns r + j%ns + i ns.
template <int r, int R>
__device__ __forceinline__ void stage_store(const float2 (&v)[R], float2* lds, int les, int t, int T, int ns,
                                            uint32_t nsm) {
#pragma unroll
    for (int s = 0; s < R / r; ++s) {
        int j = t + s * T;
        int q = (ns == 1) ? j : div_ns(j, nsm);
        int base = q * ns * (r - 1) + j;  // (j/ns) ns r + j%ns
#pragma unroll
        for (int i = 0; i < r; ++i) lds[(base + i * ns) * les] = v[s * r + i];
    }
}

// Gather a stage's inputs from LDS: v[s r + i] = element (t + s T) + i n / r.
template <int r, int R>
__device__ __forceinline__ void stage_load(float2 (&v)[R], const float2* lds, int les, int t, int T, int nr) {
#pragma unroll
    for (int s = 0; s < R / r; ++s) {
        int j = t + s * T;
#pragma unroll
        for (int i = 0; i < r; ++i) v[s * r + i] = lds[(j + i * nr) * les];
    }
}

template <int R>
__device__ __forceinline__ void store_dispatch(int r, const float2 (&v)[R], float2* lds, int les, int t, int T,
                                               int ns, uint32_t nsm) {
    if constexpr (R % 8 == 0) { if (r == 8) { stage_store<8, R>(v, lds, les, t, T, ns, nsm); return; } }
    if constexpr (R % 4 == 0) { if (r == 4) { stage_store<4, R>(v, lds, les, t, T, ns, nsm); return; } }
    if constexpr (R % 3 == 0) { if (r == 3) { stage_store<3, R>(v, lds, les, t, T, ns, nsm); return; } }
    if constexpr (R % 2 == 0) { if (r == 2) { stage_store<2, R>(v, lds, les, t, T, ns, nsm); return; } }
}

template <int R>
__device__ __forceinline__ void load_dispatch(int r, float2 (&v)[R], const float2* lds, int les, int t, int T,
                                              int nr) {
    if constexpr (R % 8 == 0) { if (r == 8) { stage_load<8, R>(v, lds, les, t, T, nr); return; } }
    if constexpr (R % 4 == 0) { if (r == 4) { stage_load<4, R>(v, lds, les, t, T, nr); return; } }
    if constexpr (R % 3 == 0) { if (r == 3) { stage_load<3, R>(v, lds, les, t, T, nr); return; } }
    if constexpr (R % 2 == 0) { if (r == 2) { stage_load<2, R>(v, lds, les, t, T, nr); return; } }
}

// Calls f(q, e) for every register q of a thread and the element e it holds in the load/store
// pattern of a radix-r first or last stage: q = s r + i holds element (t + s T) + i nr.
template <int R, class F>
__device__ __forceinline__ void for_pattern(int r, int t, int T, int nr, F&& f) {
    auto run = [&](auto rc) {
        constexpr int rr = decltype(rc)::value;
#pragma unroll
        for (int s = 0; s < R / rr; ++s)
#pragma unroll
            for (int i = 0; i < rr; ++i) f(s * rr + i, t + s * T + i * nr);
    };
    if constexpr (R % 8 == 0) { if (r == 8) { run(std::integral_constant<int, 8>{}); return; } }
    if constexpr (R % 4 == 0) { if (r == 4) { run(std::integral_constant<int, 4>{}); return; } }
    if constexpr (R % 3 == 0) { if (r == 3) { run(std::integral_constant<int, 3>{}); return; } }
    if constexpr (R % 2 == 0) { if (r == 2) { run(std::integral_constant<int, 2>{}); return; } }
}

// Element index held in v[s r + i] by the load/store pattern of a radix-r first/last stage.
__device__ __forceinline__ int pattern_index(int s, int i, int r, int t, int T, int n) {
    return t + s * T + i * (n / r);
}

// Full line transform.  On entry v holds the inputs in the pattern of plan radix[0]; on exit v
// holds the outputs in the pattern of plan radix[nst-1].  `active` threads take part in the
// LDS exchange; every thread of the block must call this (barriers inside).  `lds` points at
// element 0 of this thread's line; consecutive elements are `les` float2 apart.  The plan's
// twiddle steps already include the table stride.
template <int R, bool INV>
__device__ __forceinline__ void fft_line(float2 (&v)[R], const FftPlan& pl, float2* lds, int les, int t,
                                         const float2* tw, bool active) {
    for (int st = 0; st < pl.nst; ++st) {
        const int r = pl.radix[st];
        if (active) stage_dispatch<R, INV>(r, v, t, pl.T, pl.ns[st], pl.nsm[st], pl.tstep[st], tw);
        if (st + 1 < pl.nst) {
            if (active) store_dispatch<R>(r, v, lds, les, t, pl.T, pl.ns[st], pl.nsm[st]);
            __syncthreads();
            if (active) load_dispatch<R>(pl.radix[st + 1], v, lds, les, t, pl.T, pl.nr[st + 1]);
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ line engines
//
// The kernels are written against a line engine that owns the plan: DynLine runs a plan built on
// the host (any size), StatLine a plan fixed at compile time for one line length N, values per
// thread R and LDS element stride LES.  With every stage's radix, product ns and LDS offset known
// to the compiler, the static engine's index arithmetic folds into constants and LDS instruction
// offsets; its radix order is 3s first (each merged with a 4 or a 2 into a radix-12 or -6
// stage where R allows), then 8s, 4s, 2s; reversed for REV.

template <int R>
struct DynLine {
    static constexpr int kR = R;
    static constexpr bool kStatic = false;
    static constexpr bool kSplit = false;
    static constexpr int kT = 0;  // threads per line: known at run time only
    static constexpr int kN = 0;
    static constexpr int kTwN = 0;  // reads the table in global memory
    FftPlan p;
    int les;
    __device__ int T() const { return p.T; }
    __device__ int n() const { return p.n; }
    template <class F>
    __device__ __forceinline__ void first(int t, F&& f) const { for_pattern<R>(p.radix[0], t, p.T, p.nr[0], f); }
    template <class F>
    __device__ __forceinline__ void last(int t, F&& f) const {
        for_pattern<R>(p.radix[p.nst - 1], t, p.T, p.nr[p.nst - 1], f);
    }
    template <bool INV>
    __device__ __forceinline__ void run(float2 (&v)[R], float2* lds, int t, const float2* tw, bool active) const {
        fft_line<R, INV>(v, p, lds, les, t, tw, active);
    }
};

struct Radices {
    int nst;
    int r[kMaxStages];
};

constexpr Radices static_radices(int n, int R, bool rev) {
    Radices s{0, {}};
    int m = n, k = 0;
    while (m % 3 == 0) {  // each factor 3 joins a factor 4 or 2 in one prime-factor stage when it can
        if (R % 12 == 0 && (m / 3) % 4 == 0) {
            s.r[k++] = 12;
            m /= 12;
        } else if (R % 6 == 0 && (m / 3) % 2 == 0) {
            s.r[k++] = 6;
            m /= 6;
        } else {
            s.r[k++] = 3;
            m /= 3;
        }
    }
    while (R % 8 == 0 && m % 8 == 0) { s.r[k++] = 8; m /= 8; }
    while (R % 4 == 0 && m % 4 == 0) { s.r[k++] = 4; m /= 4; }
    while (m % 2 == 0) { s.r[k++] = 2; m /= 2; }
    s.nst = k;
    if (rev)
        for (int i = 0; i < k / 2; ++i) {
            int tmp = s.r[i];
            s.r[i] = s.r[k - 1 - i];
            s.r[k - 1 - i] = tmp;
        }
    return s;
}

constexpr int radices_ns(const Radices& s, int st) {
    int ns = 1;
    for (int i = 0; i < st; ++i) ns *= s.r[i];
    return ns;
}

// Entries of a twiddle table with stride tws that a plan reads: its largest index + 1.
constexpr int radices_tw_entries(const Radices& s, int n, int tws) {
    int mx = 0, ns = 1;
    for (int i = 0; i < s.nst; ++i) {
        const int r = s.r[i];
        const int m = (r - 1) * (n / (ns * r)) * tws * (ns - 1);
        if (m > mx) mx = m;
        ns *= r;
    }
    return mx + 1;
}

constexpr bool static_plan_ok(int n, int R) {
    if (R < 2 || n % R) return false;
    Radices s = static_radices(n, R, false);
    int prod = 1;
    for (int i = 0; i < s.nst; ++i) {
        if (R % s.r[i]) return false;
        prod *= s.r[i];
    }
    return prod == n;
}

// N: line length; R: values per thread; LES: LDS element stride (float2, or float with SPL);
// TWS: twiddle table stride (the table holds exp(-2 pi i m / (N TWS))); REV: reversed radix order;
// SPL: exchange the real and then the imaginary parts through a float buffer of N LES floats
// (half the LDS of a float2 exchange, two more barriers per stage), which lets wide column tiles
// keep more blocks resident.
template <int N, int R, int LES, int TWS, bool REV, bool SPL = false>
struct StatLine {
    static_assert(static_plan_ok(N, R), "no static plan for this line length and R");
    static constexpr int kR = R;
    static constexpr bool kStatic = true;
    static constexpr bool kSplit = SPL;
    static constexpr int kN = N;
    static constexpr int kT = N / R;
    static constexpr Radices kRad = static_radices(N, R, REV);
    static constexpr int kTwN = radices_tw_entries(kRad, N, TWS);  // staged in LDS by the kernels
    static constexpr int kFirst = kRad.r[0];
    static constexpr int kLast = kRad.r[kRad.nst - 1];
    __device__ static constexpr int T() { return kT; }
    __device__ static constexpr int n() { return N; }

    template <int r, class F>
    __device__ __forceinline__ static void pattern(int t, F&& f) {
#pragma unroll
        for (int s = 0; s < R / r; ++s)
#pragma unroll
            for (int i = 0; i < r; ++i) f(s * r + i, t + s * kT + i * (N / r));
    }
    template <class F>
    __device__ __forceinline__ void first(int t, F&& f) const { pattern<kFirst>(t, f); }
    template <class F>
    __device__ __forceinline__ void last(int t, F&& f) const { pattern<kLast>(t, f); }

    template <bool INV, int ST>
    __device__ __forceinline__ static void stage(float2 (&v)[R], float2* lds, int t, const float2* tw,
                                                 bool active) {
        if constexpr (ST < kRad.nst) {
            constexpr int r = kRad.r[ST];
            constexpr int ns = radices_ns(kRad, ST);
            constexpr int tstep = (N / (ns * r)) * TWS;
            if (active) {
#pragma unroll
                for (int s = 0; s < R / r; ++s) {
                    float2* a = &v[s * r];
                    if constexpr (ns > 1) {
                        const int j = t + s * kT;
                        const int step = tstep * (j % ns);
#pragma unroll
                        for (int i = 1; i < r; ++i) a[i] = twiddle<INV>(a[i], tw[i * step]);
                    }
                    if constexpr (r == 2) dft2<INV>(a[0], a[1]);
                    if constexpr (r == 3) dft3<INV>(a[0], a[1], a[2]);
                    if constexpr (r == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
                    if constexpr (r == 6) dft_pfa3<2, INV>(a);
                    if constexpr (r == 8) dft8<INV>(a);
                    if constexpr (r == 12) dft_pfa3<4, INV>(a);
                }
            }
            if constexpr (ST + 1 < kRad.nst) {
                constexpr int rn = kRad.r[ST + 1];
                if constexpr (SPL) {
                    // the real parts go out and come back in place before the imaginary parts
                    // leave, so no temporaries are held
                    float* lf = reinterpret_cast<float*>(lds);
                    if (active) write_part<r, ns, 0>(v, lf, t);
                    __syncthreads();
                    if (active) read_part<rn, 0>(v, lf, t);
                    __syncthreads();
                    if (active) write_part<r, ns, 1>(v, lf, t);
                    __syncthreads();
                    if (active) read_part<rn, 1>(v, lf, t);
                } else {
                    if (active) {
#pragma unroll
                        for (int s = 0; s < R / r; ++s) {
                            const int j = t + s * kT;
                            const int base = (j / ns) * ns * (r - 1) + j;  // (j/ns) ns r + j%ns
#pragma unroll
                            for (int i = 0; i < r; ++i) lds[(base + i * ns) * LES] = v[s * r + i];
                        }
                    }
                    __syncthreads();
                    if (active) {
#pragma unroll
                        for (int s = 0; s < R / rn; ++s)
#pragma unroll
                            for (int i = 0; i < rn; ++i) v[s * rn + i] = lds[(t + s * kT + i * (N / rn)) * LES];
                    }
                }
                __syncthreads();
                stage<INV, ST + 1>(v, lds, t, tw, active);
            }
        }
    }
    template <bool INV>
    __device__ __forceinline__ void run(float2 (&v)[R], float2* lds, int t, const float2* tw, bool active) const {
        stage<INV, 0>(v, lds, t, tw, active);
    }

    // Split exchange: one component (P = 0: real, 1: imaginary) of the stage's output written in
    // the order the next stage reads, and read back.
    template <int r, int ns, int P>
    __device__ __forceinline__ static void write_part(const float2 (&v)[R], float* lf, int t) {
#pragma unroll
        for (int s = 0; s < R / r; ++s) {
            const int j = t + s * kT;
            const int base = (j / ns) * ns * (r - 1) + j;
#pragma unroll
            for (int i = 0; i < r; ++i) lf[(base + i * ns) * LES] = P == 0 ? v[s * r + i].x : v[s * r + i].y;
        }
    }
    template <int rn, int P>
    __device__ __forceinline__ static void read_part(float2 (&v)[R], const float* lf, int t) {
#pragma unroll
        for (int s = 0; s < R / rn; ++s)
#pragma unroll
            for (int i = 0; i < rn; ++i) {
                const float x = lf[(t + s * kT + i * (N / rn)) * LES];
                if constexpr (P == 0) v[s * rn + i].x = x;
                else v[s * rn + i].y = x;
            }
    }
};

}  // namespace cola
