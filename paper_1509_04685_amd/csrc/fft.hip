// 3D FFT passes for cubic meshes on gfx950 (Sec. 2.2: one forward and three inverse FFTs per
// particle-mesh force).  Real fields are [x][y][z] rows of `row` floats; the half spectrum is
// transposed, [kz][x][y] of float2 (y contiguous, kz planes of n^2 values), so that the y pass
// works on contiguous rows and the x pass on columns n values apart -- no pass walks an axis at
// the stride of a whole plane.
//
// Passes (each one HBM read and one write of the array):
//   z: real rows <-> half complex via an n/2-point complex FFT plus a split step, each block
//      moving W rows of one x plane and W consecutive y of every kz plane (out of place);
//   y: contiguous complex rows, in place;
//   x: columns, a tile of TK adjacent y columns per block so that every row access moves TK * 8
//      contiguous bytes, in place.
// The particle-mesh force fuses the forward x transform, the Green's function and the inverse x
// transform in one pass that writes two outputs, so the full spectrum never goes to HBM.

#include "fft_kernels.h"


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

// Pad of the kz-plane stride of the transposed spectrum (float2): with planes exactly n^2 apart,
// the values a z pass moves for one row group (the same (x, y) in every plane) differ only in
// their high address bits.  Measured on the 768^3 step (ms per node): pad 0 9.76, 8 9.87, 16 9.41,
// 32 9.30, 48 9.33, 64 9.46, 256 9.78.
constexpr long kSpecPlanePad = 32;

Mesh3 make_mesh(int n) {
    Mesh3 g;
    g.n = n;
    g.m = n / 2;
    g.nzp = ((g.m + 1) + 15) / 16 * 16;
    g.plane = (long)n * n + kSpecPlanePad;
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

// Shape of one FFT kernel launch: R values per thread, `width` lines per block (z passes, y rows)
// or columns per tile (x columns), whether the compile-time plan of that shape is used, and (x
// columns, static plans only) whether its exchanges are split into real and imaginary parts.
struct FftShape {
    int R = 0;
    int width = 0;
    bool stat = false;
    bool split = false;
};

enum FftKind { FK_Z_R2C = 0, FK_Z_C2R, FK_ROWS_Y, FK_COLS_X, FK_X_GREEN, FK_Y_SPLIT, FK_X_MULT, FK_Z_C2R3, FK_NUM };
static const char* const kFftKindName[FK_NUM] = {"z_r2c", "z_c2r", "rows_y", "cols_x", "x_green",
                                                 "y_split", "x_mult", "z_c2r3"};

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

static bool is_z(FftKind k) { return k == FK_Z_R2C || k == FK_Z_C2R || k == FK_Z_C2R3; }
static bool is_rows(FftKind k) { return k == FK_ROWS_Y || k == FK_Y_SPLIT; }

// Line length the kernel transforms: n/2 for the z passes, n otherwise.
static int line_len(FftKind k, int n) { return is_z(k) ? n / 2 : n; }

static FftOp op_of(FftKind k) {
    switch (k) {
        case FK_Z_R2C: return OP_Z_R2C;
        case FK_Z_C2R: return OP_Z_C2R;
        case FK_Z_C2R3: return OP_Z_C2R3;
        case FK_ROWS_Y: return OP_ROWS_FWD;
        case FK_COLS_X: return OP_COLS_FWD;
        case FK_X_GREEN: return OP_X_GREEN;
        case FK_Y_SPLIT: return OP_ROWS_SPLIT;
        default: return OP_X_MULT;
    }
}

// Routes a launch to the static kernels of its mesh size (n: the mesh side).
static hipError_t launch_static(const FftLaunch& L, int n) {
    switch (n) {
        case 1536: return fft_static_1536(L);
        case 768: return fft_static_768(L);
        case 512: return fft_static_512(L);
        case 384: return fft_static_384(L);
        case 288: return fft_static_288(L);
        case 256: return fft_static_256(L);
        default: return hipErrorNotSupported;
    }
}

static bool is_cols(FftKind k) { return k == FK_COLS_X || k == FK_X_GREEN || k == FK_X_MULT; }

static bool static_available(FftKind k, int n, int R, int width, bool split = false) {
    if (split && !is_cols(k)) return false;
    FftLaunch L;
    L.op = op_of(k);
    L.n = line_len(k, n);
    L.R = R;
    L.width = width;
    L.split = split;
    L.probe = true;
    return launch_static(L, n) == hipSuccess;
}

// Threads per block: z_c2r3 runs one group of lines per force component.
static long shape_threads(FftKind k, int n, const FftShape& sh) {
    return (long)sh.width * (line_len(k, n) / sh.R) * (k == FK_Z_C2R3 ? 3 : 1);
}

// LDS of one block: z passes keep their lines L + 2 complex values apart (the line, its kz Nyquist
// value and one value against bank conflicts of the transposed accesses); z_c2r3 holds one group
// of lines per force component.
static size_t shape_lds(FftKind k, int n, const FftShape& sh) {
    int L = line_len(k, n);
    if (is_z(k)) return (size_t)sh.width * (L + 2) * sizeof(float2) * (k == FK_Z_C2R3 ? 3 : 1);
    return (size_t)sh.width * L * (sh.split ? sizeof(float) : sizeof(float2));
}

static int log2_exact(int w) {  // log2 of a power of two, -1 otherwise
    int l = 0;
    while ((1 << l) < w) ++l;
    return (1 << l) == w ? l : -1;
}

static bool shape_ok(FftKind k, int n, const FftShape& sh) {
    int L = line_len(k, n);
    if (!plan_ok(L, sh.R) || sh.width < 1) return false;
    if (sh.split && (!sh.stat || !is_cols(k))) return false;
    // z passes: a power-of-two number of lines of one x plane per block
    if (is_z(k) && (log2_exact(sh.width) < 0 || n % sh.width)) return false;
    long threads = shape_threads(k, n, sh);
    // 1024-thread blocks only for the kernels compiled for them: the static x-column plans with
    // split exchanges and z_c2r3
    if (threads > ((sh.split || k == FK_Z_C2R3) ? 1024 : 512) || threads < 1) return false;
    // z_c2r3 may take up to 150 KB: with 16 lines of 768 points its three groups need 148 KB
    return shape_lds(k, n, sh) <= (k == FK_Z_C2R3 ? 150 : 128) * 1024;
}

static FftShape default_shape(FftKind k, int n) {
    int L = line_len(k, n);
    FftPlan pl = make_plan(L);
    FftShape sh;
    sh.R = pl.R;
    if (is_z(k) || is_rows(k)) {
        sh.width = std::max(1, 256 / pl.T);
        while ((long)sh.width * pl.T > 512) sh.width /= 2;
        if (is_z(k)) {
            int w = 1;  // the largest power of two <= width that divides n
            while (w * 2 <= sh.width && n % (w * 2) == 0) w *= 2;
            sh.width = w;
            while (sh.width > 1 && !shape_ok(k, n, sh)) sh.width /= 2;  // z_c2r3: three groups
        }
    } else {
        sh.width = pick_tk(n, pl.T);
    }
    sh.stat = static_available(k, n, sh.R, sh.width);
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

// Pins the shape of one pass kind at mesh size n (what the autotuner would otherwise choose).
int set_fft_shape(int n, const char* kind, int R, int width, int stat) {
    if (!kind || !fft_size_ok(n)) return COLA_ERR_INVALID_ARG;
    int k = -1;
    for (int i = 0; i < FK_NUM; ++i)
        if (std::string(kind) == kFftKindName[i]) k = i;
    if (k < 0) return COLA_ERR_INVALID_ARG;
    if (stat < 0 || stat > 2) return COLA_ERR_INVALID_ARG;
    const FftShape sh{R, width, stat != 0, stat == 2};
    if (!shape_ok((FftKind)k, n, sh)) return COLA_ERR_INVALID_ARG;
    if (sh.stat && !static_available((FftKind)k, n, R, width, sh.split)) return COLA_ERR_INVALID_ARG;
    ShapeCache& c = shape_cache();
    std::lock_guard<std::mutex> g(c.mu);
    c.tuned[{k, n}] = sh;
    return COLA_OK;
}

// ------------------------------------------------------------------ launchers

static ColGeom cols_x(const Mesh3& g, int tk) {
    ColGeom cg;
    cg.es = g.n;
    cg.inner = g.n;
    cg.plane_stride = (int)g.plane;
    cg.tk = tk;
    cg.tiles = (g.n + tk - 1) / tk;
    return cg;
}

// Launches L with the shape's static kernel or the dynamic kernel of the same shape.
static hipError_t launch_shape(FftLaunch& L, int mesh_n, const FftShape& sh) {
    const bool z = is_z_op(L.op);
    L.n = z ? mesh_n / 2 : mesh_n;
    L.R = sh.R;
    L.width = sh.width;
    L.split = sh.split;
    if (sh.stat) {
        hipError_t e = launch_static(L, mesh_n);
        // a split exchange exists only in static plans (its LDS size is half the dynamic kernel's)
        if (e != hipErrorNotSupported || sh.split) return e;
    }
    FftPlan pl = make_plan_r(L.n, sh.R, false);
    if (z) finish_plan(pl, 2);
    const int les = (z || is_rows_op(L.op)) ? 1 : sh.width;
    hipError_t err = hipSuccess;
    hipError_t de = dispatch_r(sh.R, [&](auto rr) {
        constexpr int R = decltype(rr)::value;
        using D = DynLine<R>;
        D e{pl, les};
        switch (L.op) {
            case OP_Z_R2C: err = go_z_r2c<D>(L, e); break;
            case OP_Z_C2R: err = go_z_c2r<D>(L, e); break;
            case OP_Z_C2R3: err = go_z_c2r3<D>(L, e); break;
            case OP_ROWS_FWD: err = go_rows<D, 0>(L, e); break;
            case OP_ROWS_INV: err = go_rows<D, 1>(L, e); break;
            case OP_ROWS_SPLIT: err = go_rows<D, 2>(L, e); break;
            case OP_COLS_FWD: err = go_cols<D, 0>(L, e); break;
            case OP_X_GREEN: {
                D ei{make_plan_r(L.n, R, true), les};
                err = go_x_green<D, D, 0>(L, e, ei);
                break;
            }
            case OP_X_GREEN_FILT: {
                D ei{make_plan_r(L.n, R, true), les};
                err = go_x_green<D, D, 0, true>(L, e, ei);
                break;
            }
            case OP_X_MULT: err = go_x_mult<D, 0>(L, e); break;
        }
    });
    return err != hipSuccess ? err : de;
}

// y rows of every kz plane: op OP_ROWS_FWD / OP_ROWS_INV on A, or OP_ROWS_SPLIT (A -> A, S).
static hipError_t run_rows_shape(FftOp op, float2* A, float2* S, long bstride, const Mesh3& g, const float2* tw,
                                 float kf, int n_real, const FftShape& sh, hipStream_t st) {
    FftLaunch L;
    L.op = op;
    L.nrows = (long)(g.m + 1) * g.n;
    L.lds = shape_lds(FK_ROWS_Y, g.n, sh);
    L.grid = dim3((unsigned)((L.nrows + sh.width - 1) / sh.width), n_real);
    L.block = dim3(sh.width * (g.n / sh.R));
    L.st = st;
    L.d0 = A;
    L.d1 = S;
    L.b0 = bstride;
    L.plane = g.plane;
    L.tw = tw;
    L.kf = kf;
    const int kind = op == OP_ROWS_FWD ? PROF_Y_FWD : (op == OP_ROWS_INV ? PROF_Y_INV : PROF_Y_SPLIT);
    ProfScope ps(kind, st, g.n);
    return launch_shape(L, g.n, sh);
}

static hipError_t run_rows(FftOp op, float2* A, float2* S, long bstride, const Mesh3& g, const float2* tw, float kf,
                           int n_real, hipStream_t st) {
    return run_rows_shape(op, A, S, bstride, g, tw, kf, n_real,
                          shape_for(op == OP_ROWS_SPLIT ? FK_Y_SPLIT : FK_ROWS_Y, g.n), st);
}

static hipError_t run_cols_shape(float2* data, long bstride, const Mesh3& g, const float2* tw, int n_real,
                                 const FftShape& sh, hipStream_t st) {
    FftLaunch L;
    L.op = OP_COLS_FWD;
    L.cg = cols_x(g, sh.width);
    L.lds = shape_lds(FK_COLS_X, g.n, sh);
    L.grid = dim3((unsigned)((long)(g.m + 1) * L.cg.tiles), n_real);
    L.block = dim3(sh.width * (g.n / sh.R));
    L.st = st;
    L.d0 = data;
    L.b0 = bstride;
    L.tw = tw;
    ProfScope ps(PROF_X_FWD, st, g.n);
    return launch_shape(L, g.n, sh);
}

static hipError_t run_z_r2c_shape(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                                  const Mesh3& g, const float2* tw, int n_real, float pa, float pb,
                                  const FftShape& sh, hipStream_t st) {
    FftLaunch L;
    L.op = OP_Z_R2C;
    const int lpb = sh.width;
    L.lds = shape_lds(FK_Z_R2C, g.n, sh);
    L.grid = dim3((unsigned)((long)g.n * g.n / lpb), n_real);
    L.block = dim3(lpb * (g.m / sh.R));
    L.st = st;
    L.rin = in;
    L.in_row = in_row;
    L.in_bstride = in_bstride;
    L.cout = out;
    L.out_bstride = out_bstride;
    L.mesh_n = g.n;
    L.plane = g.plane;
    L.lw = log2_exact(lpb);
    L.tw = tw;
    L.pa = pa;
    L.pb = pb;
    ProfScope ps(PROF_Z_R2C, st, g.n);
    return launch_shape(L, g.n, sh);
}

static hipError_t run_z_r2c(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                            const Mesh3& g, const float2* tw, int n_real, float pa, float pb, hipStream_t st) {
    return run_z_r2c_shape(in, in_row, in_bstride, out, out_bstride, g, tw, n_real, pa, pb,
                           shape_for(FK_Z_R2C, g.n), st);
}

static hipError_t run_z_c2r_shape(const float2* in, long in_bstride, float* out, long out_row, long out_bstride,
                                  const Mesh3& g, const float2* tw, int n_real, float scale, const FftShape& sh,
                                  hipStream_t st) {
    FftLaunch L;
    L.op = OP_Z_C2R;
    const int lpb = sh.width;
    L.lds = shape_lds(FK_Z_C2R, g.n, sh);
    L.grid = dim3((unsigned)((long)g.n * g.n / lpb), n_real);
    L.block = dim3(lpb * (g.m / sh.R));
    L.st = st;
    L.cin = in;
    L.in_bstride = in_bstride;
    L.rout = out;
    L.out_row = out_row;
    L.out_bstride = out_bstride;
    L.mesh_n = g.n;
    L.plane = g.plane;
    L.lw = log2_exact(lpb);
    L.ghost = out_row >= g.n + 2 ? 1 : 0;
    L.tw = tw;
    L.scale = scale;
    ProfScope ps(PROF_Z_C2R, st, g.n);
    return launch_shape(L, g.n, sh);
}

static hipError_t run_z_c2r(const float2* in, long in_bstride, float* out, long out_row, long out_bstride,
                            const Mesh3& g, const float2* tw, int n_real, float scale, hipStream_t st) {
    return run_z_c2r_shape(in, in_bstride, out, out_row, out_bstride, g, tw, n_real, scale, shape_for(FK_Z_C2R, g.n),
                           st);
}

// The three force components into one interleaved mesh (k_fft_z_c2r3); `lines` rows (x, y) from
// the first (all n^2 of them in the step; fewer when the autotuner times it on a scratch buffer).
static hipError_t run_z_c2r3_shape(const float2* fx, const float2* fy, const float2* fz, long in_bstride, float* out,
                                   long out_row, long out_bstride, const Mesh3& g, const float2* tw, int n_real,
                                   float kf, const FftShape& sh, hipStream_t st, long lines = -1) {
    if (out_row < 3L * (g.n + 2)) return hipErrorInvalidValue;
    FftLaunch L;
    L.op = OP_Z_C2R3;
    const int lpb = sh.width;
    if (lines < 0) lines = (long)g.n * g.n;
    L.lds = shape_lds(FK_Z_C2R3, g.n, sh);
    L.grid = dim3((unsigned)(lines / lpb), n_real);
    L.block = dim3((unsigned)shape_threads(FK_Z_C2R3, g.n, sh));
    L.st = st;
    L.cin = fx;
    L.cin1 = fy;
    L.cin2 = fz;
    L.in_bstride = in_bstride;
    L.rout = out;
    L.out_row = out_row;
    L.out_bstride = out_bstride;
    L.mesh_n = g.n;
    L.plane = g.plane;
    L.lw = log2_exact(lpb);
    L.tw = tw;
    L.kf = kf;
    L.scale = 1.0f;
    ProfScope ps(PROF_Z_C2R3, st, g.n);
    return launch_shape(L, g.n, sh);
}

static hipError_t run_x_green_shape(float2* S, float2* A, float2* B, long bstride, const Mesh3& g,
                                    const float2* tw, float kf, int n_real, const FftShape& sh, hipStream_t st,
                                    const GreenFilter* gf = nullptr) {
    FftLaunch L;
    L.op = gf && gf->n > 0 ? OP_X_GREEN_FILT : OP_X_GREEN;
    if (gf) L.gf = *gf;
    L.cg = cols_x(g, sh.width);
    L.lds = shape_lds(FK_X_GREEN, g.n, sh);
    L.grid = dim3((unsigned)((long)(g.m + 1) * L.cg.tiles), n_real);
    L.block = dim3(sh.width * (g.n / sh.R));
    L.st = st;
    L.c0 = S;
    L.d0 = A;
    L.d1 = B;
    L.b0 = bstride;
    L.tw = tw;
    L.kf = kf;
    L.scale = 1.0f / ((float)g.n * (float)g.n * (float)g.n);
    ProfScope ps(PROF_X_GREEN, st, g.n);
    return launch_shape(L, g.n, sh);
}

static hipError_t run_x_mult_shape(const float2* spec, long spec_bstride, float2* work, long work_bstride,
                                   const Mesh3& g, const float2* tw, int n_real, int mtype, int axis_a,
                                   int axis_b, float kf, float scale, const FftShape& sh, hipStream_t st) {
    FftLaunch L;
    L.op = OP_X_MULT;
    L.cg = cols_x(g, sh.width);
    L.lds = shape_lds(FK_X_MULT, g.n, sh);
    L.grid = dim3((unsigned)((long)(g.m + 1) * L.cg.tiles), n_real);
    L.block = dim3(sh.width * (g.n / sh.R));
    L.st = st;
    L.c0 = spec;
    L.b0 = spec_bstride;
    L.d0 = work;
    L.b1 = work_bstride;
    L.tw = tw;
    L.mtype = mtype;
    L.ax_a = axis_a;
    L.ax_b = axis_b;
    L.kf = kf;
    L.scale = scale;
    ProfScope ps(PROF_X_INV_MULT, st, g.n);
    return launch_shape(L, g.n, sh);
}

hipError_t fft_zy_forward(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                          const Mesh3& g, const float2* tw, int n_real, float pa, float pb,
                          hipStream_t st) {
    hipError_t e = run_z_r2c(in, in_row, in_bstride, out, out_bstride, g, tw, n_real, pa, pb, st);
    if (e != hipSuccess) return e;
    return run_rows(OP_ROWS_FWD, out, nullptr, out_bstride, g, tw, 0.0f, n_real, st);
}

hipError_t fft3d_r2c(const float* in, long in_row, long in_bstride, float2* out, long out_bstride,
                     const Mesh3& g, const float2* tw, int n_real, float pa, float pb, hipStream_t st) {
    hipError_t e = fft_zy_forward(in, in_row, in_bstride, out, out_bstride, g, tw, n_real, pa, pb, st);
    if (e != hipSuccess) return e;
    return run_cols_shape(out, out_bstride, g, tw, n_real, shape_for(FK_COLS_X, g.n), st);
}

// x and y passes of the force: x_green (P -> P, Q), y split (P -> P: i k_y, R: plain), y inverse
// of Q; left in the transposed spectrum: F_x in Q, F_y in P, F_z (before i k_z) in R.
static hipError_t force_xy_passes(float2* P, float2* Q, float2* R, long bstride, const Mesh3& g, const float2* tw,
                                  float kf, int n_real, hipStream_t st, const GreenFilter* gf) {
    hipError_t e = run_x_green_shape(P, P, Q, bstride, g, tw, kf, n_real, shape_for(FK_X_GREEN, g.n), st, gf);
    if (e != hipSuccess) return e;
    e = run_rows(OP_ROWS_SPLIT, P, R, bstride, g, tw, kf, n_real, st);
    if (e != hipSuccess) return e;
    return run_rows(OP_ROWS_INV, Q, nullptr, bstride, g, tw, kf, n_real, st);
}

long force_row3(int n) { return (3L * (n + 2) + 31) / 32 * 32; }  // rows start on 128-byte lines

hipError_t pm_force_interleaved(float2* P, float2* Q, float2* R, float* F, long frow, long fstride, long bstride,
                                const Mesh3& g, const float2* tw, float kf, int n_real, hipStream_t st,
                                const GreenFilter* gf) {
    hipError_t e = force_xy_passes(P, Q, R, bstride, g, tw, kf, n_real, st, gf);
    if (e != hipSuccess) return e;
    return run_z_c2r3_shape(Q, P, R, bstride, F, frow, fstride, g, tw, n_real, kf, shape_for(FK_Z_C2R3, g.n), st);
}

hipError_t fft3d_c2r_mult(const float2* spec, long spec_bstride, float2* work, long work_bstride,
                          float* out, long out_row, long out_bstride, const Mesh3& g, const float2* tw,
                          int n_real, int mtype, int axis_a, int axis_b, float kf, float scale,
                          hipStream_t st) {
    hipError_t e = run_x_mult_shape(spec, spec_bstride, work, work_bstride, g, tw, n_real, mtype, axis_a, axis_b,
                                    kf, scale, shape_for(FK_X_MULT, g.n), st);
    if (e != hipSuccess) return e;
    e = run_rows(OP_ROWS_INV, work, nullptr, work_bstride, g, tw, kf, n_real, st);
    if (e != hipSuccess) return e;
    return run_z_c2r(work, work_bstride, out, out_row, out_bstride, g, tw, n_real, 1.0f, st);
}

// Times every admissible shape of each FFT kernel at mesh size n on the buffers S, A, B (each at
// least one workspace mesh buffer of size n; A differs from S and B, which may be one buffer;
// their contents are overwritten)
// and keeps the fastest per kind for the rest of the process.  `report` gets one line per kind.
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
        // z_c2r3 is timed on as many rows as its interleaved output fits in one scratch buffer
        auto z3_rows = [&](int w) {
            return std::min((long)n * n, 2L * g.total_c() / force_row3(n)) / w * w;
        };
        std::vector<FftShape> cands;
        for (int R : valid_rs(L))
            for (int w : {1, 2, 4, 8, 16, 32, 64}) {
                const long threads = (long)w * (L / R);
                if (threads < 64 && w < 64) continue;
                if (kind == FK_Z_C2R3 && z3_rows(w) < w) continue;
                const FftShape sp{R, w, true, true};
                if (shape_ok(kind, n, sp) && static_available(kind, n, R, w, true)) cands.push_back(sp);
                FftShape sh{R, w, false};
                if (!shape_ok(kind, n, sh)) continue;
                cands.push_back(sh);
                if (static_available(kind, n, R, w)) cands.push_back(FftShape{R, w, true});
            }
        if (cands.empty()) continue;
        auto launch = [&](const FftShape& sh) -> hipError_t {
            switch (kind) {
                case FK_Z_R2C:
                    return run_z_r2c_shape(reinterpret_cast<const float*>(S), 2L * g.nzp, 0, A, 0, g, tw, 1, 1.0f,
                                           0.0f, sh, st);
                case FK_Z_C2R:
                    return run_z_c2r_shape(A, 0, reinterpret_cast<float*>(B), 2L * g.nzp, 0, g, tw, 1, 1.0f, sh, st);
                case FK_ROWS_Y: return run_rows_shape(OP_ROWS_FWD, S, nullptr, 0, g, tw, kf, 1, sh, st);
                case FK_COLS_X: return run_cols_shape(S, 0, g, tw, 1, sh, st);
                case FK_X_GREEN: return run_x_green_shape(S, S, A, 0, g, tw, kf, 1, sh, st);
                case FK_Y_SPLIT: return run_rows_shape(OP_ROWS_SPLIT, A, S, 0, g, tw, kf, 1, sh, st);
                case FK_X_MULT: return run_x_mult_shape(S, 0, A, 0, g, tw, 1, MUL_IK, 0, 0, kf, 1.0f, sh, st);
                case FK_Z_C2R3:
                    return run_z_c2r3_shape(S, S, S, 0, reinterpret_cast<float*>(A), force_row3(n), 0, g, tw, 1, kf,
                                            sh, st, z3_rows(sh.width));
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
            std::snprintf(line, sizeof(line), "n=%d %s: R=%d width=%d %s %.3f ms (%zu shapes)\n", n,
                          kFftKindName[k], best_sh.R, best_sh.width,
                          best_sh.split ? "static-split" : (best_sh.stat ? "static" : "dynamic"), best,
                          cands.size());
            *report += line;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

// ------------------------------------------------------------------ layout copies

// numpy rfftn layout [x][y][kz] (m + 1 per row) <-> the transposed spectrum [kz][x][y].  One
// thread per mode; the component FFT entry points use them, the hot path does not.
__global__ void k_to_numpy(const float2* spec, long plane, float2* out, int n, int m1) {
    const long total = (long)n * n * m1;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;  // index in the numpy layout
    if (i >= total) return;
    const long xy = i / m1;
    const int kz = (int)(i - xy * m1);
    out[i] = spec[(long)kz * plane + xy];
}

__global__ void k_from_numpy(const float2* in, float2* spec, long plane, int n, int m1) {
    const long nn = (long)n * n;
    const long total = nn * m1;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;  // mode (kz, x, y) in that order
    if (i >= total) return;
    const int kz = (int)(i / nn);
    const long xy = i - kz * nn;
    spec[(long)kz * plane + xy] = in[xy * m1 + kz];
}

hipError_t copy_unpad_to_pad(const float2* src, float2* dst, const Mesh3& g, hipStream_t st) {
    long total = (long)g.n * g.n * (g.m + 1);
    ProfScope ps(PROF_COPY, st);
    hipLaunchKernelGGL(k_from_numpy, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, dst, g.plane, g.n,
                       g.m + 1);
    return hipGetLastError();
}

hipError_t copy_pad_to_unpad(const float2* src, float2* dst, const Mesh3& g, hipStream_t st) {
    long total = (long)g.n * g.n * (g.m + 1);
    ProfScope ps(PROF_COPY, st);
    hipLaunchKernelGGL(k_to_numpy, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, g.plane, dst, g.n,
                       g.m + 1);
    return hipGetLastError();
}

}  // namespace cola
