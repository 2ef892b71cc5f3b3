// Learned coarse-mesh force correction: a periodic 3D convolutional network on the PM_grid = 1
// mesh fields (delta, g) -> force correction dF, with BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for the 3x3x3 convolutions, its training kernels and Adam.  (Sec. 4.4: a force
// mesh below PM_grid = 3 biases haloes through the force resolution.)
//
// Network:  X0 = [delta, g_x, g_y, g_z] * in_scale (padded to 8 channels)
//           Z1 = conv3(W1, X0) + b1, A1 = silu(Z1);  Z2 = conv3(W2, A1) + b2, A2 = silu(Z2);
//           dF = (W3 A2 + b3) * out_scale   (1x1x1, 3 channels)
// conv3 is a periodic cross-correlation over the 27 offsets d in {-1,0,1}^3, tap index
// (dx+1) 9 + (dy+1) 3 + (dz+1).
//
// Layouts: activations BF16, channel-last [voxel][channels], voxel = (x n + y) n + z; conv
// weights BF16 [c_out][tap][c_in]; FP32 master parameters flat (lc_internal.h).  An MFMA
// fragment gives lane l the row (or column) l % 16 and the eight K values 8 (l / 16) .. + 7,
// here eight consecutive channels of one tap: 16 contiguous bytes.  The accumulator gives lane
// l the column l % 16 and rows 4 (l / 16) .. + 3.  (A K order that differs from this one is
// harmless: both operands index K the same way.)

#include <algorithm>
#include <cmath>

#include "cola_internal.h"
#include "lc_internal.h"
#include "force_gather.h"

namespace cola {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// BF16 bits of a float, rounded to nearest even (the hardware conversion, v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float((h & 0xffffu) << 16); }
// logistic function with the hardware reciprocal (1 ulp): its result is stored in BF16
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_g(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

union Frag8 {
    uint4 u;
    bf16x8 v;
    uint16_t h[8];
};

__device__ __forceinline__ uint4 pack8(const uint32_t t[8]) {
    return make_uint4(t[0] | (t[1] << 16), t[2] | (t[3] << 16), t[4] | (t[5] << 16), t[6] | (t[7] << 16));
}

static unsigned blocks_for(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <class K>
static hipError_t allow_lds_lc(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

// ------------------------------------------------------------------ MFMA fragment self-test

// D = A B with A 16x32 and B 32x16 (row-major BF16 bits) and D 16x16 FP32 row-major, through the
// fragment mapping the convolutions use.
__global__ void k_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D) {
    const int l = threadIdx.x;
    const int row = l & 15, kb = l >> 4;
    uint32_t ta[8], tb[8];
    for (int j = 0; j < 8; ++j) {
        ta[j] = A[row * 32 + kb * 8 + j];
        tb[j] = B[(kb * 8 + j) * 16 + row];
    }
    Frag8 a, b;
    a.u = pack8(ta);
    b.u = pack8(tb);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
    for (int q = 0; q < 4; ++q) D[(4 * kb + q) * 16 + row] = acc[q];
}

hipError_t lc_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D, hipStream_t st) {
    hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, st, A, B, D);
    return hipGetLastError();
}

// ------------------------------------------------------------------ 3x3x3 convolution (implicit GEMM)

constexpr int TX = 4, TY = 4, TZ = 16;                // output tile of one block
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;  // with the periodic halo
constexpr int HVOX = HX * HY * HZ;
constexpr int TV = TX * TY * TZ;

__device__ __forceinline__ int wrap_halo(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

enum { EPI_ZA = 0, EPI_A = 1, EPI_DSILU = 2, EPI_OUT = 3, EPI_OUT_STORE = 4 };

// Inputs of the first layer taken straight from the step's fields (instead of a packed X0):
// delta as BF16 (already scaled) and the three force meshes with `row` floats per row and cell z
// of a row at zs z (zs = 3 for the interleaved force mesh, whose g[c] point at component c).
struct FieldSrc {
    const uint16_t* d0;
    const float* g[3];
    long row;
    float s[3];
    int zs = 1;
};
// The output layer fused into the second convolution: dF = (W3 silu(Z2) + b3) * scale added to
// three meshes with `row` floats per row and cell z at zs z.
struct OutDst {
    float* f[3];
    long row;
    const float* w3;
    const float* b3;
    float scale;
    int zs = 1;
};

// The halo of tile `tile` (one voxel, all its C8 vectors of channels, per thread and k) into
// registers, for the tile after the one being computed.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // a register quad (uint4 is a struct)
template <int HK, int C8>
__device__ __forceinline__ void load_halo_regs(u32x4 (&h)[HK][C8], const uint4* __restrict__ ing, int tile, int n,
                                               int nty, int ntz, int tid) {
    const int tz = tile % ntz, ty = (tile / ntz) % nty, tx = tile / (ntz * nty);
#pragma unroll
    for (int k = 0; k < HK; ++k) {
        const int hv = tid + k * 256;
        if (hv < HVOX) {
            const int hz = hv % HZ, hy = (hv / HZ) % HY, hx = hv / (HZ * HY);
            const int gx = wrap_halo(tx * TX + hx - 1, n), gy = wrap_halo(ty * TY + hy - 1, n);
            const int gz = wrap_halo(tz * TZ + hz - 1, n);
            const uint4* src = ing + (((long)gx * n + gy) * n + gz) * C8;
#pragma unroll
            for (int c8 = 0; c8 < C8; ++c8) h[k][c8] = *reinterpret_cast<const u32x4*>(src + c8);
        }
    }
}

// out[v][co] = sum_tap sum_ci W[co][tap][ci] in[v + d_tap][ci] + bias[co], then
//   EPI_ZA: out = Z, out2 = silu(Z);  EPI_A: out = silu(Z);  EPI_DSILU: out = Z * silu'(prev[v][co]).
// in: [V][CINP] BF16; W: [16 NB][27][CINP] BF16; out: [V][16 NB].  Block = 4 waves on a 4x4x16
// tile, wave w computing the rows x0 + w, y0 + 0..3 (16 voxels along z each) for all outputs.
//   EPI_OUT: the output layer, dF = (W3 silu(Z) + b3) * scale, added to the meshes of `od`;
//   EPI_OUT_STORE: the same, stored instead of added.
// FIELDS (first layer only, CINP = 8): the halo is built from `fs` instead of `in`.
// At least three waves per SIMD, i.e. three blocks per CU (at most 168 VGPRs): with two, the
// 16-channel layers left the matrix cores
// and LDS idle through each tile's barriers (0.50 -> 0.41 ms per launch on 256^3); four would
// spill the 16-channel output layer.
template <int CINP, int NB, int EPI, bool FIELDS = false>
__global__ void __launch_bounds__(256, 3) k_conv3_mfma(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                    const float* __restrict__ bias, uint16_t* out, uint16_t* out2,
                                                    const uint16_t* __restrict__ prev, int n, int tiles, FieldSrc fs,
                                                    OutDst od) {
    constexpr int COP = 16 * NB;
    constexpr int KTOT = 27 * CINP;
    constexpr int KSTEPS = (KTOT + 31) / 32;
    constexpr int KUNROLL = NB == 1 ? 2 : KSTEPS;
    constexpr int C8 = CINP / 8;
    extern __shared__ uint4 smem[];
    uint4* sw = smem;                      // weights, COP * 27 * C8 vectors
    uint4* sh = smem + COP * 27 * C8;      // halo, HVOX * C8 vectors
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint4* wg = reinterpret_cast<const uint4*>(w);
    for (int i = tid; i < COP * 27 * C8; i += 256) sw[i] = wg[i];
    const int nty = n / TY, ntz = n / TZ;
    const int m = lane & 15, kb = lane >> 4;
    const uint4* ing = reinterpret_cast<const uint4*>(in);
    // Up to 16 input channels the next tile's halo is requested into registers while the current
    // tile is computed (one halo voxel, all its channels, per thread and k), so a tile's loads no
    // longer stand between its barrier and its matrix-core loop.
    constexpr int HK = (HVOX + 255) / 256;
    constexpr bool PREFETCH = !FIELDS && C8 <= 2;
    constexpr int PK = PREFETCH ? HK : 1, PC = PREFETCH ? C8 : 1;
    u32x4 hreg[PK][PC];
    if constexpr (PREFETCH)
        if ((int)blockIdx.x < tiles) load_halo_regs<PK, PC>(hreg, ing, blockIdx.x, n, nty, ntz, tid);
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int tz = tile % ntz, ty = (tile / ntz) % nty, tx = tile / (ntz * nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        const int y0v = y0;
        __syncthreads();  // the previous tile's readers are done with the halo
        if constexpr (PREFETCH) {
#pragma unroll
            for (int k = 0; k < PK; ++k) {
                const int hv = tid + k * 256;
                if (hv < HVOX)
#pragma unroll
                    for (int c8 = 0; c8 < PC; ++c8) *reinterpret_cast<u32x4*>(sh + hv * C8 + c8) = hreg[k][c8];
            }
        } else
#pragma unroll
        for (int k = 0; k < HK; ++k) {  // one halo voxel (all its channels) per thread
            const int hv = tid + k * 256;
            if (hv < HVOX) {
                const int hz = hv % HZ, hy = (hv / HZ) % HY, hx = hv / (HZ * HY);
                const int gx = wrap_halo(x0 + hx - 1, n), gy = wrap_halo(y0 + hy - 1, n);
                const int gz = wrap_halo(z0 + hz - 1, n);
                if constexpr (FIELDS) {
                    static_assert(C8 == 1, "field input has 4 channels (padded to 8)");
                    const long v = ((long)gx * n + gy) * n + gz;
                    const long o = ((long)gx * n + gy) * fs.row + (long)gz * fs.zs;
                    // a channel with a zero input scale is not read (a density-only network)
                    const float g0 = fs.s[0] != 0.0f ? fs.g[0][o] * fs.s[0] : 0.0f;
                    const float g1 = fs.s[1] != 0.0f ? fs.g[1][o] * fs.s[1] : 0.0f;
                    const float g2 = fs.s[2] != 0.0f ? fs.g[2][o] * fs.s[2] : 0.0f;
                    sh[hv] = make_uint4(fs.d0[v] | (f2bf(g0) << 16), f2bf(g1) | (f2bf(g2) << 16), 0u, 0u);
                } else {
                    const uint4* src = ing + (((long)gx * n + gy) * n + gz) * C8;
#pragma unroll
                    for (int c8 = 0; c8 < C8; ++c8) sh[hv * C8 + c8] = src[c8];
                }
            }
        }
        __syncthreads();
        // the output layer's force-mesh values are requested first, the next halo after them (loads
        // complete in order, so the epilogue does not wait for the halo)
        constexpr bool FO_EARLY = EPI == EPI_OUT && NB == 1;  // 32 channels: no registers to spare
        float fo[3] = {0.0f, 0.0f, 0.0f};
        long fo_off = 0;
        if constexpr (FO_EARLY) {
            const int lx = tid >> 6, ly = (tid >> 4) & 3, lz = tid & 15;  // voxel tid of the tile
            fo_off = ((long)(x0 + lx) * n + (y0v + ly)) * od.row + (long)(z0 + lz) * od.zs;
#pragma unroll
            for (int c = 0; c < 3; ++c) fo[c] = od.f[c][fo_off];
        }
        if constexpr (PREFETCH)
            if (tile + (int)gridDim.x < tiles) load_halo_regs<PK, PC>(hreg, ing, tile + gridDim.x, n, nty, ntz, tid);
        f32x4 acc[4][NB];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[r][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        // 16-channel layers: unrolled by two, which leaves the registers for the prefetched halo
        // (fully unrolled they needed 150-168)
#pragma unroll KUNROLL
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int k = ks * 32 + kb * 8;
            const int tap = k / CINP, c0 = k % CINP;
            Frag8 bf[NB], af[4];
            if (tap < 27) {
                const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
#pragma unroll
                for (int b = 0; b < NB; ++b) bf[b].u = sw[((b * 16 + m) * 27 + tap) * C8 + c0 / 8];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int hv = ((wave + 1 + dx) * HY + (r + 1 + dy)) * HZ + (m + 1 + dz);
                    af[r].u = sh[hv * C8 + c0 / 8];
                }
            } else {
#pragma unroll
                for (int b = 0; b < NB; ++b) bf[b].u = make_uint4(0, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) af[r].u = make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[r][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r].v, bf[b].v, acc[r][b], 0, 0, 0);
        }
        // lane holds voxels z0 + 4 kb + q of the row, output channel co = 16 b + m
        if constexpr (EPI == EPI_OUT || EPI == EPI_OUT_STORE) {
            // A2 (rounded to BF16 as in the stored-activation path) goes to LDS as [voxel][COP + 1]
            // floats in the halo's space; then one thread per voxel forms the three outputs
            constexpr int SP = COP + 1;
            static_assert(TV * SP * 4 <= HVOX * CINP * 2, "staging must fit in the halo space");
            float* stage = reinterpret_cast<float*>(sh);
            __syncthreads();  // every wave is done reading the halo
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float bb = bias[b * 16 + m];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        stage[((wave * 4 + r) * 16 + 4 * kb + q) * SP + b * 16 + m] =
                            bf2f(f2bf(silu_f(acc[r][b][q] + bb)));
                }
            __syncthreads();
            float y0 = od.b3[0], y1 = od.b3[1], y2 = od.b3[2];
#pragma unroll
            for (int co = 0; co < COP; ++co) {
                const float a = stage[tid * SP + co];
                y0 += od.w3[co] * a;
                y1 += od.w3[COP + co] * a;
                y2 += od.w3[2 * COP + co] * a;
            }
            if constexpr (EPI == EPI_OUT_STORE) {
                const int lx = tid >> 6, ly = (tid >> 4) & 3, lz = tid & 15;  // voxel tid of the tile
                const long o = ((long)(x0 + lx) * n + (y0v + ly)) * od.row + (long)(z0 + lz) * od.zs;
                od.f[0][o] = y0 * od.scale;
                od.f[1][o] = y1 * od.scale;
                od.f[2][o] = y2 * od.scale;
            } else if constexpr (FO_EARLY) {
                od.f[0][fo_off] = fo[0] + y0 * od.scale;
                od.f[1][fo_off] = fo[1] + y1 * od.scale;
                od.f[2][fo_off] = fo[2] + y2 * od.scale;
            } else {
                const int lx = tid >> 6, ly = (tid >> 4) & 3, lz = tid & 15;  // voxel tid of the tile
                const long o = ((long)(x0 + lx) * n + (y0v + ly)) * od.row + (long)(z0 + lz) * od.zs;
                od.f[0][o] += y0 * od.scale;
                od.f[1][o] += y1 * od.scale;
                od.f[2][o] += y2 * od.scale;
            }
            continue;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long vrow = ((long)(x0 + wave) * n + (y0 + r)) * n + z0 + 4 * kb;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int co = b * 16 + m;
                const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const long o = (vrow + q) * COP + co;
                    const float z = acc[r][b][q] + bb;
                    if (EPI == EPI_ZA) {
                        out[o] = (uint16_t)f2bf(z);
                        out2[o] = (uint16_t)f2bf(silu_f(z));
                    } else if (EPI == EPI_A) {
                        out[o] = (uint16_t)f2bf(silu_f(z));
                    } else {
                        out[o] = (uint16_t)f2bf(z * silu_g(bf2f(prev[o])));
                    }
                }
            }
        }
    }
}

// The first layer of a density-only network (the force channels' input scales are zero): the
// only input channel is the BF16 density d0 [V], so K = 27 taps (padded to 32) instead of 27 taps
// x 8 channels -- one MFMA K step per output block instead of seven, six of which would multiply
// zeros.  Lane (m, kb) takes taps 8 kb .. 8 kb + 7 of voxel m's row; the weights are channel 0 of
// the packed [16 NB][27][8] layer-1 weights, staged as [16 NB][32] (taps 27..31 zero).  Tiles,
// halo and epilogue (A1 = silu(Z1)) as in k_conv3_mfma.
template <int NB>
__global__ void __launch_bounds__(256, 3) k_conv3_dens(const uint16_t* __restrict__ d0, const uint16_t* __restrict__ w,
                                                    const float* __restrict__ bias, uint16_t* out, int n, int tiles) {
    constexpr int COP = 16 * NB;
    extern __shared__ uint4 smem[];
    uint4* sw = smem;                                          // [COP][32] BF16: COP * 4 vectors
    uint16_t* sh = reinterpret_cast<uint16_t*>(smem + COP * 4);  // halo densities, HVOX BF16
    uint16_t* swh = reinterpret_cast<uint16_t*>(sw);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < COP * 32; i += 256) {
        const int co = i >> 5, tap = i & 31;
        swh[i] = tap < 27 ? w[(co * 27 + tap) * 8] : (uint16_t)0;
    }
    const int nty = n / TY, ntz = n / TZ;
    const int m = lane & 15, kb = lane >> 4;
    // halo offsets of this lane's eight taps relative to the voxel's own halo position (negative
    // for the lower neighbours); taps 27..31 are padding and read nothing
    int toff[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int tap = kb * 8 + j;
        const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
        toff[j] = (dx * HY + dy) * HZ + dz;
    }
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int tz = tile % ntz, ty = (tile / ntz) % nty, tx = tile / (ntz * nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        __syncthreads();  // the previous tile's readers are done with the halo (and the weights are staged)
        for (int hv = tid; hv < HVOX; hv += 256) {
            const int hz = hv % HZ, hy = (hv / HZ) % HY, hx = hv / (HZ * HY);
            const int gx = wrap_halo(x0 + hx - 1, n), gy = wrap_halo(y0 + hy - 1, n), gz = wrap_halo(z0 + hz - 1, n);
            sh[hv] = d0[((long)gx * n + gy) * n + gz];
        }
        __syncthreads();
        Frag8 bf[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) bf[b].u = sw[(b * 16 + m) * 4 + kb];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int hv0 = ((wave + 1) * HY + (r + 1)) * HZ + (m + 1);
            Frag8 af;
#pragma unroll
            for (int j = 0; j < 8; ++j) af.h[j] = kb * 8 + j < 27 ? sh[hv0 + toff[j]] : (uint16_t)0;
            const long vrow = ((long)(x0 + wave) * n + (y0 + r)) * n + z0 + 4 * kb;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af.v, bf[b].v, f32x4{0.f, 0.f, 0.f, 0.f},
                                                                          0, 0, 0);
                const int co = b * 16 + m;
                const float bb = bias[co];
#pragma unroll
                for (int q = 0; q < 4; ++q) out[(vrow + q) * COP + co] = (uint16_t)f2bf(silu_f(acc[q] + bb));
            }
        }
    }
}

template <int NB>
static hipError_t run_conv_dens(const uint16_t* d0, const uint16_t* w, const float* bias, uint16_t* out, int n,
                                hipStream_t st) {
    const long tiles = (long)(n / TX) * (n / TY) * (n / TZ);
    const size_t lds = (size_t)16 * NB * 32 * 2 + (size_t)HVOX * 2;
    ProfScope ps(PROF_LC_CONV, st, 1);  // tag: input channels
    hipLaunchKernelGGL(k_conv3_dens<NB>, dim3((unsigned)std::min<long>(tiles, 4096)), dim3(256), lds, st, d0, w, bias,
                       out, n, (int)tiles);
    return hipGetLastError();
}

static long conv_tiles(int n) { return (long)(n / TX) * (n / TY) * (n / TZ); }

template <int CINP, int NB, int EPI, bool FIELDS = false>
static hipError_t run_conv(const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, uint16_t* out2,
                           const uint16_t* prev, int n, hipStream_t st, const FieldSrc& fs = FieldSrc{},
                           const OutDst& od = OutDst{}) {
    const long tiles = conv_tiles(n);
    const size_t lds = (size_t)16 * NB * 27 * CINP * 2 + (size_t)HVOX * CINP * 2;
    auto kern = k_conv3_mfma<CINP, NB, EPI, FIELDS>;
    if (hipError_t e = allow_lds_lc(kern, lds); e != hipSuccess) return e;
    ProfScope ps(PROF_LC_CONV, st, CINP);  // tag: input channels (padded)
    hipLaunchKernelGGL(kern, dim3((unsigned)std::min<long>(tiles, 4096)), dim3(256), lds, st, in, w, bias, out, out2,
                       prev, n, (int)tiles, fs, od);
    return hipGetLastError();
}

// ------------------------------------------------------------------ band-pass output weight

// out[c] (+)= T[c] + beta (K T[c] - K K T[c]), K the periodic [1, 2, 1] / 4 smoothing along each
// axis; T dense [3][n^3], out with `row` floats per (x, y) row and cell z at zs z.  One block per
// 8 x 8 x 16 tile:
// T with a halo of two cells goes to LDS, K is applied as three axis passes (giving K T on the
// tile plus one cell), then three more (K K T on the tile); the passes ping-pong between two
// LDS buffers.
constexpr int BX = 8, BY = 8, BZ = 16;
constexpr int BH = (BX + 4) * (BY + 4) * (BZ + 4);

__device__ __forceinline__ float k121(float a, float b, float c) { return 0.25f * a + 0.5f * b + 0.25f * c; }

__global__ void __launch_bounds__(256) k_lc_band(const float* __restrict__ T, int n, float beta, float* o0, float* o1,
                                                 float* o2, long row, int zs, int accumulate) {
    __shared__ float bufa[BH], bufb[BH];
    const int tid = threadIdx.x;
    const int ntz = n / BZ, nty = n / BY;
    const int tile = blockIdx.x;
    const int z0 = (tile % ntz) * BZ, y0 = ((tile / ntz) % nty) * BY, x0 = (tile / (ntz * nty)) * BX;
    const long V = (long)n * n * n;
    float* outs[3] = {o0, o1, o2};
    for (int c = 0; c < 3; ++c) {
        const float* src = T + c * V;
        // H: (BX+4) x (BY+4) x (BZ+4), origin at (x0-2, y0-2, z0-2)
        constexpr int HX = BX + 4, HY = BY + 4, HZ = BZ + 4;
        for (int i = tid; i < BH; i += 256) {
            const int hz = i % HZ, hy = (i / HZ) % HY, hx = i / (HZ * HY);
            const int gx = (x0 + hx - 2 + n) % n, gy = (y0 + hy - 2 + n) % n, gz = (z0 + hz - 2 + n) % n;
            bufa[i] = src[((long)gx * n + gy) * n + gz];
        }
        __syncthreads();
        float tc[4], kt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = tid + 256 * j, lz = v % BZ, ly = (v / BZ) % BY, lx = v / (BZ * BY);
            tc[j] = bufa[((lx + 2) * HY + ly + 2) * HZ + lz + 2];
        }
        // z pass: HX x HY x (BZ+2)
        constexpr int Z1 = BZ + 2;
        for (int i = tid; i < HX * HY * Z1; i += 256) {
            const int z = i % Z1, xy = i / Z1;
            const float* h = bufa + xy * HZ + z;
            bufb[i] = k121(h[0], h[1], h[2]);
        }
        __syncthreads();
        // y pass: HX x (BY+2) x Z1
        constexpr int Y1 = BY + 2;
        for (int i = tid; i < HX * Y1 * Z1; i += 256) {
            const int z = i % Z1, y = (i / Z1) % Y1, x = i / (Z1 * Y1);
            const float* h = bufb + (x * HY + y) * Z1 + z;
            bufa[i] = k121(h[0], h[Z1], h[2 * Z1]);
        }
        __syncthreads();
        // x pass: (BX+2) x Y1 x Z1 = K T on the tile plus one cell
        constexpr int X1 = BX + 2;
        for (int i = tid; i < X1 * Y1 * Z1; i += 256) {
            const int yz = i % (Y1 * Z1), x = i / (Y1 * Z1);
            const float* h = bufa + x * Y1 * Z1 + yz;
            bufb[i] = k121(h[0], h[Y1 * Z1], h[2 * Y1 * Z1]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = tid + 256 * j, lz = v % BZ, ly = (v / BZ) % BY, lx = v / (BZ * BY);
            kt[j] = bufb[((lx + 1) * Y1 + ly + 1) * Z1 + lz + 1];
        }
        // second smoothing: z pass X1 x Y1 x BZ
        for (int i = tid; i < X1 * Y1 * BZ; i += 256) {
            const int z = i % BZ, xy = i / BZ;
            const float* h = bufb + xy * Z1 + z;
            bufa[i] = k121(h[0], h[1], h[2]);
        }
        __syncthreads();
        // y pass: X1 x BY x BZ
        for (int i = tid; i < X1 * BY * BZ; i += 256) {
            const int z = i % BZ, y = (i / BZ) % BY, x = i / (BZ * BY);
            const float* h = bufa + (x * Y1 + y) * BZ + z;
            bufb[i] = k121(h[0], h[BZ], h[2 * BZ]);
        }
        __syncthreads();
        float* dst = outs[c];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = tid + 256 * j, lz = v % BZ, ly = (v / BZ) % BY, lx = v / (BZ * BY);
            const float* h = bufb + (lx * BY + ly) * BZ + lz;
            const float kkt = k121(h[0], h[BY * BZ], h[2 * BY * BZ]);
            const float val = tc[j] + beta * (kt[j] - kkt);
            const long o = ((long)(x0 + lx) * n + (y0 + ly)) * row + (long)(z0 + lz) * zs;
            if (accumulate) dst[o] += val;
            else dst[o] = val;
        }
        __syncthreads();  // the buffers are reused by the next component
    }
}

hipError_t lc_band(const float* T, int n, float beta, float* const out[3], long row, int accumulate,
                   hipStream_t st, int zs) {
    ProfScope ps(PROF_LC_MISC, st);
    const long tiles = (long)(n / BX) * (n / BY) * (n / BZ);
    hipLaunchKernelGGL(k_lc_band, dim3((unsigned)tiles), dim3(256), 0, st, T, n, beta, out[0], out[1], out[2], row,
                       zs, accumulate);
    return hipGetLastError();
}

// ------------------------------------------------------------------ weight gradient

constexpr int SDZ = TV + 8;       // padded channel row of the staged upstream gradient
constexpr int SXP = HVOX + 8;     // padded channel row of the staged input halo

// dW[co][ci][tap] += sum_v dZ[v][co] X[v + d_tap][ci] and db[co] += sum_v dZ[v][co] over the
// tiles of this block: MFMA with M = output channels, N = input channels, K = 32 voxels (two
// 16-voxel z rows); wave w owns the taps w, w + 4, ...; one atomic flush per block.
template <int CINP, int MB>
__global__ void __launch_bounds__(256) k_conv3_wgrad(const uint16_t* __restrict__ dz, const uint16_t* __restrict__ x,
                                                     float* dw, float* db, int n, int cin, int tiles) {
    constexpr int COP = 16 * MB;
    constexpr int NBN = (CINP + 15) / 16;
    constexpr int TPW = 7;
    extern __shared__ uint4 smem[];
    uint16_t* sdz = reinterpret_cast<uint16_t*>(smem);  // [COP][SDZ], channel-major
    uint16_t* sx = sdz + COP * SDZ;                      // [CINP][SXP], channel-major
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kb = lane >> 4;
    const int nty = n / TY, ntz = n / TZ;
    const uint4* dzg = reinterpret_cast<const uint4*>(dz);
    const uint4* xg = reinterpret_cast<const uint4*>(x);
    f32x4 acc[TPW][MB][NBN];
#pragma unroll
    for (int a = 0; a < TPW; ++a)
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NBN; ++j) acc[a][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int tz = tile % ntz, ty = (tile / ntz) % nty, tx = tile / (ntz * nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        __syncthreads();
        for (int i = tid; i < TV * (COP / 8); i += 256) {
            const int c8 = i % (COP / 8), tv = i / (COP / 8);
            const int lz = tv % TZ, ly = (tv / TZ) % TY, lx = tv / (TZ * TY);
            const long v = ((long)(x0 + lx) * n + (y0 + ly)) * n + (z0 + lz);
            Frag8 f;
            f.u = dzg[v * (COP / 8) + c8];
#pragma unroll
            for (int h = 0; h < 8; ++h) sdz[(c8 * 8 + h) * SDZ + tv] = f.h[h];
        }
#pragma unroll
        for (int k = 0; k < (HVOX + 255) / 256; ++k) {
            const int hv = tid + k * 256;
            if (hv < HVOX) {
                const int hz = hv % HZ, hy = (hv / HZ) % HY, hx = hv / (HZ * HY);
                const int gx = wrap_halo(x0 + hx - 1, n), gy = wrap_halo(y0 + hy - 1, n);
                const int gz = wrap_halo(z0 + hz - 1, n);
                const uint4* src = xg + (((long)gx * n + gy) * n + gz) * (CINP / 8);
#pragma unroll
                for (int c8 = 0; c8 < CINP / 8; ++c8) {
                    Frag8 f;
                    f.u = src[c8];
#pragma unroll
                    for (int h = 0; h < 8; ++h) sx[(c8 * 8 + h) * SXP + hv] = f.h[h];
                }
            }
        }
        __syncthreads();
        if (tid < COP) {
            float s = 0.0f;
            for (int tv = 0; tv < TV; ++tv) s += bf2f(sdz[tid * SDZ + tv]);
            bacc += s;
        }
        for (int ksv = 0; ksv < TV / 32; ++ksv) {
            const int row = ksv * 2 + (kb >> 1), zh = (kb & 1) * 8;  // voxels z = zh .. zh + 7 of row
            const int lx = row / TY, ly = row % TY;
            Frag8 af[MB];
#pragma unroll
            for (int i = 0; i < MB; ++i)
                af[i].u = *reinterpret_cast<const uint4*>(sdz + (i * 16 + m) * SDZ + row * TZ + zh);
#pragma unroll
            for (int a = 0; a < TPW; ++a) {
                const int tap = wave + 4 * a;
                if (tap < 27) {
                    const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dzz = tap % 3 - 1;
                    const int hv0 = ((lx + 1 + dx) * HY + (ly + 1 + dy)) * HZ + (zh + 1 + dzz);
#pragma unroll
                    for (int j = 0; j < NBN; ++j) {
                        const int ci = j * 16 + m;
                        Frag8 bfr;
                        if (ci < CINP) {
                            const uint16_t* p = sx + ci * SXP + hv0;
                            uint32_t t8[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q) t8[q] = p[q];
                            bfr.u = pack8(t8);
                        } else {
                            bfr.u = make_uint4(0, 0, 0, 0);
                        }
#pragma unroll
                        for (int i = 0; i < MB; ++i)
                            acc[a][i][j] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i].v, bfr.v, acc[a][i][j], 0, 0, 0);
                    }
                }
            }
        }
    }
    // flush: lane holds rows co = 16 i + 4 kb + q, column ci = 16 j + m
#pragma unroll
    for (int a = 0; a < TPW; ++a) {
        const int tap = wave + 4 * a;
        if (tap < 27) {
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NBN; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int co = i * 16 + 4 * kb + q, ci = j * 16 + m;
                        if (ci < cin) atomicAdd(&dw[((long)co * cin + ci) * 27 + tap], acc[a][i][j][q]);
                    }
        }
    }
    if (tid < COP) atomicAdd(&db[tid], bacc);
}

template <int CINP, int MB>
static hipError_t run_wgrad(const uint16_t* dz, const uint16_t* x, float* dw, float* db, int n, int cin,
                            hipStream_t st) {
    const long tiles = conv_tiles(n);
    const size_t lds = (size_t)16 * MB * SDZ * 2 + (size_t)CINP * SXP * 2;
    auto kern = k_conv3_wgrad<CINP, MB>;
    if (hipError_t e = allow_lds_lc(kern, lds); e != hipSuccess) return e;
    ProfScope ps(PROF_LC_WGRAD, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)std::min<long>(tiles, 1024)), dim3(256), lds, st, dz, x, dw, db, n, cin,
                       (int)tiles);
    return hipGetLastError();
}

// ------------------------------------------------------------------ input packing, output layer

__device__ __forceinline__ long mesh_off(long v, int n, long row) {
    const long r = v / n;
    return r * row + (v - r * n);
}

__global__ void k_lc_pack(const float* delta, const float* gx, const float* gy, const float* gz, long row, int n,
                          float s0, float s1, float s2, float s3, uint16_t* x0) {
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long)n * n * n) return;
    const long o = mesh_off(v, n, row);
    reinterpret_cast<uint4*>(x0)[v] = make_uint4(f2bf(delta[o] * s0) | (f2bf(gx[o] * s1) << 16),
                                                 f2bf(gy[o] * s2) | (f2bf(gz[o] * s3) << 16), 0u, 0u);
}

// delta * s0 as compact BF16 (one value per voxel), the first-layer input saved before the
// transform overwrites the density
__global__ void k_lc_pack_delta(const float* delta, long row, int n, float s0, uint16_t* d0) {
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long)n * n * n) return;
    d0[v] = (uint16_t)f2bf(delta[mesh_off(v, n, row)] * s0);
}

// dF[c] = (W3 A2[v] + b3) * out_scale, written to (or added into) three dense meshes of `row` floats
// per row (the training path; the step's output layer is the fused EPI_OUT epilogue).
template <int C>
__global__ void k_lc_out(const uint16_t* a2, const float* w3, const float* b3, float out_scale, int n, long row,
                         float* fx, float* fy, float* fz, int accumulate) {
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long)n * n * n) return;
    float y0 = b3[0], y1 = b3[1], y2 = b3[2];
    const uint4* p = reinterpret_cast<const uint4*>(a2 + v * C);
#pragma unroll
    for (int c8 = 0; c8 < C / 8; ++c8) {
        Frag8 f;
        f.u = p[c8];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const float a = bf2f(f.h[h]);
            const int co = c8 * 8 + h;
            y0 += w3[co] * a;
            y1 += w3[C + co] * a;
            y2 += w3[2 * C + co] * a;
        }
    }
    const long o = mesh_off(v, n, row);
    if (accumulate) {
        fx[o] += y0 * out_scale;
        fy[o] += y1 * out_scale;
        fz[o] += y2 * out_scale;
    } else {
        fx[o] = y0 * out_scale;
        fy[o] = y1 * out_scale;
        fz[o] = y2 * out_scale;
    }
}

// Backward of the output layer: dY = d_dF * out_scale; dZ2 = (W3^T dY) silu'(Z2);
// dW3 += sum_v dY A2^T, db3 += sum_v dY (wave shuffles, then one atomic per value and block).
template <int C>
__global__ void __launch_bounds__(256) k_lc_out_back(const float* ddf, const uint16_t* z2, const float* w3,
                                                     float out_scale, int n, uint16_t* dz2, float* dw3, float* db3) {
    constexpr int NV = 3 * (C + 1);
    __shared__ float red[4][NV];
    const long V = (long)n * n * n;
    float part[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) part[i] = 0.0f;
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long)gridDim.x * blockDim.x) {
        const float dy0 = ddf[v] * out_scale, dy1 = ddf[V + v] * out_scale, dy2 = ddf[2 * V + v] * out_scale;
        part[0] += dy0;
        part[C + 1] += dy1;
        part[2 * (C + 1)] += dy2;
        const uint4* zp = reinterpret_cast<const uint4*>(z2 + v * C);
        uint4* dp = reinterpret_cast<uint4*>(dz2 + v * C);
#pragma unroll
        for (int c8 = 0; c8 < C / 8; ++c8) {
            Frag8 f;
            f.u = zp[c8];
            uint32_t t[8];
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const int co = c8 * 8 + h;
                const float z = bf2f(f.h[h]);
                const float a = silu_f(z);
                const float da = w3[co] * dy0 + w3[C + co] * dy1 + w3[2 * C + co] * dy2;
                t[h] = f2bf(da * silu_g(z));
                part[1 + co] += dy0 * a;
                part[C + 2 + co] += dy1 * a;
                part[2 * C + 3 + co] += dy2 * a;
            }
            dp[c8] = pack8(t);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        float s = part[i];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) red[wave][i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NV; i += blockDim.x) {
        const float s = red[0][i] + red[1][i] + red[2][i] + red[3][i];
        const int c = i / (C + 1), j = i % (C + 1);
        if (j == 0) atomicAdd(&db3[c], s);
        else atomicAdd(&dw3[c * C + j - 1], s);
    }
}

// ------------------------------------------------------------------ particle loss

__device__ __forceinline__ void cic_abs(float pos, float inv_h, int n, int& i0, int& i1, float& f) {
    const float u = pos * inv_h;
    const float fl = floorf(u);
    f = u - fl;
    int m = (int)fl % n;
    m = m < 0 ? m + n : m;
    m = min(max(m, 0), n - 1);  // a non-finite position still maps inside the mesh
    i0 = m;
    i1 = m + 1 == n ? 0 : m + 1;
}

// stats[1] += sum_p |g3 - g1|^2  (float64)
__global__ void k_lc_denom(const float* g1x, const float* g1y, const float* g1z, const float* g3x,
                           const float* g3y, const float* g3z, long np, double* stats) {
    __shared__ double red[256];
    double s = 0.0;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (long)gridDim.x * blockDim.x) {
        const double a = g3x[p] - g1x[p], b = g3y[p] - g1y[p], c = g3z[p] - g1z[p];
        s += a * a + b * b + c * c;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&stats[1], red[0]);
}

// r_p = g1 + G[dF]_p - g3;  stats[0] += |r|^2 / denom;  d_dF += G^T (2 r / denom)  (G = CIC gather
// at absolute positions on the dense n^3 mesh).
__global__ void k_lc_loss(const float* px, const float* py, const float* pz, long np, int n, float inv_h,
                          const float* dfx, const float* dfy, const float* dfz, const float* g1x, const float* g1y,
                          const float* g1z, const float* g3x, const float* g3y, const float* g3z, double* stats,
                          float* ddf) {
    __shared__ double red[256];
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double l2 = 0.0;
    if (p < np) {
        int ix0, ix1, iy0, iy1, iz0, iz1;
        float fx, fy, fz;
        cic_abs(px[p], inv_h, n, ix0, ix1, fx);
        cic_abs(py[p], inv_h, n, iy0, iy1, fy);
        cic_abs(pz[p], inv_h, n, iz0, iz1, fz);
        const int ix[2] = {ix0, ix1}, iy[2] = {iy0, iy1}, iz[2] = {iz0, iz1};
        const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
        float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const long v = ((long)ix[a] * n + iy[b]) * n + iz[c];
                    const float w = wx[a] * wy[b] * wz[c];
                    g0 += w * dfx[v];
                    g1 += w * dfy[v];
                    g2 += w * dfz[v];
                }
        const float r0 = g1x[p] + g0 - g3x[p], r1 = g1y[p] + g1 - g3y[p], r2 = g1z[p] + g2 - g3z[p];
        const double inv = 1.0 / stats[1];
        l2 = ((double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2) * inv;
        const float s = (float)(2.0 * inv);
        const long V = (long)n * n * n;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const long v = ((long)ix[a] * n + iy[b]) * n + iz[c];
                    const float w = wx[a] * wy[b] * wz[c] * s;
                    atomicAdd(&ddf[v], w * r0);
                    atomicAdd(&ddf[V + v], w * r1);
                    atomicAdd(&ddf[2 * V + v], w * r2);
                }
    }
    red[threadIdx.x] = l2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&stats[0], red[0]);
}

// ------------------------------------------------------------------ Adam, weight packing

// Adam (Kingma & Ba 2015) on FP32 master parameters with bias corrections c1 = 1 - b1^t,
// c2 = 1 - b2^t; the gradient is cleared for the next accumulation.
__global__ void k_lc_adam(float* p, float* g, float* m, float* v, long np, float lr, float b1, float b2, float eps,
                          float c1, float c2) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        g[i] = 0.0f;
    }
}

//   wb1[co][tap][ci < 8] = w1[co][ci][tap] (0 for ci >= 4);  wb2[co][tap][ci] = w2[co][ci][tap];
//   wt2[ci][tap][co] = w2[co][ci][26 - tap]   (offset -d: the data gradient of layer 2).
__global__ void k_lc_pack_weights(const float* w1, const float* w2, int C, uint16_t* wb1, uint16_t* wb2,
                                  uint16_t* wt2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C * 27 * 8) {
        const int ci = i % 8, tap = (i / 8) % 27, co = i / (8 * 27);
        wb1[i] = ci < 4 ? (uint16_t)f2bf(w1[(co * 4 + ci) * 27 + tap]) : (uint16_t)0;
    }
    if (i < C * 27 * C) {
        const int c_in = i % C, tap = (i / C) % 27, c_out = i / (C * 27);
        wb2[i] = (uint16_t)f2bf(w2[(c_out * C + c_in) * 27 + tap]);
        // transposed weights: output channel c_out of the data gradient is input channel c_out of
        // layer 2, its input channel c_in is layer 2's output channel c_in
        wt2[i] = (uint16_t)f2bf(w2[(c_in * C + c_out) * 27 + (26 - tap)]);
    }
}

// ------------------------------------------------------------------ positions, gather, copies

__global__ void k_positions(const float* x, long n_per_real, long total, int n_part, int axis, float cell, float qoff,
                            float box, float* pos) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const long idx = i % n_per_real;
    const long np2 = (long)n_part * n_part;
    const int id = axis == 0 ? (int)(idx / np2) : (axis == 1 ? (int)((idx / n_part) % n_part) : (int)(idx % n_part));
    float u = (float)id * cell + qoff + x[i];
    u -= box * floorf(u / box);
    pos[i] = u >= box ? u - box : u;
}

// CIC interpolation of the interleaved force mesh (rows of `row` floats, cell z of a row at 3 z,
// ghost cells z = n, n + 1) to absolute positions.
__global__ void k_gather_abs(const float* px, const float* py, const float* pz, long np, int n, float inv_h,
                             const float* F, long row, float* ox, float* oy, float* oz) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    int ix0, ix1, iy0, iy1, iz0, iz1;
    float ux, uy, uz;
    cic_abs(px[p], inv_h, n, ix0, ix1, ux);
    cic_abs(py[p], inv_h, n, iy0, iy1, uy);
    cic_abs(pz[p], inv_h, n, iz0, iz1, uz);
    float g[3];
    gather_interleaved(F, row, n, ix0, iy0, iz0, ux, uy, uz, g);
    ox[p] = g[0];
    oy[p] = g[1];
    oz[p] = g[2];
}

__global__ void k_mesh_unpad(const float* src, long row, int n, float* dst) {
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long)n * n * n) return;
    dst[v] = src[mesh_off(v, n, row)];
}

// The three components of the interleaved force mesh into three dense n^3 arrays.
__global__ void k_mesh_unpad3(const float* F, long row, int n, float* g0, float* g1, float* g2) {
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long)n * n * n) return;
    const long r = v / n;
    const float* c = F + r * row + 3 * (v - r * n);
    g0[v] = c[0];
    g1[v] = c[1];
    g2[v] = c[2];
}

// ------------------------------------------------------------------ host launchers

hipError_t lc_pack_weights(const float* w1, const float* w2, int C, uint16_t* wb1, uint16_t* wb2, uint16_t* wt2,
                           hipStream_t st) {
    ProfScope ps(PROF_LC_MISC, st);
    hipLaunchKernelGGL(k_lc_pack_weights, dim3(blocks_for((long)C * 27 * std::max(C, 8), 256)), dim3(256), 0, st,
                       w1, w2, C, wb1, wb2, wt2);
    return hipGetLastError();
}

hipError_t lc_pack(const float* delta, const float* const g[3], long row, int n, const float in_scale[4],
                   uint16_t* x0, hipStream_t st) {
    ProfScope ps(PROF_LC_MISC, st);
    hipLaunchKernelGGL(k_lc_pack, dim3(blocks_for((long)n * n * n, 256)), dim3(256), 0, st, delta, g[0], g[1], g[2],
                       row, n, in_scale[0], in_scale[1], in_scale[2], in_scale[3], x0);
    return hipGetLastError();
}

hipError_t lc_pack_delta(const float* delta, long row, int n, float s0, uint16_t* x0, hipStream_t st) {
    ProfScope ps(PROF_LC_MISC, st);
    hipLaunchKernelGGL(k_lc_pack_delta, dim3(blocks_for((long)n * n * n, 256)), dim3(256), 0, st, delta, row, n, s0,
                       x0);
    return hipGetLastError();
}

template <int C>
static hipError_t forward_c(const LcParams& P, const LcActs& A, int n, float out_scale, float band,
                            float* const out[3], long row, int accumulate, bool keep_z, hipStream_t st) {
    constexpr int NB = C / 16;
    hipError_t e = keep_z ? run_conv<8, NB, EPI_ZA>(A.x0, P.wb1, P.b1, A.z1, A.a1, nullptr, n, st)
                          : run_conv<8, NB, EPI_A>(A.x0, P.wb1, P.b1, A.a1, nullptr, nullptr, n, st);
    if (e != hipSuccess) return e;
    e = keep_z ? run_conv<C, NB, EPI_ZA>(A.a1, P.wb2, P.b2, A.z2, A.a2, nullptr, n, st)
               : run_conv<C, NB, EPI_A>(A.a1, P.wb2, P.b2, A.a2, nullptr, nullptr, n, st);
    if (e != hipSuccess) return e;
    if (band != 0.0f) {  // dF into T (dense), then the band-pass weight into `out`
        const long V = (long)n * n * n;
        {
            ProfScope ps(PROF_LC_MISC, st);
            hipLaunchKernelGGL(k_lc_out<C>, dim3(blocks_for(V, 256)), dim3(256), 0, st, A.a2, P.w3, P.b3, out_scale,
                               n, (long)n, A.t, A.t + V, A.t + 2 * V, 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        return lc_band(A.t, n, band, out, row, accumulate, st);
    }
    ProfScope ps(PROF_LC_MISC, st);
    hipLaunchKernelGGL(k_lc_out<C>, dim3(blocks_for((long)n * n * n, 256)), dim3(256), 0, st, A.a2, P.w3, P.b3,
                       out_scale, n, row, out[0], out[1], out[2], accumulate);
    return hipGetLastError();
}

template <int C>
static hipError_t forward_fields_c(const LcParams& P, uint16_t* a1, const uint16_t* d0, float* F, long row, int n,
                                   const float in_scale[4], float out_scale, float band, float* t, hipStream_t st) {
    constexpr int NB = C / 16;
    float* const g[3] = {F, F + 1, F + 2};  // the interleaved force mesh: component c at 3 z + c
    FieldSrc fs{d0, {g[0], g[1], g[2]}, row, {in_scale[1], in_scale[2], in_scale[3]}, 3};
    const bool dens_only = in_scale[1] == 0.0f && in_scale[2] == 0.0f && in_scale[3] == 0.0f;
    hipError_t e = dens_only ? run_conv_dens<NB>(d0, P.wb1, P.b1, a1, n, st)
                             : run_conv<8, NB, EPI_A, true>(nullptr, P.wb1, P.b1, a1, nullptr, nullptr, n, st, fs);
    if (e != hipSuccess) return e;
    if (band != 0.0f) {  // dF stored in t, then added to the force meshes through the band-pass weight
        const long V = (long)n * n * n;
        OutDst od{{t, t + V, t + 2 * V}, (long)n, P.w3, P.b3, out_scale};
        e = run_conv<C, NB, EPI_OUT_STORE>(a1, P.wb2, P.b2, nullptr, nullptr, nullptr, n, st, FieldSrc{}, od);
        if (e != hipSuccess) return e;
        return lc_band(t, n, band, g, row, 1, st, 3);
    }
    OutDst od{{g[0], g[1], g[2]}, row, P.w3, P.b3, out_scale, 3};
    return run_conv<C, NB, EPI_OUT>(a1, P.wb2, P.b2, nullptr, nullptr, nullptr, n, st, FieldSrc{}, od);
}

hipError_t lc_forward_fields(const LcParams& P, uint16_t* a1, const uint16_t* d0, float* F, long row, int n,
                             const float in_scale[4], float out_scale, float band, float* t, hipStream_t st) {
    if (P.C == 16) return forward_fields_c<16>(P, a1, d0, F, row, n, in_scale, out_scale, band, t, st);
    if (P.C == 32) return forward_fields_c<32>(P, a1, d0, F, row, n, in_scale, out_scale, band, t, st);
    return hipErrorInvalidValue;
}

hipError_t lc_forward(const LcParams& P, const LcActs& A, int n, float out_scale, float band, float* const out[3],
                      long row, int accumulate, bool keep_z, hipStream_t st) {
    if (P.C == 16) return forward_c<16>(P, A, n, out_scale, band, out, row, accumulate, keep_z, st);
    if (P.C == 32) return forward_c<32>(P, A, n, out_scale, band, out, row, accumulate, keep_z, st);
    return hipErrorInvalidValue;
}

template <int C>
static hipError_t backward_c(const LcParams& P, const LcActs& A, LcGrads& G, int n, float out_scale, float band,
                             const float* ddf, hipStream_t st) {
    constexpr int NB = C / 16;
    const long V = (long)n * n * n;
    if (band != 0.0f) {  // the band-pass weight is self-adjoint: upstream d_df + band B d_df
        float* t3[3] = {A.t, A.t + V, A.t + 2 * V};
        if (hipError_t e = lc_band(ddf, n, band, t3, (long)n, 0, st); e != hipSuccess) return e;
        ddf = A.t;
    }
    {
        ProfScope ps(PROF_LC_MISC, st);
        hipLaunchKernelGGL(k_lc_out_back<C>, dim3((unsigned)std::min<long>(blocks_for(V, 256), 1024)), dim3(256), 0,
                           st, ddf, A.z2, P.w3, out_scale, n, A.dz2, G.w3, G.b3);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
    if (hipError_t e = run_wgrad<C, NB>(A.dz2, A.a1, G.w2, G.b2, n, C, st); e != hipSuccess) return e;
    if (hipError_t e = run_conv<C, NB, EPI_DSILU>(A.dz2, P.wt2, nullptr, A.dz1, nullptr, A.z1, n, st); e != hipSuccess)
        return e;
    return run_wgrad<8, NB>(A.dz1, A.x0, G.w1, G.b1, n, 4, st);
}

hipError_t lc_backward(const LcParams& P, const LcActs& A, LcGrads& G, int n, float out_scale, float band,
                       const float* ddf, hipStream_t st) {
    if (P.C == 16) return backward_c<16>(P, A, G, n, out_scale, band, ddf, st);
    if (P.C == 32) return backward_c<32>(P, A, G, n, out_scale, band, ddf, st);
    return hipErrorInvalidValue;
}

hipError_t lc_loss(const float* const pos[3], long np, int n, double box, const float* const df[3],
                   const float* const g1[3], const float* const g3[3], double* stats, float* ddf,
                   hipStream_t st) {
    hipError_t e = launch_fill_d(stats, 2, 0.0, st);
    if (e != hipSuccess) return e;
    if ((e = launch_fill(ddf, 3L * n * n * n, 0.0f, st)) != hipSuccess) return e;
    ProfScope ps(PROF_LC_MISC, st);
    hipLaunchKernelGGL(k_lc_denom, dim3((unsigned)std::min<long>(blocks_for(np, 256), 1024)), dim3(256), 0, st,
                       g1[0], g1[1], g1[2], g3[0], g3[1], g3[2], np, stats);
    hipLaunchKernelGGL(k_lc_loss, dim3(blocks_for(np, 256)), dim3(256), 0, st, pos[0], pos[1], pos[2], np, n,
                       (float)(n / box), df[0], df[1], df[2], g1[0], g1[1], g1[2], g3[0], g3[1], g3[2], stats, ddf);
    return hipGetLastError();
}

hipError_t lc_adam(float* p, float* g, float* m, float* v, long np, float lr, float b1, float b2, float eps, int t,
                   hipStream_t st) {
    const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
    ProfScope ps(PROF_LC_MISC, st);
    hipLaunchKernelGGL(k_lc_adam, dim3((unsigned)std::min<long>(blocks_for(np, 256), 4096)), dim3(256), 0, st, p, g,
                       m, v, np, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t lc_positions(const float* const x[3], long n_per_real, int n_real, int n_part, double box, double qoff,
                        float* const pos[3], hipStream_t st) {
    const long total = n_per_real * n_real;
    ProfScope ps(PROF_LC_MISC, st);
    for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL(k_positions, dim3(blocks_for(total, 256)), dim3(256), 0, st, x[d], n_per_real, total,
                           n_part, d, (float)(box / n_part), (float)qoff, (float)box, pos[d]);
    return hipGetLastError();
}

hipError_t gather_absolute(const float* const pos[3], long np, int n, double box, const float* F, long row,
                           float* const out[3], hipStream_t st) {
    ProfScope ps(PROF_GATHER, st);
    hipLaunchKernelGGL(k_gather_abs, dim3(blocks_for(np, 256)), dim3(256), 0, st, pos[0], pos[1], pos[2], np, n,
                       (float)(n / box), F, row, out[0], out[1], out[2]);
    return hipGetLastError();
}

hipError_t mesh_unpad3(const float* F, long row, int n, float* const g[3], hipStream_t st) {
    ProfScope ps(PROF_COPY, st);
    hipLaunchKernelGGL(k_mesh_unpad3, dim3(blocks_for((long)n * n * n, 256)), dim3(256), 0, st, F, row, n, g[0], g[1],
                       g[2]);
    return hipGetLastError();
}

hipError_t mesh_unpad(const float* src, long row, int n, float* dst, hipStream_t st) {
    ProfScope ps(PROF_COPY, st);
    hipLaunchKernelGGL(k_mesh_unpad, dim3(blocks_for((long)n * n * n, 256)), dim3(256), 0, st, src, row, n, dst);
    return hipGetLastError();
}

}  // namespace cola
