// Internal declarations of the learned coarse-mesh force correction (lc_kernels.hip, lc_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/cola.h"

namespace cola {

// FP32 master parameters, flat: w1 (C,4,27) b1 (C) w2 (C,C,27) b2 (C) w3 (3,C) b3 (3).
struct LcOffsets {
    long w1, b1, w2, b2, w3, b3, total;
};
inline LcOffsets lc_offsets(int C) {
    LcOffsets o;
    o.w1 = 0;
    o.b1 = o.w1 + 108L * C;
    o.w2 = o.b1 + C;
    o.b2 = o.w2 + 27L * C * C;
    o.w3 = o.b2 + C;
    o.b3 = o.w3 + 3L * C;
    o.total = o.b3 + 3;
    return o;
}

// BF16 copies of the conv weights: wb1 [C][27][8] (input channels padded 4 -> 8),
// wb2 [C][27][C], wt2 [C][27][C] (mirrored taps, swapped channels: data gradient of layer 2).
struct LcPackedOffsets {
    size_t wb1, wb2, wt2, total;  // bytes
};
inline size_t lc_align(size_t x) { return (x + 255) / 256 * 256; }
inline LcPackedOffsets lc_packed_offsets(int C) {
    LcPackedOffsets o;
    o.wb1 = 0;
    o.wb2 = lc_align((size_t)C * 27 * 8 * 2);
    o.wt2 = o.wb2 + lc_align((size_t)C * 27 * C * 2);
    o.total = o.wt2 + lc_align((size_t)C * 27 * C * 2);
    return o;
}

struct LcParams {
    int C;
    const float *w1, *b1, *w2, *b2, *w3, *b3;  // FP32 (device)
    const uint16_t *wb1, *wb2, *wt2;           // BF16 (device)
};
struct LcGrads {
    float *w1, *b1, *w2, *b2, *w3, *b3;
};
// BF16 activations, channel-last: x0 [V][8]; the others [V][C].  z1, z2, dz1, dz2 only when training.
struct LcActs {
    uint16_t *x0, *z1, *a1, *z2, *a2, *dz1, *dz2;
    float* t;  // [3][V] FP32 scratch of the band-pass output weight
};

hipError_t lc_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D, hipStream_t st);
hipError_t lc_pack_weights(const float* w1, const float* w2, int C, uint16_t* wb1, uint16_t* wb2, uint16_t* wt2,
                           hipStream_t st);
// X0 = (delta, g) * in_scale from meshes with `row` floats per (x, y) row.
hipError_t lc_pack(const float* delta, const float* const g[3], long row, int n, const float in_scale[4],
                   uint16_t* x0, hipStream_t st);
// The step's input path: delta * s0 saved as compact BF16 (d0, n^3 values) before the transform
// overwrites the density; later the network reads d0 and the force mesh directly and adds dF to
// it.  F: the step's interleaved force mesh (component c of cell z of a row at 3 z + c, `row`
// floats per row); a1: [n^3][C] BF16 scratch.
hipError_t lc_pack_delta(const float* delta, long row, int n, float s0, uint16_t* d0, hipStream_t st);
// band != 0: dF goes through t ([3][n^3] scratch) and the band-pass weight (lc_band).
hipError_t lc_forward_fields(const LcParams& P, uint16_t* a1, const uint16_t* d0, float* F, long row, int n,
                             const float in_scale[4], float out_scale, float band, float* t, hipStream_t st);
// dF (times out_scale, then through the band-pass weight) written to, or added into, three meshes
// with `row` floats per row.  keep_z stores z1, z2 for the backward pass.
hipError_t lc_forward(const LcParams& P, const LcActs& A, int n, float out_scale, float band, float* const out[3],
                      long row, int accumulate, bool keep_z, hipStream_t st);
// Accumulates the parameter gradients for upstream d_df (dense [3][n^3]).
hipError_t lc_backward(const LcParams& P, const LcActs& A, LcGrads& G, int n, float out_scale, float band,
                       const float* ddf, hipStream_t st);
// out[c] (+)= T[c] + beta (K T[c] - K K T[c]), K the periodic [1, 2, 1] / 4 smoothing per axis;
// T dense [3][n^3] (n a multiple of 16), out with `row` floats per row and cell z of a row at zs z;
// T and out must not overlap.
hipError_t lc_band(const float* T, int n, float beta, float* const out[3], long row, int accumulate,
                   hipStream_t st, int zs = 1);
// Particle loss (stats[0] = L, stats[1] = denominator; zeroed here) and d_df = dL/d(dF) (overwritten).
hipError_t lc_loss(const float* const pos[3], long np, int n, double box, const float* const df[3],
                   const float* const g1[3], const float* const g3[3], double* stats, float* ddf,
                   hipStream_t st);
hipError_t lc_adam(float* p, float* g, float* m, float* v, long np, float lr, float b1, float b2, float eps, int t,
                   hipStream_t st);
// Absolute positions q + x wrapped into [0, box) (lattice as in the step).
hipError_t lc_positions(const float* const x[3], long n_per_real, int n_real, int n_part, double box, double qoff,
                        float* const pos[3], hipStream_t st);
// CIC interpolation of the interleaved force mesh F (pm_force_interleaved: `row` floats per row,
// ghost cells included) to absolute positions.
hipError_t gather_absolute(const float* const pos[3], long np, int n, double box, const float* F, long row,
                           float* const out[3], hipStream_t st);
// Copy of a mesh with `row` floats per row into a dense n^3 array.
hipError_t mesh_unpad(const float* src, long row, int n, float* dst, hipStream_t st);
// The three components of the interleaved force mesh F into dense n^3 arrays g[0..2].
hipError_t mesh_unpad3(const float* F, long row, int n, float* const g[3], hipStream_t st);

// Workspace of the network (lc_api.cpp): x0 for n_real realizations, a1 and a2 shared, and when
// training z1, z2, dz1, dz2.
struct LcWsLayout {
    size_t x0 = 0, a1 = 0, a2 = 0, t = 0, z1 = 0, z2 = 0, dz1 = 0, dz2 = 0, total = 0;
    long x0_stride = 0;  // uint16 per realization (x0 holds n_real compact deltas in the step)
};
LcWsLayout lc_ws_layout(int n, int C, int n_real, bool training);
LcActs lc_carve(void* ws, const LcWsLayout& L);
// COLA_OK or the status for an unusable network description.
int lc_check_net(const cola_lc_net* net, bool training);
LcParams lc_params_of(const cola_lc_net* net);
bool lc_mesh_ok(int n);

}  // namespace cola
