// CIC interpolation of the interleaved force mesh at one particle (Sec. 2.2: the mesh force is
// interpolated back to the particles with the same cloud-in-cell weights as the deposit).
#pragma once

#include <hip/hip_runtime.h>

namespace cola {

// F: rows of `row` floats, cell z of row (x, y) at F[(x n + y) row + 3 z .. + 2] = (F_x, F_y, F_z),
// with the ghost cells z = n, n + 1 repeating z = 0, 1 -- so the pair of z corners (m, m + 1) is 24
// contiguous bytes that never wrap.  (mx, my, mz): the lower corner; (ux, uy, uz): the fractional
// offsets from it.  The four corner columns are requested before any arithmetic.
__device__ __forceinline__ void gather_interleaved(const float* F, long row, int n, int mx, int my, int mz, float ux,
                                                   float uy, float uz, float g[3]) {
    const int xs[2] = {mx, mx + 1 == n ? 0 : mx + 1}, ys[2] = {my, my + 1 == n ? 0 : my + 1};
    const float wx[2] = {1.0f - ux, ux}, wy[2] = {1.0f - uy, uy}, wz[2] = {1.0f - uz, uz};
    float v[4][6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            __builtin_memcpy(v[2 * a + b], F + ((long)xs[a] * n + ys[b]) * row + 3L * mz, 6 * sizeof(float));
    g[0] = g[1] = g[2] = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float wab = wx[a] * wy[b];
            const float w0 = wab * wz[0], w1 = wab * wz[1];
#pragma unroll
            for (int c = 0; c < 3; ++c) g[c] += w0 * v[2 * a + b][c] + w1 * v[2 * a + b][3 + c];
        }
}

}  // namespace cola
