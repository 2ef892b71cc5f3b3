// Compile-time FFT plans for 768^3 meshes: y rows and x columns of length 768, z passes of length
// 384 (the half-length complex transform of the real rows).  Shapes offered to the autotuner beside
// the dynamic kernels of the same shape.

#include "fft_kernels.h"

namespace cola {

hipError_t fft_static_768(const FftLaunch& L) {
    if (is_z_op(L.op)) {
        if (L.n != 384) return hipErrorNotSupported;
        if (L.R == 24) return static_z_ops<384, 24>(L);
        if (L.R == 12) return static_z_ops<384, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.n != 768) return hipErrorNotSupported;
    if (is_rows_op(L.op)) {
        if (L.R == 24) return static_rows_ops<768, 24>(L);
        if (L.R == 12) return static_rows_ops<768, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.split) {
        if (L.R == 24 && L.width == 16) return static_cols_ops<768, 24, 16, true>(L);
        if (L.R == 24 && L.width == 8) return static_cols_ops<768, 24, 8, true>(L);
        // 16-column tiles (whole 128-byte rows) in 1024-thread blocks of 49 KB: two per CU
        if (L.R == 12 && L.width == 16) return static_cols_ops<768, 12, 16, true>(L);
        return hipErrorNotSupported;
    }
    if (L.R == 24 && L.width == 8) return static_cols_ops<768, 24, 8>(L);
    if (L.R == 24 && L.width == 16) return static_cols_ops<768, 24, 16>(L);
    if (L.R == 12 && L.width == 8) return static_cols_ops<768, 12, 8>(L);
    return hipErrorNotSupported;
}

}  // namespace cola
