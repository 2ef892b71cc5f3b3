// Compile-time FFT plans for 288^3 meshes: y rows and x columns of length 288, z passes of length
// 144 (the half-length complex transform of the real rows).  Shapes offered to the autotuner beside
// the dynamic kernels of the same shape.

#include "fft_kernels.h"

namespace cola {

hipError_t fft_static_288(const FftLaunch& L) {
    if (is_z_op(L.op)) {
        if (L.n != 144) return hipErrorNotSupported;
        if (L.R == 24) return static_z_ops<144, 24>(L);
        if (L.R == 12) return static_z_ops<144, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.n != 288) return hipErrorNotSupported;
    if (is_rows_op(L.op)) {
        if (L.R == 24) return static_rows_ops<288, 24>(L);
        if (L.R == 12) return static_rows_ops<288, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.split) return hipErrorNotSupported;
    if (L.R == 24 && L.width == 8) return static_cols_ops<288, 24, 8>(L);
    if (L.R == 24 && L.width == 16) return static_cols_ops<288, 24, 16>(L);
    if (L.R == 12 && L.width == 8) return static_cols_ops<288, 12, 8>(L);
    if (L.R == 12 && L.width == 16) return static_cols_ops<288, 12, 16>(L);
    return hipErrorNotSupported;
}

}  // namespace cola
