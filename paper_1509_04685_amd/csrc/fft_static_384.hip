// Compile-time FFT plans for 384^3 meshes: y rows and x columns of length 384, z passes of length
// 192 (the half-length complex transform of the real rows).  Shapes offered to the autotuner beside
// the dynamic kernels of the same shape.

#include "fft_kernels.h"

namespace cola {

hipError_t fft_static_384(const FftLaunch& L) {
    if (is_z_op(L.op)) {
        if (L.n != 192) return hipErrorNotSupported;
        if (L.R == 24) return static_z_ops<192, 24>(L);
        if (L.R == 12) return static_z_ops<192, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.n != 384) return hipErrorNotSupported;
    if (is_rows_op(L.op)) {
        if (L.R == 24) return static_rows_ops<384, 24>(L);
        if (L.R == 12) return static_rows_ops<384, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.split) return hipErrorNotSupported;
    if (L.R == 24 && L.width == 8) return static_cols_ops<384, 24, 8>(L);
    if (L.R == 24 && L.width == 16) return static_cols_ops<384, 24, 16>(L);
    if (L.R == 12 && L.width == 8) return static_cols_ops<384, 12, 8>(L);
    if (L.R == 12 && L.width == 16) return static_cols_ops<384, 12, 16>(L);
    return hipErrorNotSupported;
}

}  // namespace cola
