// Compile-time FFT plans for 512^3 meshes: y rows and x columns of length 512, z passes of length
// 256 (the half-length complex transform of the real rows).  Shapes offered to the autotuner beside
// the dynamic kernels of the same shape.

#include "fft_kernels.h"

namespace cola {

hipError_t fft_static_512(const FftLaunch& L) {
    if (is_z_op(L.op)) {
        if (L.n != 256) return hipErrorNotSupported;
        if (L.R == 16) return static_z_ops<256, 16>(L);
        if (L.R == 8) return static_z_ops<256, 8>(L);
        return hipErrorNotSupported;
    }
    if (L.n != 512) return hipErrorNotSupported;
    if (is_rows_op(L.op)) {
        if (L.R == 16) return static_rows_ops<512, 16>(L);
        if (L.R == 8) return static_rows_ops<512, 8>(L);
        return hipErrorNotSupported;
    }
    if (L.split) return hipErrorNotSupported;
    if (L.R == 16 && L.width == 8) return static_cols_ops<512, 16, 8>(L);
    if (L.R == 16 && L.width == 16) return static_cols_ops<512, 16, 16>(L);
    if (L.R == 8 && L.width == 8) return static_cols_ops<512, 8, 8>(L);
    return hipErrorNotSupported;
}

}  // namespace cola
