// Compile-time FFT plans for 1536^3 meshes: y rows and x columns of length 1536, z passes of length
// 768 (the half-length complex transform of the real rows).  Shapes offered to the autotuner beside
// the dynamic kernels of the same shape.

#include "fft_kernels.h"

namespace cola {

hipError_t fft_static_1536(const FftLaunch& L) {
    if (is_z_op(L.op)) {
        if (L.n != 768) return hipErrorNotSupported;
        if (L.R == 24) return static_z_ops<768, 24>(L);
        if (L.R == 12) return static_z_ops<768, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.n != 1536) return hipErrorNotSupported;
    if (is_rows_op(L.op)) {
        if (L.R == 24) return static_rows_ops<1536, 24>(L);
        if (L.R == 12) return static_rows_ops<1536, 12>(L);
        return hipErrorNotSupported;
    }
    if (L.split) {
        if (L.R == 24 && L.width == 8) return static_cols_ops<1536, 24, 8, true>(L);
        if (L.R == 12 && L.width == 8) return static_cols_ops<1536, 12, 8, true>(L);  // 1024 threads
        return hipErrorNotSupported;
    }
    if (L.R == 24 && L.width == 8) return static_cols_ops<1536, 24, 8>(L);
    if (L.R == 24 && L.width == 4) return static_cols_ops<1536, 24, 4>(L);
    if (L.R == 12 && L.width == 4) return static_cols_ops<1536, 12, 4>(L);
    return hipErrorNotSupported;
}

}  // namespace cola
