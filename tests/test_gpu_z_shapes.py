"""Every admissible kernel shape of the two plain z passes against numpy's float64 FFTs.

The z r2c pass transforms real rows of n values into n/2 + 1 complex ones (through an n/2-point
complex transform) and writes them transposed into the half spectrum [k_z][x][y]; the z c2r pass
reads that layout back.  A block holds W lines in LDS, n/2 + 2 complex values apart, and reads or
writes them transposed (line j, plane k at j (n/2 + 2) + k).  Each admissible shape (values per
thread R, lines per block W, compile-time or run-time plan) is pinned in turn for both passes and
the 3D r2c and c2r compared with numpy on one seeded field: relative RMS <= 2e-6 log2(n) and max
error <= 2e-5 of the largest value, as the other FFT tests.  n = 72 has run-time plans only,
n = 288 compile-time ones too (R = 12, 24).  A shape that the host rejects (R not a plan of n/2,
W not a power of two dividing n, too many threads or too much LDS) is skipped, and each size must
still cover at least eight shapes, both plan kinds included where they exist.
"""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1509_04685_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04685_amd as c
    return c


@pytest.mark.parametrize("n", [72, 288])
def test_z_pass_every_shape(cola, n):
    x = W.random_field(n, seed=4100 + n, dtype=np.float32)
    xk = np.fft.rfftn(x.astype(np.float64))
    x_dev = torch.as_tensor(x, device="cuda")
    xk_dev = torch.as_tensor(xk, device="cuda")  # complex128
    xk32 = xk_dev.to(torch.complex64)
    want_back = x_dev.double() * float(n) ** 3
    tol = 2e-6 * math.log2(n)
    kmax = float(xk_dev.abs().max())
    ran = []
    for stat in (False, True):
        for R in (2, 3, 4, 6, 8, 12, 16, 24):
            for width in (1, 2, 4, 8, 16, 32, 64):
                try:
                    cola.fft_set_shape(n, "z_r2c", R, width, use_static=stat)
                    cola.fft_set_shape(n, "z_c2r", R, width, use_static=stat)
                except cola.ColaError:
                    continue
                say(f"z passes {n}^3: R={R} width={width} static={stat}")
                got = cola.fft_r2c(x_dev).to(torch.complex128)
                err = (got - xk_dev).abs()
                rel = float(torch.sqrt((err ** 2).mean() / (xk_dev.abs() ** 2).mean()))
                assert rel < tol, ("r2c", R, width, stat, rel)
                assert float(err.max()) < 2e-5 * kmax, ("r2c", R, width, stat)
                back = cola.fft_c2r(xk32).double()
                rel_b = float(torch.sqrt(((back - want_back) ** 2).mean() / (want_back ** 2).mean()))
                assert rel_b < tol, ("c2r", R, width, stat, rel_b)
                ran.append((R, width, stat))
    say(f"z passes {n}^3: {len(ran)} shapes")
    assert len(ran) >= 8
    if n == 288:
        assert any(s for _, _, s in ran) and any(not s for _, _, s in ran)
