"""The x-column FFT plans whose LDS exchanges move the real and then the imaginary parts (half the
LDS of a float2 exchange), against closed forms on 768^3 and 1536^3 meshes (768 with R = 12 and
16-column tiles, and 1536 with R = 12 and 8-column tiles, run 1024-thread blocks).

A plane wave delta = cos(2 pi m / n), m = (a i + b j + c l) mod n, has the force
g_d = -(k_d / k^2) sin(2 pi m / n); the unnormalised inverse transform of a half spectrum with a
single entry 1 at (a, b, c), 0 < c < n/2, is 2 cos(2 pi m / n); the forward transform of the plane
wave is n^3 / 2 at (a, b, c) and 0 elsewhere.  The x-column passes (x_green in the force, x_mult in
the c2r, cols_x in the r2c) are pinned to the split plans; the other passes keep their shapes.
Checked at 40 000 sampled cells in float64 (error <= 2e-5 of the amplitude) and over the whole mesh
in float32 slabs (error <= 1e-4 of the amplitude).
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

A, B, C = 3, 301, 11  # mode integers: none on a Nyquist plane, all three axes present


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04685_amd as c
    return c


def phase_slab(n, x0, x1):
    i = torch.arange(x0, x1, device="cuda", dtype=torch.int32)
    j = torch.arange(n, device="cuda", dtype=torch.int32)
    m = ((A * i[:, None, None]) % n + (B * j[None, :, None]) % n) % n
    m = (m + (C * j[None, None, :]) % n) % n
    return m.float() * (2.0 * np.pi / n)


def plane_wave(n):
    x = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    for x0 in range(0, n, 128):
        x[x0:x0 + 128] = torch.cos(phase_slab(n, x0, x0 + 128))
    return x


def check_field(n, field, want_fn, amp, label):
    rng = np.random.default_rng(5)
    idx = rng.integers(0, n, size=(3, 40_000))
    ph = 2.0 * np.pi * ((A * idx[0] + B * idx[1] + C * idx[2]) % n) / n
    it = torch.as_tensor(idx, device="cuda")
    got = field[it[0], it[1], it[2]].double().cpu().numpy()
    err = np.abs(got - want_fn(ph)).max() / amp
    worst = 0.0
    for x0 in range(0, n, 128):
        ref = want_fn(phase_slab(n, x0, x0 + 128))
        worst = max(worst, float((field[x0:x0 + 128] - ref).abs().max()) / amp)
        del ref
    say(f"  {label}: sampled {err:.2e}, whole mesh {worst:.2e} of the amplitude")
    assert err < 2e-5, label
    assert worst < 1e-4, label


@pytest.mark.parametrize("n,R,width", [(768, 24, 16), (768, 24, 8), (768, 12, 16), (1536, 24, 8), (1536, 12, 8)])
def test_split_exchange_plans(cola, n, R, width):
    if n == 1536 and torch.cuda.get_device_properties(0).total_memory < 200 * 2 ** 30:
        pytest.skip("needs about 130 GB of device memory")
    say(f"split exchange: n={n}, x columns R={R} x {width}")
    for kind in ("cols_x", "x_green", "x_mult"):
        cola.fft_set_shape(n, kind, R, width, split=True)
    # force
    delta = plane_wave(n)
    g = cola.mesh_force(delta, float(n))
    del delta
    torch.cuda.empty_cache()
    kf = 2.0 * np.pi / n
    k = np.array([A, B, C], dtype=np.float64) * kf
    k2 = float((k ** 2).sum())
    amp = float(np.abs(k).max() / k2)
    for d in range(3):
        coef = -k[d] / k2

        def want(ph, coef=coef):
            return coef * (np.sin(ph) if isinstance(ph, np.ndarray) else torch.sin(ph))
        check_field(n, g[d], want, amp, f"g_{'xyz'[d]}")
    del g
    torch.cuda.empty_cache()
    # c2r
    spec = torch.zeros((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    spec[A, B, C] = 1.0
    out = cola.fft_c2r(spec)
    del spec
    torch.cuda.empty_cache()

    def want2(ph):
        return 2.0 * (np.cos(ph) if isinstance(ph, np.ndarray) else torch.cos(ph))
    check_field(n, out, want2, 2.0, "c2r")
    del out
    torch.cuda.empty_cache()
    # r2c
    x = plane_wave(n)
    out = cola.fft_r2c(x)
    del x
    torch.cuda.empty_cache()
    peak = complex(out[A, B, C].item())
    amp = 0.5 * float(n) ** 3
    assert abs(peak.real - amp) < 1e-5 * amp and abs(peak.imag) < 1e-5 * amp
    out[A, B, C] = 0
    rest = float(out.abs().max().cpu())
    say(f"  r2c: peak {peak.real:.6e} (expected {amp:.6e}), largest other mode {rest:.2e}")
    assert rest < 1e-4 * amp
    del out
    torch.cuda.empty_cache()


def test_split_shape_rejected_where_absent(cola):
    """Split plans exist for x-column kinds only and only where compiled."""
    with pytest.raises(Exception):
        cola.fft_set_shape(768, "rows_y", 24, 8, split=True)
    with pytest.raises(Exception):
        cola.fft_set_shape(512, "x_green", 16, 8, split=True)
