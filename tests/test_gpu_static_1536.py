"""Every FFT pass of the 1536^3 mesh (the 512^3-particle workload) against closed forms.

A plane wave delta = cos(2 pi m / n), m = (a i + b j + c l) mod n, has the force
g_d = -(k_d / k^2) sin(2 pi m / n) (g_k = i k delta_k / k^2 for both of its modes), and the
unnormalised inverse transform of a half spectrum with a single entry 1 at (a, b, c), 0 < c < n/2,
is 2 cos(2 pi m / n).  The phase index m is formed exactly in integers, so the references are exact
up to float64 rounding.

Each compile-time plan of fft_static_1536.hip is pinned in turn (values per thread and tile
width), and once more the shapes the autotuner picks (the launch configuration of the bench):
  * force (cola_mesh_force, the step's force passes): z r2c, y forward rows, fused x
    Green/gradient, y split, y inverse rows, and the one z c2r pass that writes the three
    components interleaved (i k_z for F_z), then copied out per component;
  * c2r: x inverse with multiplier, y inverse rows, z c2r;
  * r2c: z r2c, y forward rows, x forward columns.
Checked at 40 000 sampled cells in float64 on the host (error <= 2e-5 of the amplitude), and over
the whole mesh on the device in float32 slabs (error <= 1e-4 of the amplitude).
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

N = 1536
A, B, C = 3, 700, 11  # mode integers: none on a Nyquist plane, all three axes present


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if torch.cuda.get_device_properties(0).total_memory < 200 * 2 ** 30:
        pytest.skip("needs about 150 GB of device memory")
    import paper_1509_04685_amd as c
    return c


def phase_slab(x0, x1):
    """2 pi m / n on planes x0..x1-1 (float32 device tensor), m formed exactly in int32."""
    i = torch.arange(x0, x1, device="cuda", dtype=torch.int32)
    j = torch.arange(N, device="cuda", dtype=torch.int32)
    m = ((A * i[:, None, None]) % N + (B * j[None, :, None]) % N) % N
    m = (m + (C * j[None, None, :]) % N) % N
    return m.float() * (2.0 * np.pi / N)


def plane_wave():
    x = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
    for x0 in range(0, N, 128):
        x[x0:x0 + 128] = torch.cos(phase_slab(x0, x0 + 128))
    return x


def samples(seed=5, k=40_000):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, N, size=(3, k))
    m = (A * idx[0] + B * idx[1] + C * idx[2]) % N
    return idx, 2.0 * np.pi * m / N


def check_field(field, want_fn, amp, label):
    """field: (N, N, N) device tensor; want_fn(phase) -> expected values (numpy or torch)."""
    idx, ph = samples()
    it = torch.as_tensor(idx, device="cuda")
    got = field[it[0], it[1], it[2]].double().cpu().numpy()
    err = np.abs(got - want_fn(ph)).max() / amp
    worst = 0.0
    for x0 in range(0, N, 128):
        ref = want_fn(phase_slab(x0, x0 + 128))
        worst = max(worst, float((field[x0:x0 + 128] - ref).abs().max()) / amp)
        del ref
    say(f"  {label}: sampled {err:.2e}, whole mesh {worst:.2e} of the amplitude")
    assert err < 2e-5, label
    assert worst < 1e-4, label


def run_force(cola, tag):
    say(f"force {tag}")
    delta = plane_wave()
    box = 1536.0
    g = cola.mesh_force(delta, box)
    del delta
    torch.cuda.empty_cache()
    kf = 2.0 * np.pi / box
    k = np.array([A, B, C], dtype=np.float64) * kf
    k2 = float((k ** 2).sum())
    amp = float(np.abs(k).max() / k2)
    for d in range(3):
        coef = -k[d] / k2

        def want(ph, coef=coef):
            return coef * (np.sin(ph) if isinstance(ph, np.ndarray) else torch.sin(ph))
        check_field(g[d], want, amp, f"g_{'xyz'[d]}")
    del g
    torch.cuda.empty_cache()


def run_c2r(cola, tag):
    say(f"c2r {tag}")
    spec = torch.zeros((N, N, N // 2 + 1), dtype=torch.complex64, device="cuda")
    spec[A, B, C] = 1.0
    out = cola.fft_c2r(spec)
    del spec
    torch.cuda.empty_cache()

    def want(ph):
        return 2.0 * (np.cos(ph) if isinstance(ph, np.ndarray) else torch.cos(ph))
    check_field(out, want, 2.0, "c2r")
    del out
    torch.cuda.empty_cache()


def run_r2c(cola, tag):
    say(f"r2c {tag}")
    x = plane_wave()
    out = cola.fft_r2c(x)
    del x
    torch.cuda.empty_cache()
    amp = 0.5 * float(N) ** 3
    peak = complex(out[A, B, C].item())
    assert abs(peak.real - amp) < 1e-5 * amp and abs(peak.imag) < 1e-5 * amp
    out[A, B, C] = 0
    rest = float(out.abs().max().cpu())
    say(f"  r2c: peak {peak.real:.6e} (expected {amp:.6e}), largest other mode {rest:.2e}")
    assert rest < 1e-4 * amp
    del out
    torch.cuda.empty_cache()


# (z-pass values per thread, y-row values per thread, x-column values per thread, column tile
# width): the compile-time plans of fft_static_1536.hip
STATIC = [(24, 24, 24, 8), (12, 12, 24, 4), (24, 12, 12, 4)]


@pytest.mark.parametrize("rz,rr,rc,w", STATIC)
def test_static_plans_1536(cola, rz, rr, rc, w):
    zw = 256 // (768 // rz)  # lines per block of the z passes and y rows: 256 threads
    rw = 256 // (1536 // rr)
    for kind in ("z_r2c", "z_c2r", "z_c2r3"):  # z_c2r3: three groups of zw lines, 768 threads
        cola.fft_set_shape(N, kind, rz, zw, True)
    for kind in ("rows_y", "y_split"):
        cola.fft_set_shape(N, kind, rr, rw, True)
    for kind in ("cols_x", "x_green", "x_mult"):
        cola.fft_set_shape(N, kind, rc, w, True)
    tag = f"static z R={rz}, y rows R={rr}, x columns R={rc} x {w}"
    run_force(cola, tag)
    run_c2r(cola, tag)
    run_r2c(cola, tag)


def test_autotuned_shapes_1536(cola):
    """The shapes the bench runs with: autotuned on the 512^3 / 1536^3 workload's workspace."""
    prob = cola.make_problem(1536.0, 512, 3, 19.0, 40)
    ws = cola.Workspace(prob)
    report = cola.autotune(prob, ws)
    del ws
    torch.cuda.empty_cache()
    say(report)
    run_force(cola, "autotuned")
    run_c2r(cola, "autotuned")
