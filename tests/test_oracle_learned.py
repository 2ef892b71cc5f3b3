"""Pins of the float64 learned-correction reference: convolution against a brute-force loop and
a shifted-delta kernel, and every gradient against central finite differences (rel <= 1e-8)."""

import numpy as np
import pytest

from oracle import learned as L


def brute_conv3(w, b, x):
    o, i = w.shape[:2]
    n = x.shape[1]
    out = np.zeros((o, n, n, n))
    for p in np.ndindex(n, n, n):
        for t, (dx, dy, dz) in enumerate(L.TAPS):
            q = ((p[0] + dx) % n, (p[1] + dy) % n, (p[2] + dz) % n)
            out[(slice(None),) + p] += w[:, :, t] @ x[(slice(None),) + q]
    return out + b[:, None, None, None]


def test_conv3_matches_brute_force():
    rng = np.random.default_rng(1)
    w = rng.normal(size=(3, 2, 27))
    b = rng.normal(size=3)
    x = rng.normal(size=(2, 4, 4, 4))
    assert np.allclose(L.conv3(w, b, x), brute_conv3(w, b, x), atol=1e-12)


def test_conv3_delta_kernel_is_a_shift():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 5, 5, 5))
    w = np.zeros((1, 1, 27))
    t = L.TAPS.index((1, 0, -1))
    w[0, 0, t] = 1.0
    out = L.conv3(w, np.zeros(1), x)
    # out[p] = x[p + (1, 0, -1)]
    assert np.allclose(out[0], np.roll(x[0], shift=(-1, 0, 1), axis=(0, 1, 2)))


def test_silu_grad():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    assert np.allclose(L.silu_grad(z), (L.silu(z + h) - L.silu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def _setup(n=4, c=3, seed=3):
    rng = np.random.default_rng(seed)
    net = L.Net(channels=c, seed=seed, in_scale=(0.5, 2.0, 2.0, 2.0), out_scale=0.7)
    net.w3 *= 10.0
    delta = rng.normal(size=(n, n, n))
    g = rng.normal(size=(3, n, n, n))
    box = 10.0
    pos = rng.uniform(0, box, size=(3, 40))
    g1 = rng.normal(size=(3, 40))
    g3 = g1 + rng.normal(size=(3, 40))
    return net, delta, g, box, pos, g1, g3


def _loss(net, delta, g, box, pos, g1, g3):
    df, _ = L.forward(net, delta, g)
    return L.particle_loss(df, pos, box, g1, g3)[0]


@pytest.mark.parametrize("band", [0.0, 0.8])
def test_gradients_match_finite_differences(band):
    net, delta, g, box, pos, g1, g3 = _setup()
    net.band = band
    df, cache = L.forward(net, delta, g)
    _, d_df = L.particle_loss(df, pos, box, g1, g3)
    grads = L.backward(net, cache, d_df)
    rng = np.random.default_rng(7)
    h = 1e-6
    for p, gr in zip(net.params(), grads):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            old = p[idx]
            p[idx] = old + h
            lp = _loss(net, delta, g, box, pos, g1, g3)
            p[idx] = old - h
            lm = _loss(net, delta, g, box, pos, g1, g3)
            p[idx] = old
            fd = (lp - lm) / (2 * h)
            assert fd == pytest.approx(gr[idx], rel=1e-6, abs=1e-9), (p.shape, idx)


def test_band_pass_on_plane_waves_and_constants():
    n = 12
    idx = np.indices((n, n, n))
    for m in ((0, 0, 1), (1, 2, 3), (6, 0, 0), (3, 3, 3), (5, 1, 4)):
        phase = 2 * np.pi * (m[0] * idx[0] + m[1] * idx[1] + m[2] * idx[2]) / n
        x = np.cos(phase + 0.3)
        c = np.prod([np.cos(np.pi * md / n) ** 2 for md in m])
        assert np.allclose(L.binomial_smooth(x), c * x, atol=1e-12)
        assert np.allclose(L.band_pass(x), c * (1 - c) * x, atol=1e-12)
    assert np.allclose(L.band_pass(np.full((2, n, n, n), 3.7)), 0.0, atol=1e-12)
    # self-adjoint: <B x, y> = <x, B y>
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=(n, n, n)), rng.normal(size=(n, n, n))
    assert abs(np.sum(L.band_pass(a) * b) - np.sum(a * L.band_pass(b))) < 1e-10


def test_loss_is_one_without_correction():
    net, delta, g, box, pos, g1, g3 = _setup()
    zero = np.zeros((3,) + delta.shape)
    assert L.particle_loss(zero, pos, box, g1, g3)[0] == pytest.approx(1.0)


def test_adam_first_step_moves_by_lr_times_sign():
    # From m = v = 0 the bias corrections give m_hat = g and v_hat = g^2 exactly, so the first
    # update is -lr g / (|g| + eps): a step of lr against the sign of each gradient.
    rng = np.random.default_rng(11)
    p = rng.normal(size=50)
    g = rng.normal(size=50) * 10.0 ** rng.uniform(-3, 3, size=50)
    lr, eps = 1e-2, 1e-15
    p1, m, v = L.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    assert np.allclose(p1 - p, -lr * np.sign(g), rtol=1e-7, atol=0)


def test_adam_constant_gradient_keeps_unit_steps():
    # With the same gradient at every step, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    # bias-corrected ratio is g / |g| at every t.
    rng = np.random.default_rng(12)
    p = rng.normal(size=20)
    g = rng.normal(size=20)
    m = np.zeros(20)
    v = np.zeros(20)
    lr = 3e-3
    for t in range(1, 30):
        p_new, m, v = L.adam_step(p, g, m, v, t, lr, eps=1e-14)
        assert np.allclose(p_new - p, -lr * np.sign(g), rtol=1e-8, atol=0), t
        p = p_new


def test_corrected_accel_reduces_to_pm_force():
    from oracle import pm
    rng = np.random.default_rng(13)
    n, box = 8, 20.0
    pos = rng.uniform(0, box, size=(3, 300))
    net = L.Net(channels=4, seed=5, out_scale=0.5)
    net.w3[:] = 0.0
    base = pm.pm_accel(pos, n, box)
    assert np.allclose(L.corrected_accel(net, pos, n, box), base, rtol=0, atol=1e-12)
    # a constant output (bias only) shifts every particle's force by bias * out_scale, since the
    # CIC weights of each particle sum to one
    net.b3[:] = [1.0, -2.0, 0.25]
    shifted = L.corrected_accel(net, pos, n, box)
    assert np.allclose(shifted - base, (net.b3 * 0.5)[:, None], rtol=0, atol=1e-12)


def test_flat_params_roundtrip_and_order():
    net = L.Net(channels=4, seed=6)
    flat = L.flat_params(net)
    c = 4
    assert flat.size == 27 * c * c + 113 * c + 3
    assert np.array_equal(flat[:108 * c], net.w1.ravel())
    assert np.array_equal(flat[-3:], net.b3)
    other = L.Net(channels=4, seed=7)
    L.set_flat_params(other, flat)
    for a, b in zip(net.params(), other.params()):
        assert np.array_equal(a, b)


def test_green_transfer_values_and_reductions():
    """T(u), u = |m| / (n/2): the cubic Hermite interpolant with slopes 0, centred, one-sided, worked
    by hand on knots (0, 1), (0.5, 2), (1, 0): slopes m = (0, -1, -4); at the midpoint of a piece
    T = (t_j + t_j+1) / 2 + h (m_j - m_j+1) / 8, at s = 3/4 of the first piece
    T = h00 t0 + h01 t1 + h h11 m1 with h00 = 5/32, h01 = 27/32, h11 = -9/64; constant beyond the
    end knots.  T = 1 gives the plain corrected force and a constant T = c scales the mesh force by
    c (network output switched off)."""
    n = 16
    T = L.green_transfer(n, [0.0, 0.5, 1.0], [1.0, 2.0, 0.0])
    assert T[0, 0, 0] == 1.0
    assert T[0, 4, 0] == pytest.approx(2.0)                               # u = 1/2, a knot
    assert T[0, 2, 0] == pytest.approx(1.5 + 0.5 * (0.0 + 1.0) / 8)        # u = 1/4, midpoint
    assert T[0, 0, 6] == pytest.approx(1.0 + 0.5 * (-1.0 + 4.0) / 8)       # u = 3/4, midpoint
    assert T[3, 0, 0] == pytest.approx(5 / 32 + 27 / 32 * 2.0 + 0.5 * (-9 / 64) * (-1.0))  # u = 3/8
    assert T[8, 8, 8] == 0.0                                               # u = sqrt(3): beyond
    assert T[n - 3, 0, 0] == T[3, 0, 0]                                    # m = -3
    rng = np.random.default_rng(17)
    box = 20.0
    pos = rng.uniform(0, box, size=(3, 400))
    net = L.Net(channels=4, seed=5, out_scale=0.5)
    base = L.corrected_accel(net, pos, n, box)
    same = L.corrected_accel(net, pos, n, box, transfer=([0.0, 1.0], [1.0, 1.0]))
    assert np.allclose(same, base, rtol=0, atol=1e-12)
    net.w3[:] = 0.0
    net.b3[:] = 0.0
    plain = L.corrected_accel(net, pos, n, box)
    scaled = L.corrected_accel(net, pos, n, box, transfer=([0.2, 0.9], [0.7, 0.7]))
    assert np.allclose(scaled, 0.7 * plain, rtol=1e-12, atol=1e-14)
