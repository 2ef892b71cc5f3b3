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


def test_gradients_match_finite_differences():
    net, delta, g, box, pos, g1, g3 = _setup()
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


def test_loss_is_one_without_correction():
    net, delta, g, box, pos, g1, g3 = _setup()
    zero = np.zeros((3,) + delta.shape)
    assert L.particle_loss(zero, pos, box, g1, g3)[0] == pytest.approx(1.0)
