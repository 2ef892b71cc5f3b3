"""Learned short-range force correction on the coarse mesh (FP64 reference).

Test infrastructure only (see the package docstring).

Sec. 4.4 shows that a force mesh with PM_grid = 2 instead of 3 biases haloes through the force
resolution, and the conclusions (Sec. 7) ask for PM_grid of at least 3; the paper offers no
cheaper fix.  The correction studied here is this project's own: a small periodic 3D
convolutional network that maps the coarse (PM_grid = 1) mesh fields to a force correction,

  X0 = [delta, g_x, g_y, g_z] * input scales            (4 channels on the n^3 mesh)
  Z1 = conv3(W1, X0) + b1,  A1 = silu(Z1)               (3x3x3 taps, C channels)
  Z2 = conv3(W2, A1) + b2,  A2 = silu(Z2)               (3x3x3 taps, C channels)
  Y  = conv1(W3, A2) + b3,  dF = Y * out_scale          (1x1x1, 3 channels)
  optional band weight beta:  dF <- dF + beta (K dF - K K dF),
  K the periodic [1, 2, 1] / 4 smoothing along each mesh axis: K - K^2 multiplies a mode by
  c (1 - c) with c = prod_d cos^2(pi m_d / n), a band-pass that vanishes at k = 0 (as k^2) and at
  the Nyquist corner and peaks where c = 1/2.

conv3 is a periodic cross-correlation, Z[o][x] = sum_i sum_d W[o][i][d] X[i][x + d] with
d in {-1, 0, 1}^3 and tap index (dx+1)*9 + (dy+1)*3 + (dz+1); silu(z) = z / (1 + e^-z).  The
corrected force g + dF is interpolated to the particles with CIC.  Training minimises the
particle-level relative residual against the fine-mesh force on the same positions,

  L = sum_p |g1_p + G[dF]_p - g3_p|^2 / sum_p |g3_p - g1_p|^2,

G the CIC gather (L = 1 without the network).

Optional radial transfer of the Green's function (calibrated at trajectory level, not trained):
the mesh force becomes g_k = i k T(u) delta_k / k^2, u = |m| / (n/2) for the signed mode integers
m (|k| over the mesh's Nyquist wavenumber), T the cubic Hermite interpolant of knots (u_j, t_j)
with slope 0 at the first knot, centred-difference slopes inside and the one-sided slope at the
last knot, constant beyond the end knots; the network's input g is that filtered force and dF is
added unfiltered.
"""

import numpy as np
from scipy import fft as sfft

from . import lpt, pm

TAPS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def conv3(w, b, x):
    """Periodic 3x3x3 cross-correlation: w (O, I, 27), b (O,), x (I, n, n, n) -> (O, n, n, n)."""
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for t, (dx, dy, dz) in enumerate(TAPS):
        xs = np.roll(x, shift=(-dx, -dy, -dz), axis=(1, 2, 3))  # xs[i][p] = x[i][p + d]
        out += np.tensordot(w[:, :, t], xs, axes=([1], [0]))
    return out + b[:, None, None, None]


def conv3_backward(w, x, dz):
    """Gradients of conv3: returns (dw, db, dx) for upstream dz (O, n, n, n)."""
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for t, (ddx, ddy, ddz) in enumerate(TAPS):
        xs = np.roll(x, shift=(-ddx, -ddy, -ddz), axis=(1, 2, 3))
        dw[:, :, t] = np.tensordot(dz, xs, axes=([1, 2, 3], [1, 2, 3]))
        # z[o][p] gets w[o][i][t] x[i][p + d]: x[i][q] receives w[o][i][t] dz[o][q - d]
        contrib = np.tensordot(w[:, :, t], dz, axes=([0], [0]))
        dx += np.roll(contrib, shift=(ddx, ddy, ddz), axis=(1, 2, 3))
    db = dz.sum(axis=(1, 2, 3))
    return dw, db, dx


def conv1(w, b, x):
    """1x1x1 convolution: w (O, I), b (O,), x (I, ...)."""
    return np.tensordot(w, x, axes=([1], [0])) + b[:, None, None, None]


def binomial_smooth(x):
    """K: the periodic [1, 2, 1] / 4 smoothing along each of the last three axes."""
    for ax in (-3, -2, -1):
        x = 0.25 * np.roll(x, 1, axis=ax) + 0.5 * x + 0.25 * np.roll(x, -1, axis=ax)
    return x


def band_pass(x):
    """K x - K K x (symmetric, so it is its own adjoint)."""
    kx = binomial_smooth(x)
    return kx - binomial_smooth(kx)


class Net:
    """Parameters of the correction network (float64)."""

    def __init__(self, channels=16, seed=0, in_scale=(1.0, 1.0, 1.0, 1.0), out_scale=1.0, band=0.0):
        rng = np.random.default_rng(seed)
        c = channels
        self.c = c
        self.w1 = rng.normal(0, np.sqrt(2.0 / (4 * 27)), (c, 4, 27))
        self.b1 = np.zeros(c)
        self.w2 = rng.normal(0, np.sqrt(2.0 / (c * 27)), (c, c, 27))
        self.b2 = np.zeros(c)
        self.w3 = rng.normal(0, np.sqrt(1.0 / c), (3, c)) * 0.1
        self.b3 = np.zeros(3)
        self.in_scale = np.asarray(in_scale, dtype=np.float64)
        self.out_scale = float(out_scale)
        self.band = float(band)

    def params(self):
        return [self.w1, self.b1, self.w2, self.b2, self.w3, self.b3]


def forward(net, delta, g):
    """Correction dF (3, n, n, n) from delta (n, n, n) and mesh force g (3, n, n, n); returns (dF, cache)."""
    x0 = np.concatenate([delta[None], g]) * net.in_scale[:, None, None, None]
    z1 = conv3(net.w1, net.b1, x0)
    a1 = silu(z1)
    z2 = conv3(net.w2, net.b2, a1)
    a2 = silu(z2)
    y = conv1(net.w3, net.b3, a2)
    df = y * net.out_scale
    if net.band != 0.0:
        df = df + net.band * band_pass(df)
    return df, (x0, z1, a1, z2, a2)


def backward(net, cache, d_df):
    """Parameter gradients for upstream d_df (3, n, n, n) = dL/d(dF)."""
    x0, z1, a1, z2, a2 = cache
    if net.band != 0.0:
        d_df = d_df + net.band * band_pass(d_df)
    dy = d_df * net.out_scale
    dw3 = np.tensordot(dy, a2, axes=([1, 2, 3], [1, 2, 3]))
    db3 = dy.sum(axis=(1, 2, 3))
    da2 = np.tensordot(net.w3, dy, axes=([0], [0]))
    dz2 = da2 * silu_grad(z2)
    dw2, db2, da1 = conv3_backward(net.w2, a1, dz2)
    dz1 = da1 * silu_grad(z1)
    dw1, db1, _ = conv3_backward(net.w1, x0, dz1)
    return [dw1, db1, dw2, db2, dw3, db3]


def particle_loss(df_mesh, pos, box, g1, g3):
    """L and dL/d(dF mesh) for particles at pos (3, N) with coarse force g1 and target g3 (3, N)."""
    n = df_mesh.shape[-1]
    r = g1 + pm.cic_gather(df_mesh, pos, box) - g3
    denom = float(np.sum((g3 - g1) ** 2))
    loss = float(np.sum(r ** 2)) / denom
    # adjoint of the gather: CIC deposit of 2 r / denom
    idx, wts = pm._cic_corners(pos, n, box)
    grad = np.zeros((3, n ** 3))
    for c in range(3):
        vals = 2.0 * r[c] / denom
        grad[c] = np.bincount(idx.ravel(), weights=(wts * vals[None, :]).ravel(), minlength=n ** 3)
    return loss, grad.reshape(3, n, n, n)


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1; returns new (params, m, v).

    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    params <- params - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    """
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def hermite_transfer(u, u_knots, t_knots):
    """The transfer at u (any array): cubic Hermite on the knots, slope 0 at the first knot,
    (t_{j+1} - t_{j-1}) / (u_{j+1} - u_{j-1}) inside, one-sided at the last knot; t_0 below the
    first knot and t_last beyond the last (scipy's CubicHermiteSpline for the pieces)."""
    from scipy.interpolate import CubicHermiteSpline
    uk = np.asarray(u_knots, np.float64)
    tk = np.asarray(t_knots, np.float64)
    m = np.zeros_like(tk)
    m[1:-1] = (tk[2:] - tk[:-2]) / (uk[2:] - uk[:-2])
    m[-1] = (tk[-1] - tk[-2]) / (uk[-1] - uk[-2])
    u = np.asarray(u, np.float64)
    out = CubicHermiteSpline(uk, tk, m)(np.clip(u, uk[0], uk[-1]))
    return np.where(u <= uk[0], tk[0], np.where(u >= uk[-1], tk[-1], out))


def green_transfer(n, u_knots, t_knots):
    """T(u) on the rfftn grid of an n^3 mesh, u = |m| / (n/2) (hermite_transfer)."""
    mx, my, mz = lpt.mode_integers(n)
    u = np.sqrt((mx ** 2 + my ** 2 + mz ** 2).astype(np.float64)) / (n / 2.0)
    return hermite_transfer(u, u_knots, t_knots)


def corrected_accel(net, pos, n_mesh, box, transfer=None):
    """Mesh force plus the network's correction, interpolated to the particles (3, N).  transfer:
    (u_knots, t_knots) of the Green's function's radial transfer, or None for T = 1.  The transfer
    multiplies delta_k before the plain force operator (pm.force_mesh), which is the same as
    multiplying its Green's function."""
    delta = pm.density_contrast(pos, n_mesh, box)
    if transfer is None:
        g = pm.force_mesh(delta, box)
    else:
        dk = sfft.rfftn(delta) * green_transfer(n_mesh, *transfer)
        g = pm.force_mesh(sfft.irfftn(dk, s=delta.shape), box)
    df, _ = forward(net, delta, g)
    return pm.cic_gather(g + df, pos, box)


def flat_params(net):
    """Parameters in one flat array, in the order w1 b1 w2 b2 w3 b3 (C order within each)."""
    return np.concatenate([p.ravel() for p in net.params()])


def set_flat_params(net, flat):
    off = 0
    for p in net.params():
        p[...] = np.asarray(flat[off:off + p.size]).reshape(p.shape)
        off += p.size
