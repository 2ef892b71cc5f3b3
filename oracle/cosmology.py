"""Background cosmology, growth factors, COLA time integrals and the linear spectrum (FP64).

Test infrastructure only (see the package docstring).

Units: lengths in h^-1 Mpc, wavenumbers in h Mpc^-1, time through the scale factor a,
H0 = 1, so that the canonical momentum p = a^2 dx/dt is in units of H0 h^-1 Mpc.

Paper passages followed:
  * flat LCDM with Omega_m = 0.25, Omega_L = 0.75, Omega_b = 0.044, n_s = 0.95,
    sigma_8 = 0.8, h = 0.7 -- Sec. 2.1 (the MICE-GC cosmology, which all runs share);
  * time nodes spaced uniformly in f(a), Delta f = (f(a_f) - f(a_i)) / (n - 1) -- Eq. 3,
    Sec. 4.2; the rule "initial a equals the step width" of Sec. 4.3 fixes that n counts
    the nodes including both ends (10 steps -> z_i = 9, 40 steps -> z_i = 39);
  * the growth factors and kick/drift integrals are not written in the paper (it cites
    the COLA papers); they follow from the equation of motion of Eq. 2 written with
    p = a^2 dx/dt and are derived in cola.py.
  * the paper's linear spectrum came from CAMB (Sec. 2.1), which is not available; the
    BBKS fit with the Sugiyama shape parameter stands in for it.
"""

import math

import numpy as np
from scipy import integrate


class Cosmology:
    """Flat LCDM parameters (Sec. 2.1)."""

    def __init__(self, omega_m=0.25, omega_b=0.044, h=0.7, n_s=0.95, sigma_8=0.8):
        self.omega_m = float(omega_m)
        self.omega_b = float(omega_b)
        self.h = float(h)
        self.n_s = float(n_s)
        self.sigma_8 = float(sigma_8)

    @property
    def omega_l(self):
        return 1.0 - self.omega_m


# --------------------------------------------------------------------------- expansion

def hubble_e(a, om):
    """E(a) = H(a)/H0 for flat LCDM without radiation."""
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(om * a ** -3 + (1.0 - om))


# --------------------------------------------------------------------------- growth

def growth_d1_heath(a, om):
    """Linear growth by the Heath integral, D1(a) ∝ E(a) ∫_0^a da'/(a' E(a'))^3,
    normalised to D1(1) = 1."""

    def unnorm(x):
        val, _ = integrate.quad(lambda t: 1.0 / (t * hubble_e(t, om)) ** 3, 0.0, x,
                                epsabs=0.0, epsrel=1e-13, limit=200)
        return 2.5 * om * hubble_e(x, om) * val

    norm = unnorm(1.0)
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    return np.array([unnorm(x) / norm for x in a])


def _growth_rhs(y, state, om):
    """Growth ODEs in y = ln a.

    With d/dt = a E d/da, the growing modes obey
        D'' + (2 + dlnE/dlna) D' = (3/2) Omega_m a^-3 / E^2 * source
    where ' = d/dlna, source = D1 for the first order and (D2 - D1^2) for the second
    order (the second-order LPT growth equation, whose EdS solution is -3/7 D1^2).
    """
    a = math.exp(y)
    e2 = om * a ** -3 + (1.0 - om)
    dlne = -1.5 * om * a ** -3 / e2
    coef = 1.5 * om * a ** -3 / e2
    d1, v1, d2, v2 = state
    return [v1, -(2.0 + dlne) * v1 + coef * d1,
            v2, -(2.0 + dlne) * v2 + coef * (d2 - d1 * d1)]


def growth_factors(a, om, a_start=1e-6):
    """(D1, D2, dD1/da, dD2/da) at the requested scale factors, normalised to D1(1) = 1.

    Integrated from deep in matter domination, where the growing modes are D1 = a and
    D2 = -(3/7) a^2, with an explicit 8th-order Runge-Kutta at rtol 1e-13.
    """
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    order = np.argsort(a)
    ys = np.log(a[order])
    y_eval = np.unique(np.concatenate([ys, [0.0]]))
    y0 = math.log(a_start)
    init = [a_start, a_start, -3.0 / 7.0 * a_start ** 2, -6.0 / 7.0 * a_start ** 2]
    sol = integrate.solve_ivp(_growth_rhs, (y0, max(0.0, y_eval[-1])), init,
                              method="DOP853", t_eval=y_eval, rtol=1e-13, atol=1e-300,
                              args=(om,))
    if not sol.success:
        raise RuntimeError(sol.message)
    idx1 = np.searchsorted(y_eval, 0.0)
    norm = sol.y[0, idx1]
    pos = np.searchsorted(y_eval, ys)
    d1 = sol.y[0, pos] / norm
    d2 = sol.y[2, pos] / norm ** 2
    # d/da = (1/a) d/dlna
    dd1 = sol.y[1, pos] / norm / a[order]
    dd2 = sol.y[3, pos] / norm ** 2 / a[order]
    out = np.empty((4, a.size))
    out[0, order], out[1, order], out[2, order], out[3, order] = d1, d2, dd1, dd2
    return out


# --------------------------------------------------------------------------- time integrals

def kick_integral(a0, a1, om):
    """K(a0, a1) = ∫ da / (a^2 E(a)): dp/da = (3/2) Omega_m g / (a^2 E)."""
    if a1 == a0:
        return 0.0
    val, _ = integrate.quad(lambda a: 1.0 / (a * a * hubble_e(a, om)), a0, a1,
                            epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def drift_integral(a0, a1, om):
    """Dr(a0, a1) = ∫ da / (a^3 E(a)): dx/da = p / (a^3 E)."""
    if a1 == a0:
        return 0.0
    val, _ = integrate.quad(lambda a: 1.0 / (a ** 3 * hubble_e(a, om)), a0, a1,
                            epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def time_nodes(a_init, n_steps, a_final=1.0, sampling="linear", power=None):
    """Eq. 3: n nodes uniformly spaced in f(a) from a_i to a_f, Delta f = (f(a_f)-f(a_i))/(n-1).

    sampling: "linear" f = a (the optimum of Sec. 4.2), "log" f = ln a, "power" f = a^p.
    """
    if n_steps < 2:
        raise ValueError("need at least two nodes")
    j = np.arange(n_steps, dtype=np.float64)
    if sampling == "linear":
        da = (a_final - a_init) / (n_steps - 1)
        nodes = a_init + j * da
    elif sampling == "log":
        df = (math.log(a_final) - math.log(a_init)) / (n_steps - 1)
        nodes = np.exp(math.log(a_init) + j * df)
    elif sampling == "power":
        df = (a_final ** power - a_init ** power) / (n_steps - 1)
        nodes = (a_init ** power + j * df) ** (1.0 / power)
    else:
        raise ValueError(sampling)
    nodes[-1] = a_final
    return nodes


def half_nodes(nodes):
    """Mid-points between consecutive nodes: a_{j+1/2} = (a_j + a_{j+1}) / 2."""
    nodes = np.asarray(nodes, dtype=np.float64)
    return 0.5 * (nodes[:-1] + nodes[1:])


# --------------------------------------------------------------------------- linear spectrum

def bbks_shape(cosmo):
    """Sugiyama shape parameter Gamma = Omega_m h exp(-Omega_b (1 + sqrt(2h)/Omega_m))."""
    return cosmo.omega_m * cosmo.h * math.exp(
        -cosmo.omega_b * (1.0 + math.sqrt(2.0 * cosmo.h) / cosmo.omega_m))


def bbks_transfer(k, cosmo):
    """BBKS transfer function T(q), q = k / Gamma, k in h/Mpc."""
    k = np.asarray(k, dtype=np.float64)
    q = k / bbks_shape(cosmo)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (np.log1p(2.34 * q) / (2.34 * q)
             * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)
    return np.where(q > 0, t, 1.0)


def tophat_window(x):
    """Fourier transform of a unit-volume spherical top-hat, 3 (sin x - x cos x) / x^3."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
    # below x = 0.1 the closed form cancels; its Taylor series is exact to 1e-14 there
    x2 = x * x
    series = 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 ** 3 / 15120.0
    return np.where(x > 0.1, w, series)


def sigma_r(pk_fn, radius, k_min=1e-7, k_max_r=2000.0):
    """sigma(R)^2 = ∫ dk k^2 P(k) W^2(kR) / (2 pi^2), integrated over ln k.

    The range [k_min, k_max_r / R] is cut into pieces no wider than about one
    oscillation of the window so that each adaptive quadrature sees a smooth integrand.
    """

    def integrand(lnk):
        k = math.exp(lnk)
        return k ** 3 * pk_fn(k) * float(tophat_window(k * radius)) ** 2 / (2.0 * math.pi ** 2)

    lo = math.log(k_min)
    hi = math.log(k_max_r / radius)
    # below kR = 1 the integrand is smooth; above it, cut at multiples of pi in kR
    x_edges = np.concatenate([[k_min * radius], np.arange(1.0, k_max_r, math.pi), [k_max_r]])
    edges = np.concatenate([np.linspace(lo, math.log(x_edges[1] / radius), 40)[:-1],
                            np.log(x_edges[1:] / radius)])
    assert abs(edges[-1] - hi) < 1e-12
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(integrand, a, b, epsabs=1e-24, epsrel=1e-11, limit=100)
        total += val
    return math.sqrt(total)


def linear_amplitude(cosmo):
    """Amplitude A of P(k) = A k^n_s T(k)^2 such that sigma(8 h^-1 Mpc) = sigma_8 at z = 0."""
    unnorm = sigma_r(lambda k: k ** cosmo.n_s * float(bbks_transfer(k, cosmo)) ** 2, 8.0)
    return (cosmo.sigma_8 / unnorm) ** 2


def linear_power(k, cosmo, amplitude=None):
    """Linear matter power spectrum at z = 0 (D1 = 1) in (h^-1 Mpc)^3."""
    if amplitude is None:
        amplitude = linear_amplitude(cosmo)
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        p = amplitude * k ** cosmo.n_s * bbks_transfer(k, cosmo) ** 2
    return np.where(k > 0, p, 0.0)


# --------------------------------------------------------------------------- paper constants

RHO_CRIT = 2.775e11  # critical density today in h^2 M_sun / Mpc^3 (h^-1 M_sun per (h^-1 Mpc)^3)


def particle_mass(cosmo, box, n_part):
    """m_p = Omega_m rho_crit (L / N)^3 in h^-1 M_sun."""
    return cosmo.omega_m * RHO_CRIT * (box / n_part) ** 3


def mesh_cell(box, n_part, pm_factor):
    """Force-mesh cell size: the mesh has pm_factor * n_part cells per side (Sec. 2.2)."""
    return box / (n_part * pm_factor)


def warren_mass(n, m_p):
    """Warren et al. halo mass M = m_p N (1 - N^-0.6) (Sec. 2.5)."""
    n = np.asarray(n, dtype=np.float64)
    return m_p * n * (1.0 - n ** -0.6)
