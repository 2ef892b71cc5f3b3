"""Pins of the time samplings of Eq. 3 (Sec. 4.2, Fig. 4): nodes equally spaced in f(a) for
f = a, ln a, a^0.5 and a^0.8, 40 nodes from z_i = 39 to a = 1.

  * linear: constant step density rho = 1 / da = (n - 1) / (1 - a_i), which is 40 for these nodes;
  * log: consecutive nodes in a constant ratio (a_f / a_i)^(1/(n-1));
  * power: a^p equally spaced; the density follows rho ~ f'(a) / df within O(da / a);
  * the text's comparison: at z < 2 the logarithmic sampling has the lowest step density of the
    four, and it has the highest density at the first step.
"""

import numpy as np

from oracle import cosmology as C

A_I = 1.0 / 40.0
N = 40


def nodes(kind, p=None):
    return C.time_nodes(A_I, N, 1.0, kind, p)


def density(a):
    return 1.0 / np.diff(a)


def test_linear_density_is_constant_40():
    rho = density(nodes("linear"))
    assert np.allclose(rho, 40.0, rtol=1e-12)


def test_log_nodes_are_geometric():
    a = nodes("log")
    r = a[1:] / a[:-1]
    assert np.allclose(r, (1.0 / A_I) ** (1.0 / (N - 1)), rtol=1e-12)
    assert a[0] == A_I and a[-1] == 1.0


def test_power_nodes_equally_spaced_in_a_to_the_p():
    for p in (0.5, 0.8):
        a = nodes("power", p)
        assert np.allclose(np.diff(a ** p), (1.0 - A_I ** p) / (N - 1), rtol=1e-10)
        # step density ~ f'(a) / df, evaluated at the mid-point of each step
        mid = 0.5 * (a[1:] + a[:-1])
        approx = p * mid ** (p - 1.0) / ((1.0 - A_I ** p) / (N - 1))
        rel = np.abs(density(a) / approx - 1.0)
        assert np.all(rel < 0.05 * np.diff(a) / mid + 1e-9)


def test_log_is_sparsest_late_and_densest_first():
    grids = {"linear": nodes("linear"), "log": nodes("log"), "p05": nodes("power", 0.5),
             "p08": nodes("power", 0.8)}
    # density at a common late time (z < 2, a > 1/3): interpolate each scheme's density at a = 0.5, 0.8
    for a_t in (0.4, 0.5, 0.8, 0.95):
        vals = {k: density(g)[np.searchsorted(g, a_t) - 1] for k, g in grids.items()}
        assert min(vals, key=vals.get) == "log"
    first = {k: density(g)[0] for k, g in grids.items()}
    assert max(first, key=first.get) == "log"
    # and the linear sampling has the most uniform density (ratio of largest to smallest)
    spread = {k: density(g).max() / density(g).min() for k, g in grids.items()}
    assert min(spread, key=spread.get) == "linear"
