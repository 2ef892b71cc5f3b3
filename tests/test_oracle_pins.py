"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form, a
library routine computing the same definition by another method, brute force on a tiny
input, an invariant, or a value the paper prints.  A plausible slip in the oracle (a
dropped term, a wrong sign or index, a transposed operand, a wrong normalisation) should
fail at least one of them.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy import fft as sfft
from scipy import integrate, special

from oracle import cola, cosmology, lpt, noise, pm, power

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
COSMO = cosmology.Cosmology()  # Sec. 2.1 cosmology


# --------------------------------------------------------------------------- helpers (tests only)

def naive_dft3(f):
    """Brute-force 3D DFT  F(m) = sum_x f(x) exp(-2 pi i m.x / n)  over the full cube."""
    n = f.shape[0]
    idx = np.arange(n)
    e = np.exp(-2j * np.pi * np.outer(idx, idx) / n)
    coords = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    out = np.zeros(n ** 3, dtype=complex)
    flat = f.ravel()
    for i, (mx, my, mz) in enumerate(coords):
        out[i] = np.sum(flat * (e[mx][:, None, None] * e[my][None, :, None]
                                * e[mz][None, None, :]).ravel())
    return out.reshape(n, n, n)


def sheets(n_x, n_yz, box):
    """Planes of particles: n_x planes in x (dense), one particle per mesh cell centre in y, z."""
    gx = np.arange(n_x) * (box / n_x)
    gy = (np.arange(n_yz) + 0.5) * (box / n_yz)
    X, Y, Z = np.meshgrid(gx, gy, gy, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


# --------------------------------------------------------------------------- P1: FFT conventions

@pytest.mark.parametrize("n", [6, 8, 12])
def test_p1_rfftn_is_the_dft(n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, n, n))
    ref = naive_dft3(f)
    assert np.allclose(sfft.rfftn(f), ref[:, :, : n // 2 + 1], rtol=0, atol=1e-11 * n ** 3)
    assert np.allclose(sfft.irfftn(ref[:, :, : n // 2 + 1], s=f.shape), f, atol=1e-12)


def test_p1_force_operator_brute_force():
    """pm.force_mesh equals (1/G) sum_k (i k_d / k^2) delta_k e^{ik.x} over the full cube,
    with k=0 and each component's own Nyquist plane left out."""
    n, box = 6, 10.0
    rng = np.random.default_rng(1)
    delta = rng.standard_normal((n, n, n))
    dk = naive_dft3(delta)
    m = np.fft.fftfreq(n, 1.0 / n).round().astype(int)  # includes -n/2
    kf = 2 * np.pi / box
    idx = np.arange(n)
    x = idx  # cell units; e^{ik.x} = e^{2 pi i m.j / n}
    ref = np.zeros((3, n, n, n))
    for ia, mx in enumerate(m):
        for ib, my in enumerate(m):
            for ic, mz in enumerate(m):
                k2 = (mx ** 2 + my ** 2 + mz ** 2) * kf ** 2
                if k2 == 0:
                    continue
                phase = np.exp(2j * np.pi * (mx * x[:, None, None] + my * x[None, :, None]
                                             + mz * x[None, None, :]) / n)
                for d, md in enumerate((mx, my, mz)):
                    if abs(md) == n // 2:
                        continue
                    ref[d] += np.real(1j * kf * md / k2 * dk[ia, ib, ic] * phase)
    ref /= n ** 3
    got = pm.force_mesh(delta, box)
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


# --------------------------------------------------------------------------- P2: growth and time integrals

def test_p2_einstein_de_sitter_closed_forms():
    a = np.array([0.05, 0.2, 0.5, 1.0])
    gf = cosmology.growth_factors(a, 1.0)
    assert np.allclose(gf[0], a, rtol=1e-10)
    assert np.allclose(gf[1], -3.0 / 7.0 * a ** 2, rtol=1e-10)
    assert np.allclose(gf[2], 1.0, rtol=1e-9)
    assert np.allclose(gf[3], -6.0 / 7.0 * a, rtol=1e-9)
    for a0, a1 in [(0.05, 0.15), (0.3, 0.35), (0.9, 1.0)]:
        assert cosmology.kick_integral(a0, a1, 1.0) == pytest.approx(
            2 * (math.sqrt(a1) - math.sqrt(a0)), rel=1e-12)
        assert cosmology.drift_integral(a0, a1, 1.0) == pytest.approx(
            2 * (a0 ** -0.5 - a1 ** -0.5), rel=1e-12)


def test_p2_heath_integral_equals_ode():
    a = np.array([0.05, 0.1, 0.3, 0.5, 0.8, 1.0])
    for om in (0.25, 0.3, 0.5):
        assert np.allclose(cosmology.growth_d1_heath(a, om),
                           cosmology.growth_factors(a, om)[0], rtol=1e-10)


def test_p2_growth_derivatives_and_second_order_limit():
    om = 0.25
    a = np.array([0.3, 0.6])
    h = 1e-5
    gp = cosmology.growth_factors(a + h, om)
    gm = cosmology.growth_factors(a - h, om)
    g = cosmology.growth_factors(a, om)
    assert np.allclose(g[2], (gp[0] - gm[0]) / (2 * h), rtol=1e-8)
    assert np.allclose(g[3], (gp[1] - gm[1]) / (2 * h), rtol=1e-8)
    # deep in matter domination LCDM reduces to EdS: D2 -> -3/7 D1^2
    early = cosmology.growth_factors([1e-3], om)
    assert early[1, 0] / (-3.0 / 7.0 * early[0, 0] ** 2) == pytest.approx(1.0, abs=1e-8)
    # Lambda slows the second-order growth less than the square of the first order:
    # D2 / (-3/7 D1^2) rises slightly above 1 by a = 1 (the Omega_m^(-1/143) fit gives ~1.0097)
    late = cosmology.growth_factors([1.0], om)
    ratio = late[1, 0] / (-3.0 / 7.0)
    assert 1.005 < ratio < 1.015
    assert ratio == pytest.approx(om ** (-1.0 / 143.0), rel=5e-4)


def test_p2_kick_drift_integrals_against_plain_quadrature():
    om = 0.25
    for a0, a1 in [(0.05, 0.0743590), (0.5, 0.55), (0.97, 1.0)]:
        x = np.linspace(a0, a1, 20001)
        e = np.sqrt(om * x ** -3 + 1 - om)
        assert cosmology.kick_integral(a0, a1, om) == pytest.approx(
            integrate.simpson(1 / (x ** 2 * e), x=x), rel=1e-10)
        assert cosmology.drift_integral(a0, a1, om) == pytest.approx(
            integrate.simpson(1 / (x ** 3 * e), x=x), rel=1e-10)


# --------------------------------------------------------------------------- P3: spectrum normalisation

def test_p3_tophat_window_is_the_ball_transform():
    """W(kR) equals the Fourier transform of a unit-volume ball, done by radial quadrature."""
    r = 8.0
    for k in (0.01, 0.1, 0.4, 1.3, 5.0):
        val, _ = integrate.quad(lambda s: np.sinc(k * s / np.pi) * 4 * np.pi * s * s, 0, r,
                                epsabs=1e-14, epsrel=1e-12, limit=200)
        assert float(cosmology.tophat_window(k * r)) == pytest.approx(
            val / (4 / 3 * np.pi * r ** 3), rel=1e-9, abs=1e-12)


def test_p3_sigma_of_white_spectrum_closed_form():
    """P = const: Parseval gives sigma^2(R) = P / V_R, V_R = 4 pi R^3 / 3; the integral is
    cut at kR = X, so subtract the tail 9 / (4 pi^2 X) P / R^3."""
    r, x_max = 8.0, 2000.0
    s = cosmology.sigma_r(lambda k: 1.0, r, k_max_r=x_max)
    expect = 1.0 / (4 / 3 * np.pi * r ** 3) - 9.0 / (4 * np.pi ** 2 * x_max) / r ** 3
    assert s ** 2 == pytest.approx(expect, rel=1e-5)


def test_p3_sigma8_recovered_by_a_plain_sum():
    amp = cosmology.linear_amplitude(COSMO)
    k = np.linspace(1e-5, 20.0, 400001)
    integrand = k ** 2 * cosmology.linear_power(k, COSMO, amp) \
        * cosmology.tophat_window(8.0 * k) ** 2 / (2 * np.pi ** 2)
    assert math.sqrt(integrate.simpson(integrand, x=k)) == pytest.approx(0.8, rel=1e-6)


def test_p3_bbks_limits():
    gamma = cosmology.bbks_shape(COSMO)
    # Sugiyama: Omega_m h exp(-Omega_b (1 + sqrt(2h)/Omega_m))
    assert gamma == pytest.approx(0.25 * 0.7 * math.exp(-0.044 * (1 + math.sqrt(1.4) / 0.25)))
    assert float(cosmology.bbks_transfer(1e-7, COSMO)) == pytest.approx(1.0, abs=1e-5)
    # large q: T -> ln(2.34 q) / (2.34 q) / (6.71 q)
    q = 1e6
    t = float(cosmology.bbks_transfer(q * gamma, COSMO))
    assert t == pytest.approx(math.log(2.34 * q) / (2.34 * q) / (6.71 * q), rel=1e-3)
    # monotone decreasing
    kk = np.logspace(-4, 2, 200)
    assert np.all(np.diff(cosmology.bbks_transfer(kk, COSMO)) < 0)


# --------------------------------------------------------------------------- P4: noise and initial field

def test_p4_philox_matches_numpy():
    """numpy's Philox (4x64, 10 rounds) returns the block of counter+1 first."""
    seed = 987654321
    for ctr in (1, 2, 12345, 2 ** 40 + 7):
        ref = np.random.Philox(counter=[ctr - 1, 0, 0, 0], key=[seed, 0]).random_raw(4)
        got = noise.philox4x64((np.array([ctr], np.uint64), np.zeros(1, np.uint64),
                                np.zeros(1, np.uint64), np.zeros(1, np.uint64)), (seed, 0))
        assert [int(g[0]) for g in got] == [int(r) for r in ref]


def test_p4_white_noise_moments():
    w = noise.white_noise(32, 7)
    assert abs(w.mean()) < 4 / math.sqrt(w.size)
    assert w.var() == pytest.approx(1.0, abs=4 * math.sqrt(2.0 / w.size))
    kurt = np.mean(w ** 4) / np.mean(w ** 2) ** 2
    assert kurt == pytest.approx(3.0, abs=0.1)
    assert not np.array_equal(w, noise.white_noise(32, 8))


def test_p4_first_order_divergence():
    """div Psi1 = -delta on every mode off the Nyquist planes."""
    n, box = 16, 200.0
    dk = lpt.gaussian_field_k(n, box, 3, COSMO)
    psi = lpt.first_order(dk, n, box)
    kx, ky, kz, _ = lpt.wavevectors(n, box)
    div = sum(1j * kv * sfft.rfftn(psi[d]) for d, kv in enumerate((kx, ky, kz)))
    mask = np.broadcast_to(
        lpt.nyquist_mask(n, 0) * lpt.nyquist_mask(n, 1) * lpt.nyquist_mask(n, 2), dk.shape) > 0
    assert np.allclose(div[mask], -dk[mask], atol=1e-12 * np.abs(dk).max())


def test_p4_initial_spectrum_chi2():
    """The binned power of the generated field matches P(k) with Gaussian scatter."""
    n, box = 32, 256.0
    amp = cosmology.linear_amplitude(COSMO)
    chi2, dof = 0.0, 0
    mx, my, mz = lpt.mode_integers(n)
    m2 = mx ** 2 + my ** 2 + mz ** 2
    kmag = 2 * np.pi / box * np.sqrt(m2)
    pmodel = cosmology.linear_power(kmag, COSMO, amp)
    w = np.broadcast_to(power.mode_weights(n), m2.shape)
    for seed in (1, 2, 3, 4):
        dk = lpt.gaussian_field_k(n, box, seed, COSMO, amp)
        delta = sfft.irfftn(dk, s=(n, n, n))
        _, pk, cnt = power.field_power(delta, box, n // 2)
        for b in range(1, n // 2):
            sel = (m2 >= b * b) & (m2 < (b + 1) ** 2)
            expect = np.sum(w[sel] * pmodel[sel]) / np.sum(w[sel])
            # independent complex modes ~ half the full-space count
            var = 2.0 * np.sum(w[sel] * pmodel[sel] ** 2) / np.sum(w[sel]) ** 2
            chi2 += (pk[b] - expect) ** 2 / var
            dof += 1
    assert 0.6 < chi2 / dof < 1.5


# --------------------------------------------------------------------------- P5: 2LPT closed forms

def test_p5_two_cosines_second_order():
    n, box = 16, 64.0
    kf = 2 * np.pi / box
    k1, k2 = 2 * kf, 3 * kf
    A, B = 0.7, -0.4
    q = lpt.lagrangian_grid(n, box)
    delta = A * np.cos(k1 * q[0]) + B * np.cos(k2 * q[1])
    dk = sfft.rfftn(delta)
    s = lpt.second_order_source(dk, n, box)
    assert np.allclose(s, A * B * np.cos(k1 * q[0]) * np.cos(k2 * q[1]), atol=1e-12)
    psi2 = lpt.second_order(dk, n, box)
    c = A * B / (k1 ** 2 + k2 ** 2)
    assert np.allclose(psi2[0], c * k1 * np.sin(k1 * q[0]) * np.cos(k2 * q[1]), atol=1e-12)
    assert np.allclose(psi2[1], c * k2 * np.cos(k1 * q[0]) * np.sin(k2 * q[1]), atol=1e-12)
    assert np.allclose(psi2[2], 0.0, atol=1e-12)
    psi1 = lpt.first_order(dk, n, box)
    assert np.allclose(psi1[0], -A / k1 * np.sin(k1 * q[0]), atol=1e-12)
    assert np.allclose(psi1[1], -B / k2 * np.sin(k2 * q[1]), atol=1e-12)


def test_p5_single_plane_wave_has_no_second_order():
    n, box = 12, 50.0
    q = lpt.lagrangian_grid(n, box)
    dk = sfft.rfftn(0.3 * np.cos(2 * np.pi / box * (q[0] + 2 * q[2])))
    assert np.allclose(lpt.second_order(dk, n, box), 0.0, atol=1e-13)


# --------------------------------------------------------------------------- P6/P7: plane-wave dynamics

def _plane_wave_run(n_g, n_steps, frame, amp=0.3, box=64.0, n_x=256):
    prob = cola.Problem(box, n_g, 1, 19.0, n_steps)
    sched = cola.Schedule(prob, COSMO)
    q = sheets(n_x, n_g, box)
    kw = 2 * np.pi / box
    psi1 = np.zeros_like(q)
    psi1[0] = -(amp / kw) * np.sin(kw * q[0])
    zero = np.zeros_like(q)
    if frame == "cola":
        st = cola.State(sched.d1[0] * psi1, zero.copy(), psi1, zero, q=q)
        cola.step(st, prob, sched, n_steps - 1)
    else:
        c1, _ = cola.lpt_momentum_coefficients(sched.a[0], COSMO.omega_m)
        st = cola.State(sched.d1[0] * psi1, c1 * psi1, psi1, zero, q=q)
        cola.step_pm_only(st, prob, sched, n_steps - 1)
    exact = sched.d1[-1] * psi1
    return st.disp, exact


def test_p6_zeldovich_plane_wave_any_step_count():
    """Before shell crossing 1D Zel'dovich is exact, so COLA's bracket is zero in the
    continuum: the result must match q + D1 Psi1 for any number of steps, up to the PM
    error, which drops ~4x per mesh doubling (O(kH)^2)."""
    errs = {}
    for n_g in (8, 16, 32):
        for n_steps in (3, 10):
            disp, exact = _plane_wave_run(n_g, n_steps, "cola")
            errs[n_g, n_steps] = np.abs(disp - exact).max() / np.abs(exact).max()
    for n_steps in (3, 10):
        assert errs[8, n_steps] / errs[16, n_steps] > 3.0
        assert errs[16, n_steps] / errs[32, n_steps] > 3.0
        assert errs[32, n_steps] < 0.012
    # the step count barely matters: 3 nodes do as well as 10
    assert abs(errs[32, 3] - errs[32, 10]) < 0.5 * errs[32, 10]


def test_p7_pm_only_converges_to_cola_at_second_order():
    """With the LPT frame switched off, the plain leapfrog reaches the COLA answer only as
    the steps shrink, at O(da^2): this pins the kick (3/2 Omega_m K) and drift (Dr)."""
    diffs = []
    for n_steps in (10, 20, 40):
        d_pm, exact = _plane_wave_run(16, n_steps, "pm")
        d_cola, _ = _plane_wave_run(16, n_steps, "cola")
        diffs.append(np.abs(d_pm - d_cola).max() / np.abs(exact).max())
    assert diffs[0] > 0.02
    assert diffs[0] / diffs[1] > 2.5
    assert diffs[1] / diffs[2] > 2.5


# --------------------------------------------------------------------------- P8: momentum, self-force

def test_p8_momentum_conservation():
    rng = np.random.default_rng(5)
    box, n_g = 100.0, 16
    pos = rng.uniform(0, box, (3, 300))
    g = pm.pm_accel(pos, n_g, box)
    assert np.abs(g.sum(axis=1)).max() < 1e-10 * np.abs(g).sum()


def test_p8_lone_particle_feels_no_force():
    rng = np.random.default_rng(6)
    box, n_g = 50.0, 12
    for _ in range(5):
        pos = rng.uniform(0, box, (3, 1))
        g = pm.pm_accel(pos, n_g, box)
        assert np.abs(g).max() < 1e-11 * box


# --------------------------------------------------------------------------- P9: Ewald two-body

def ewald_field(r, box, alpha_l=5.0, n_real=2, m_max=10):
    """grad G of the periodic Green's function (lap G = delta_D - 1/L^3) at separation r."""
    alpha = alpha_l / box
    grad = np.zeros(3)
    rng_n = range(-n_real, n_real + 1)
    for i in rng_n:
        for j in rng_n:
            for k in rng_n:
                s = r + box * np.array([i, j, k])
                d = np.linalg.norm(s)
                dg = special.erfc(alpha * d) / (4 * np.pi * d * d) \
                    + 2 * alpha / math.sqrt(math.pi) * math.exp(-(alpha * d) ** 2) / (4 * np.pi * d)
                grad += dg * s / d
    m = np.arange(-m_max, m_max + 1)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    kv = 2 * np.pi / box * np.stack([mx, my, mz], -1).reshape(-1, 3)
    k2 = np.sum(kv ** 2, 1)
    keep = k2 > 0
    kv, k2 = kv[keep], k2[keep]
    coef = np.exp(-k2 / (4 * alpha ** 2)) / k2 * np.sin(kv @ r)
    # grad of -(1/L^3) sum e^{-k^2/4a^2} cos(k.r)/k^2 = (1/L^3) sum k sin(k.r) e^{..}/k^2
    grad += (coef[:, None] * kv).sum(0) / box ** 3
    return grad


def test_p9_ewald_two_body():
    """PM force on particle A from B against -(1/n_bar) grad G_per(x_A - x_B), over random
    orientations and offsets.  The PM smooths at short range, so the median error falls
    with separation.  Pairs that share a mesh line are the known outliers of a spectral
    gradient: the Nyquist plane of a CIC spike is dropped by the derivative and that part of
    the field does not decay along the line; they are covered by the median, not a max."""
    box, n_g = 64.0, 64
    n_bar = 2 / box ** 3
    rng = np.random.default_rng(9)
    med = {}
    for sep in (4.0, 8.0, 12.0):
        rel, radial = [], []
        for _ in range(40):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            xa = rng.uniform(0, box, 3)
            xb = xa - sep * u
            pos = np.mod(np.stack([xa, xb], 1), box)
            g = pm.pm_accel(pos, n_g, box)[:, 0]
            ref = -ewald_field(xa - xb, box) / n_bar
            rel.append(np.linalg.norm(g - ref) / np.linalg.norm(ref))
            radial.append(np.dot(g, u) / np.dot(ref, u))
        med[sep] = float(np.median(rel))
        # sign (attraction) and normalisation of the mean radial force
        assert 0.9 < np.mean(radial) < 1.1
    assert med[4.0] < 0.04
    assert med[8.0] < 0.01
    assert med[12.0] < 0.005
    assert med[4.0] > med[8.0] > med[12.0]


def test_p9_pair_force_between_cell_centres():
    """Source and test point at cell centres carry no Nyquist content: the CIC pair force
    then follows the Ewald field to ~1% from 4 cells out."""
    box, n_g = 64.0, 64
    for sep in (4.0, 8.0):
        for axis in range(3):
            xb = np.array([10.5, 20.5, 30.5])
            xa = xb.copy()
            xa[axis] += sep
            g = pm.pm_accel(np.stack([xa, xb], 1), n_g, box)[:, 0]
            ref = -ewald_field(xa - xb, box) / (2 / box ** 3)
            assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 0.03


def test_p9_ewald_reference_itself():
    """The Ewald sum used above: far from images it reduces to -r_hat/(4 pi r^2) ... with a
    background correction; it is independent of the splitting parameter."""
    box = 64.0
    r = np.array([3.0, -1.0, 2.0])
    a = ewald_field(r, box, alpha_l=4.0, n_real=2, m_max=12)
    b = ewald_field(r, box, alpha_l=6.0, n_real=2, m_max=14)
    assert np.allclose(a, b, rtol=1e-9)
    d = np.linalg.norm(r)
    assert np.allclose(a, r / d / (4 * np.pi * d * d), rtol=2e-3)


# --------------------------------------------------------------------------- P10: paper constants

def test_p10_paper_constants():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        gold = json.load(fh)
    # Eq. 3 with the rule "initial scale factor = step width" (Sec. 4.3)
    for n_steps, z_i in gold["initial_redshift_rule"]["cases"]:
        a_i = 1.0 / (1.0 + z_i)
        nodes = cosmology.time_nodes(a_i, n_steps)
        assert nodes[1] - nodes[0] == pytest.approx(a_i, rel=1e-12)
    pm_ = gold["particle_mass"]
    mp = cosmology.particle_mass(COSMO, pm_["box"], pm_["n_part"])
    assert mp == pytest.approx(pm_["value"], rel=pm_["rel_tol"])
    mp2 = cosmology.particle_mass(COSMO, 1536.0, 2048)
    assert mp2 == pytest.approx(mp, rel=1e-12)
    for case in gold["mesh_cell"]["cases"]:
        assert cosmology.mesh_cell(case["box"], case["n_part"], case["pm_grid"]) == pytest.approx(
            case["value"], rel=1e-12)
    for case in gold["warren_mass"]["cases"]:
        m = cosmology.warren_mass(case["n"], mp)
        assert math.log10(m) == pytest.approx(case["log10_m"], abs=case["abs_tol"])
    # Sec. 4.4: PM_grid 3 -> 2 saves 70% of time if time scales with PM_grid^3
    assert 1 - (2 / 3) ** 3 == pytest.approx(gold["pm_grid_time_saving"]["value"], abs=0.01)


# --------------------------------------------------------------------------- P11: estimator expectation

def test_p11_poisson_shot_noise_expectation():
    """For Poisson particles the raw CIC estimator averages to
    (1/n_bar) prod_d [1 - (2/3) sin^2(pi m_d / n)] (aliased CIC window)."""
    rng = np.random.default_rng(11)
    box, n, n_part, n_real = 100.0, 16, 4000, 24
    n_bar = n_part / box ** 3
    acc = np.zeros(n // 2)
    cnt = None
    for _ in range(n_real):
        pos = rng.uniform(0, box, (3, n_part))
        _, pk, cnt = power.power_spectrum(pos, n, box, n // 2, deconvolve=False)
        acc += pk
    acc /= n_real
    mx, my, mz = lpt.mode_integers(n)
    m2 = mx ** 2 + my ** 2 + mz ** 2
    fac = ((1 - 2 / 3 * np.sin(np.pi * mx / n) ** 2) * (1 - 2 / 3 * np.sin(np.pi * my / n) ** 2)
           * (1 - 2 / 3 * np.sin(np.pi * mz / n) ** 2)) / n_bar
    w = np.broadcast_to(power.mode_weights(n), m2.shape)
    for b in range(1, n // 2):
        sel = (m2 >= b * b) & (m2 < (b + 1) ** 2)
        expect = np.sum(w[sel] * fac[sel]) / np.sum(w[sel])
        sigma = expect * math.sqrt(2.0 / (cnt[b] * n_real))
        assert abs(acc[b] - expect) < 4.5 * sigma, (b, acc[b], expect, sigma)


def test_p11_single_mode_normalisation():
    """A mesh field A cos(k.x) has P = (L^3/n^6) |n^3 A / 2|^2 in its bin, no window."""
    n, box, amp = 16, 80.0, 0.25
    x = np.arange(n) * box / n
    kf = 2 * np.pi / box
    delta = amp * np.cos(3 * kf * x)[:, None, None] * np.ones((n, n, n))
    _, pk, cnt = power.field_power(delta, box, n // 2)
    assert pk[3] * cnt[3] == pytest.approx(2 * box ** 3 / n ** 6 * (n ** 3 * amp / 2) ** 2)
    assert np.allclose(np.delete(pk, 3), 0.0, atol=1e-20)


# --------------------------------------------------------------------------- P12: lattices

def test_p12_lattices_give_zero_density_and_force():
    box, n = 40.0, 8
    q = lpt.lagrangian_grid(n, box).reshape(3, -1)
    for shift in (0.0, 0.5):
        pos = q + shift * box / n
        assert np.allclose(pm.density_contrast(pos, n, box), 0.0, atol=1e-13)
        assert np.abs(pm.pm_accel(pos, n, box)).max() < 1e-12
        k, pk, _ = power.power_spectrum(pos, n, box, n // 2)
        assert np.abs(pk).max() < 1e-25
    # PM_grid = 3: not uniform on the mesh, but every particle sits at a symmetric point
    pos = q + 0.3
    assert np.abs(pm.pm_accel(pos, 3 * n, box)).max() < 1e-11


# --------------------------------------------------------------------------- P13: linear growth

def test_p13_low_k_power_grows_as_d1_squared():
    """In a box large enough to be linear, the fundamental-mode power grows as
    (D1(a)/D1(a0))^2 for any step count (Appendix B: COLA keeps the linear growth
    regardless of the number of steps).  PM_grid = 3 as in the paper's optimum; the
    remaining ~1% is the lattice/mesh discreteness of a 32^3 particle load."""
    box, n_p = 4000.0, 32
    ratios = []
    for n_steps in (4, 10):
        prob = cola.Problem(box, n_p, 3, 19.0, n_steps)
        sched = cola.Schedule(prob, COSMO)
        st = cola.initial_state(prob, COSMO, seed=21)
        p0 = power.power_spectrum(cola.positions(st, prob), 96, box, 8)[1]
        cola.step(st, prob, sched, n_steps - 1)
        p1 = power.power_spectrum(cola.positions(st, prob), 96, box, 8)[1]
        ratios.append(p1[1] / p0[1] / (sched.d1[-1] / sched.d1[0]) ** 2)
    assert ratios[0] == pytest.approx(1.0, abs=0.02)
    assert ratios[1] == pytest.approx(1.0, abs=0.02)
    assert ratios[0] == pytest.approx(ratios[1], abs=0.006)


def test_p13_estimator_recovers_the_field_power_times_growth():
    """Particles displaced by 2LPT from the offset lattice: the CIC estimator returns the
    realization's own field power times D1^2 at low k."""
    box, n_p = 2000.0, 16
    prob = cola.Problem(box, n_p, 2, 19.0, 4)
    st = cola.initial_state(prob, COSMO, seed=21)
    d1 = cosmology.growth_factors([prob.a_init], COSMO.omega_m)[0, 0]
    dk = lpt.gaussian_field_k(n_p, box, 21, COSMO)
    pf = power.field_power(sfft.irfftn(dk, s=(n_p,) * 3), box, 8)[1]
    p0 = power.power_spectrum(cola.positions(st, prob), 32, box, 8)[1]
    assert np.allclose(p0[1:4] / pf[1:4] / d1 ** 2, 1.0, atol=0.01)


# --------------------------------------------------------------------------- P14: resume

def test_p14_resume_is_bitwise():
    prob = cola.Problem(100.0, 8, 2, 19.0, 6)
    sched = cola.Schedule(prob, COSMO)
    a = cola.initial_state(prob, COSMO, seed=4)
    b = a.copy()
    cola.step(a, prob, sched, 5)
    cola.step(b, prob, sched, 2)
    b.force = None  # a resumed run re-evaluates the node force: same inputs, same bits
    cola.step(b, prob, sched, 5)
    assert np.array_equal(a.disp, b.disp) and np.array_equal(a.p_res, b.p_res)


def test_p14_output_between_nodes_leaves_run_unchanged():
    prob = cola.Problem(100.0, 8, 2, 19.0, 6)
    cosmo = COSMO
    s1, snaps = cola.run(prob, cosmo, 4, outputs=(0.5, 1.0))
    s2, _ = cola.run(prob, cosmo, 4)
    assert np.array_equal(s1.disp, s2.disp)
    assert np.array_equal(snaps[1.0], s1.disp)
    # the partial drift is the step's own drift cut short: just before the next node it
    # lands on that node's displacement
    sched = cola.Schedule(prob, cosmo)
    j = int(np.searchsorted(sched.a, 0.5) - 1)
    st = cola.initial_state(prob, cosmo, 4)
    cola.step(st, prob, sched, j)
    near = cola.displacement_at(st, prob, sched, sched.a[j + 1] - 1e-12)
    cola.step(st, prob, sched, j + 1)
    assert np.allclose(near, st.disp, rtol=0, atol=1e-8)


# --------------------------------------------------------------------------- P15: aliasing correction

def _abs_modes(n):
    m = [np.abs(v).astype(np.float64) for v in np.broadcast_arrays(*lpt.mode_integers(n))]
    return m, m[0] ** 2 + m[1] ** 2 + m[2] ** 2


@pytest.mark.parametrize("n", [8, 12])
def test_p15_aliasing_sum_flat_spectrum_closed_form(n):
    """At n_eff = 0 the CIC aliasing sum is separable, and each axis sums to
    sum_j sinc^4(pi (x + j)) = 1 - (2/3) sin^2(pi x) (the sum of (x + j)^-4 is
    pi^4 (1 + 2 cos^2(pi x)) / (3 sin^4(pi x))).  The images dropped beyond |j_d| = J add at most
    2 / (3 pi^4 (J - 1/2)^3) per axis, against a per-axis sum of at least 1/3."""
    m, _ = _abs_modes(n)
    closed = np.prod([1 - 2 / 3 * np.sin(np.pi * v / n) ** 2 for v in m], axis=0)
    for J in (2, 6):
        bound = 3 * 3 * 2 / (3 * np.pi ** 4 * (J - 0.5) ** 3)
        err = np.abs(power.aliasing_sum(n, 0.0, J) / closed - 1).max()
        assert 0 < err < bound, (J, err, bound)


def test_p15_aliasing_sum_k_squared_closed_form():
    """At n_eff = 2 the factor |u|^2 = sum_d u_d^2 splits the sum into three separable products;
    with sum_j (x + j)^-2 = pi^2 / sin^2(pi x), the untruncated sum is
      C = (n^2 / (pi^2 |m|^2)) sum_d sin^2(pi m_d / n) prod_{e != d} [1 - (2/3) sin^2(pi m_e / n)].
    The truncated series approaches it from below, within 2 / (pi^2 (J - 1/2)) relative."""
    n = 6
    m, m2 = _abs_modes(n)
    f = [1 - 2 / 3 * np.sin(np.pi * v / n) ** 2 for v in m]
    g = [n * n * np.sin(np.pi * v / n) ** 2 / np.pi ** 2 for v in m]
    ok = m2 > 0
    closed = (g[0] * f[1] * f[2] + f[0] * g[1] * f[2] + f[0] * f[1] * g[2])[ok] / m2[ok]
    prev = None
    for J in (4, 12):
        c = power.aliasing_sum(n, 2.0, J)[ok]
        rel = 1 - c / closed
        assert rel.min() > 0 and rel.max() < 2 / (np.pi ** 2 * (J - 0.5)), (J, rel.max())
        if prev is not None:
            assert np.all(rel < prev)
        prev = rel


def test_p15_aliasing_sum_reduces_to_the_window_without_images():
    """No images: C = W^2, the plain CIC deconvolution, for any slope; and C is even in each m_d."""
    n = 10
    w2 = power.cic_window(n) ** 2
    for a in (-2.5, 0.0, 1.0):
        c = power.aliasing_sum(n, a, images=0)
        assert np.allclose(c.ravel()[1:], w2.ravel()[1:], rtol=1e-13)
    c = power.aliasing_sum(n, -1.5)
    assert np.allclose(c[1:n // 2, :, :], c[n - 1:n // 2:-1, :, :][:n // 2 - 1], rtol=1e-13)


def test_p15_local_slopes_of_a_power_law():
    """An exact power law gives its exponent in every bin whose window holds two bins (whatever the
    mode counts); empty bins and lone bins get 0; slopes are clamped to [-4, 4]."""
    k = np.array([0.0, 0.1, 0.2, 0.0, 0.25, 0.3, 0.36, 0.8])
    cnt = np.array([0.0, 6, 26, 0, 58, 80, 140, 900])
    for a in (-2.3, 0.7):
        pk = np.where(k > 0, 3.0 * np.where(k > 0, k, 1.0) ** a, 0.0)
        s = power.local_slopes(k, pk, cnt)
        assert np.allclose(s[[2, 4, 5, 6]], a, rtol=1e-12)
        assert s[0] == 0 and s[3] == 0 and s[1] == 0 and s[7] == 0  # 0.1 and 0.8: no neighbour in the window
    steep = np.where(k > 0, np.where(k > 0, k, 1.0) ** -9, 0.0)
    assert np.all(power.local_slopes(k, steep, cnt)[[2, 4, 5, 6]] == -4.0)
    # a kink: the slope of a window straddling it lies between the two exponents
    kk = np.where(k > 0, k, 1.0) / 0.22
    pk = np.where(k > 0, np.where(kk <= 1.0, kk ** -2.0, kk ** -1.0), 0.0)
    s = power.local_slopes(k, pk, cnt)
    assert -2.0 < s[4] < -1.0


def test_p15_corrected_shot_noise_is_flat():
    """Poisson particles have a flat spectrum 1/n_bar; the window-deconvolved estimate rises
    towards the mesh corners (the aliased CIC sum over W^2), the corrected estimate stays flat."""
    rng = np.random.default_rng(15)
    box, n, n_part = 100.0, 32, 400_000
    n_bar = n_part / box ** 3
    pos = rng.uniform(0, box, (3, n_part))
    _, pu, cnt = power.power_spectrum(pos, n, box, 27)
    _, pc, cnt2 = power.power_spectrum_corrected(pos, n, box, 27)
    assert np.array_equal(cnt, cnt2)
    sel = cnt > 50
    sig = np.sqrt(2.0 / cnt[sel])  # an exponential variable per mode pair
    r = pc[sel] * n_bar
    assert np.all(np.abs(r - 1) < 4 * sig + 0.005), np.abs(r - 1).max()
    assert abs(np.average(r, weights=cnt[sel]) - 1) < 0.01
    assert pu[20] * n_bar > 1.5  # what the correction removes near the corner (|m| = 20 > n/2)


def _zeldovich_lattice(n_p, box, n_eff, sigma, seed):
    """A lattice of n_p^3 particles displaced by a power-law Gaussian field (P ~ k^n_eff, rms
    density sigma) to first order; no shot noise, the lattice harmonics alias only to k = 0 on a
    mesh whose size divides n_p."""
    rng = np.random.default_rng(seed)
    f = np.fft.fftfreq(n_p, 1.0 / n_p)
    mx, my, mz = f[:, None, None], f[None, :, None], np.arange(n_p // 2 + 1)[None, None, :]
    m2 = mx ** 2 + my ** 2 + mz ** 2
    safe = np.where(m2 > 0, m2, 1.0)
    dk = sfft.rfftn(rng.standard_normal((n_p,) * 3)) * np.where(m2 > 0, safe ** (n_eff / 4), 0.0)
    dk *= sigma / sfft.irfftn(dk, s=(n_p,) * 3).std()
    kf = 2 * np.pi / box
    q = (np.indices((n_p,) * 3).reshape(3, -1) + 0.5) * (box / n_p)
    psi = [sfft.irfftn(1j * v / (safe * kf) * np.where(m2 > 0, dk, 0), s=(n_p,) * 3).ravel() for v in (mx, my, mz)]
    return np.mod(q + np.array(psi), box)


def test_p15_corrected_coarse_mesh_matches_a_fine_mesh():
    """Jing (2005) in practice: a 16^3 mesh's corrected P(k) of power-law particles agrees with
    the P(k) of the same particles on a 256^3 mesh (whose own aliasing is negligible at these k)
    up to the coarse Nyquist frequency, where the window-deconvolved estimate is 20-40% high.
    Averaged over four realizations: the correction works on expectation values, and each
    realization's aliased modes add coherently (a few per cent of scatter per bin)."""
    box, n, nb = 100.0, 16, 10
    rc, ru = [], []
    for seed in range(4):
        pos = _zeldovich_lattice(128, box, -1.5, 0.2, 40 + seed)
        _, pu, cnt = power.power_spectrum(pos, n, box, nb)
        _, pc, _ = power.power_spectrum_corrected(pos, n, box, nb)
        _, pf, _ = power.power_spectrum(pos, 256, box, nb)
        rc.append(pc[1:] / pf[1:] - 1)
        ru.append(pu[1:] / pf[1:] - 1)
    rc, ru = np.mean(rc, 0), np.mean(ru, 0)
    assert np.all(np.abs(rc[:8]) < 0.03), rc  # bins 1..8 (8 = Nyquist)
    assert np.abs(rc[:8]).max() < 0.25 * np.abs(ru[:8]).max()
    assert ru[7] > 0.2
