"""Parity of the HIP path (through the C ABI) with the float64 oracle, on identical seeded inputs.

Tolerances (float32 grids and FFTs against float64):
  * FFT: relative RMS <= 2e-6 x log2(n) per transform, max error <= 2e-5 of the max;
  * CIC density: |d| <= 1e-7 n (|delta| + 1 + cells/particles) per cell (float32 cell
    coordinate and atomic sums in any order);
  * PM force on identical positions: relative RMS <= 1e-5;
  * 2LPT initial conditions: relative RMS <= 1e-5 per field;
  * one COLA step: relative RMS displacement <= 1e-5 (the stated gate);
  * final P(k) after the 10-node run: max |P_gpu / P_oracle - 1| <= 1e-3 for k < 1 h/Mpc.
"""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, cosmology as ocosmo, lpt as olpt, pm as opm, power as opower  # noqa: E402
from paper_1509_04685_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04685_amd as c
    return c


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


# ----------------------------------------------------------------------------- FFT

@pytest.mark.parametrize("n", [4, 6, 8, 12, 16, 18, 24, 36, 48, 64, 96, 128, 192])
def test_fft_r2c_c2r(cola, n):
    say(f"fft n={n}")
    x = W.random_field(n, seed=100 + n)
    xk = np.fft.rfftn(x)
    got = cola.fft_r2c(to_dev(x)).cpu().numpy()
    err = np.abs(got - xk)
    tol = 2e-6 * max(1.0, math.log2(n))
    assert np.sqrt(np.mean(err ** 2) / np.mean(np.abs(xk) ** 2)) < tol
    assert err.max() < 2e-5 * np.abs(xk).max()
    back = cola.fft_c2r(torch.as_tensor(xk.astype(np.complex64), device="cuda")).cpu().numpy()
    assert rel_rms(back, x * n ** 3) < tol


def test_fft_large_sizes(cola):
    for n in (288, 384):
        say(f"fft n={n}")
        x = W.random_field(n, seed=7 + n, dtype=np.float32)
        xk = np.fft.rfftn(x.astype(np.float64))
        got = cola.fft_r2c(to_dev(x)).cpu().numpy()
        assert np.sqrt(np.mean(np.abs(got - xk) ** 2) / np.mean(np.abs(xk) ** 2)) < 2e-6 * math.log2(n)
        # sampled plain DFT at a few modes of the largest mesh
        idx = np.arange(n)
        for (a, b, c) in ((1, 2, 3), (n // 2, 5, n // 2), (n - 1, n // 3, 7)):
            ex = np.exp(-2j * np.pi * a * idx / n)
            ey = np.exp(-2j * np.pi * b * idx / n)
            ez = np.exp(-2j * np.pi * c * idx / n)
            ref = np.einsum("i,j,k,ijk->", ex, ey, ez, x.astype(np.float64))
            assert abs(got[a, b, c] - ref) < 1e-5 * np.abs(xk).max()


# ----------------------------------------------------------------------------- CIC density

@pytest.mark.parametrize("n_mesh,n,clustered", [(16, 3000, False), (48, 20000, True), (96, 200000, True)])
def test_cic_density(cola, n_mesh, n, clustered):
    say(f"cic n_mesh={n_mesh} n={n}")
    box = 100.0
    pos = (W.clustered_positions(n, box, 5) if clustered else W.uniform_positions(n, box, 5))
    pos32 = pos.astype(np.float32)
    got = cola.cic_density(to_dev(pos32), n_mesh, box).cpu().numpy()
    ref = opm.density_contrast(pos32.astype(np.float64), n_mesh, box)
    # The cell coordinate u = pos * n / L is formed in float32 (about 1e-7 n cell of rounding
    # per particle) and float32 atomics sum each cell in any order: the bound scales with the
    # cell's own value plus one particle's contribution (scale = cells / particles).
    scale = n_mesh ** 3 / n
    rel = float((np.abs(got - ref) / (1e-7 * n_mesh * (np.abs(ref) + 1.0 + scale))).max())
    assert rel < 1.0, rel


# ----------------------------------------------------------------------------- PM force

def gpu_state_from_disp(cola, prob, disp):
    st = cola.ParticleState(prob)
    st.x.copy_(to_dev(disp))
    return st


@pytest.mark.parametrize("n_part,pm,box,scale", [(8, 3, 50.0, 2.0), (16, 3, 100.0, 3.0), (32, 3, 256.0, 6.0),
                                                  (24, 2, 120.0, 4.0), (16, 1, 64.0, 2.0)])
def test_pm_force_identical_positions(cola, n_part, pm, box, scale):
    say(f"pm force n_part={n_part} pm={pm}")
    prob = cola.make_problem(box, n_part, pm, 19.0, 10)
    disp = W.random_displacements(n_part, scale, seed=n_part * 10 + pm).astype(np.float32)
    st = gpu_state_from_disp(cola, prob, disp)
    ws = cola.Workspace(prob)
    acc = cola.pm_force(prob, st, ws).cpu().numpy()
    op = ocola.Problem(box, n_part, pm, 19.0, 10)
    ref = opm.pm_accel(ocola.positions(ocola.State(disp.astype(np.float64), None, None, None), op),
                       op.n_mesh, box)
    assert rel_rms(acc, ref) < 1e-5
    # momentum conservation on the device
    assert np.abs(acc.astype(np.float64).sum(1)).max() < 1e-5 * np.abs(acc).sum(1).max()


@pytest.mark.parametrize("n_part,box", [(96, 300.0), (128, 400.0)])
def test_pm_force_static_plans(cola, n_part, box):
    """288^3 and 384^3 force meshes after the autotuner, which picks the compile-time plans
    (radix-6/12 prime-factor stages, twiddles read from LDS) for these sizes: every pass of the
    force (z r2c, y, fused x Green/gradient, y split, y inverse, three z c2r) against the float64
    oracle."""
    say(f"pm force static plans n_part={n_part}")
    prob = cola.make_problem(box, n_part, 3, 19.0, 10)
    ws = cola.Workspace(prob)
    report = cola.autotune(prob, ws)
    print(report)
    disp = W.random_displacements(n_part, 5.0, seed=5).astype(np.float32)
    st = gpu_state_from_disp(cola, prob, disp)
    acc = cola.pm_force(prob, st, ws).cpu().numpy()
    op = ocola.Problem(box, n_part, 3, 19.0, 10)
    ref = opm.pm_accel(ocola.positions(ocola.State(disp.astype(np.float64), None, None, None), op),
                       op.n_mesh, box)
    assert rel_rms(acc, ref) < 1e-5


def test_pm_force_lattice_is_zero(cola):
    say("pm force lattice")
    prob = cola.make_problem(256.0, 32, 3, 19.0, 10)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob)
    acc = cola.pm_force(prob, st, ws).cpu().numpy()
    assert np.abs(acc).max() < 1e-5


# ----------------------------------------------------------------------------- initial conditions

COSMO_KW = W.COSMOLOGY


def oracle_ic(n_part, box, seed, z_init=19.0, pm=3, n_steps=10):
    op = ocola.Problem(box, n_part, pm, z_init, n_steps)
    c = ocosmo.Cosmology(**COSMO_KW)
    return op, c, ocola.initial_state(op, c, seed)


@pytest.mark.parametrize("n_part,box,seed", [(16, 128.0, 3), (32, 256.0, 1), (48, 300.0, 1001)])
def test_ic_2lpt(cola, n_part, box, seed):
    say(f"ic n_part={n_part} seed={seed}")
    prob = cola.make_problem(box, n_part, 3, 19.0, 10)
    cosmo = cola.make_cosmology(**COSMO_KW)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob)
    cola.ic_2lpt(prob, cosmo, [seed], st, ws)
    _, _, ref = oracle_ic(n_part, box, seed)
    for name, got, want in (("psi1", st.psi1, ref.psi1), ("psi2", st.psi2, ref.psi2), ("x", st.x, ref.disp)):
        e = rel_rms(got.cpu().numpy(), want)
        assert e < 1e-5, (name, e)
    assert np.abs(st.p.cpu().numpy()).max() == 0.0
    assert st.node == 0


def test_ic_batch_matches_single(cola):
    say("ic batch")
    cosmo = cola.make_cosmology(**COSMO_KW)
    prob2 = cola.make_problem(128.0, 16, 3, 19.0, 10, n_real=2)
    st2 = cola.ParticleState(prob2)
    cola.ic_2lpt(prob2, cosmo, [5, 6], st2, cola.Workspace(prob2))
    prob1 = cola.make_problem(128.0, 16, 3, 19.0, 10)
    for r, seed in enumerate((5, 6)):
        st1 = cola.ParticleState(prob1)
        cola.ic_2lpt(prob1, cosmo, [seed], st1, cola.Workspace(prob1))
        n = 16 ** 3
        assert torch.equal(st1.psi1, st2.psi1[:, r * n:(r + 1) * n])
        assert torch.equal(st1.x, st2.x[:, r * n:(r + 1) * n])


# ----------------------------------------------------------------------------- stepping

def run_pair(cola, cfg, j_end, seed):
    prob = cola.make_problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
    cosmo = cola.make_cosmology(**COSMO_KW)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=cfg["n_part"] * cfg["pm_factor"])
    cola.ic_2lpt(prob, cosmo, [seed], st, ws)
    cola.step(prob, cosmo, st, j_end, ws)
    op = ocola.Problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
    c = ocosmo.Cosmology(**COSMO_KW)
    sched = ocola.Schedule(op, c)
    ost = ocola.initial_state(op, c, seed)
    ocola.step(ost, op, sched, j_end)
    return prob, cosmo, st, ws, op, sched, ost


def test_one_step_displacement(cola):
    cfg = W.CONFIGS["plain_32_96"]
    say("one step plain_32_96")
    prob, cosmo, st, ws, op, sched, ost = run_pair(cola, cfg, 1, 1)
    x = st.x.cpu().numpy()
    assert rel_rms(x, ost.disp) < 1e-5
    # the residual displacement (what the particle-mesh adds to 2LPT) agrees too
    lpt = sched.d1[1] * ost.psi1 + sched.d2[1] * ost.psi2
    assert rel_rms(x - lpt, ost.disp - lpt) < 1e-4
    assert rel_rms(st.p.cpu().numpy(), ost.p_res) < 1e-4


def test_full_run_power_spectrum(cola):
    cfg = W.CONFIGS["plain_32_96"]
    say("full run plain_32_96")
    n = cfg["n_steps"] - 1
    prob, cosmo, st, ws, op, sched, ost = run_pair(cola, cfg, n, 1)
    n_pk, n_bins = 96, 48
    km, pk, nm = cola.power_spectrum(prob, cosmo, st, 1.0, n_pk, n_bins, ws)
    km, pk, nm = km.cpu().numpy()[0], pk.cpu().numpy()[0], nm.cpu().numpy()[0]
    ok_, opk, onm = opower.power_spectrum(ocola.positions(ost, op), n_pk, cfg["box"], n_bins)
    assert np.array_equal(nm, onm)
    sel = (onm > 0) & (ok_ < 1.0)
    assert sel.sum() > 20
    assert np.allclose(km[sel], ok_[sel], rtol=1e-12)
    assert np.abs(pk[sel] / opk[sel] - 1).max() < 1e-3
    # the final displacement itself stays close after 10 nonlinear steps
    assert rel_rms(st.x.cpu().numpy(), ost.disp) < 1e-3


def test_power_spectrum_between_nodes(cola):
    cfg = W.CONFIGS["plain_32_96"]
    say("pk between nodes")
    prob, cosmo, st, ws, op, sched, ost = run_pair(cola, cfg, 4, 2)
    a_out = 0.5 * (sched.a[4] + sched.a[5]) + 0.01
    km, pk, nm = cola.power_spectrum(prob, cosmo, st, a_out, 96, 40, ws)
    disp = ocola.displacement_at(ost, op, sched, a_out)
    ok_, opk, onm = opower.power_spectrum(np.mod(ocola.lagrangian_positions(32, 256.0, 96) + disp, 256.0),
                                          96, 256.0, 40)
    pk = pk.cpu().numpy()[0]
    sel = onm > 0
    assert np.abs(pk[sel] / opk[sel] - 1).max() < 1e-3
    # the state is unchanged by the output: stepping on matches a run without it
    x_before = st.x.clone()
    assert st.node == 4
    cola.step(prob, cosmo, st, 5, ws)
    ocola.step(ost, op, sched, 5)
    assert rel_rms(st.x.cpu().numpy(), ost.disp) < 1e-4
    assert not torch.equal(x_before, st.x)


def test_resume_matches_uninterrupted(cola):
    cfg = W.CONFIGS["plain_32_96"]
    say("resume")
    cosmo = cola.make_cosmology(**COSMO_KW)
    prob = cola.make_problem(cfg["box"], 32, 3, 19.0, 10)
    a = cola.ParticleState(prob)
    b = cola.ParticleState(prob)
    wa, wb = cola.Workspace(prob), cola.Workspace(prob)
    cola.ic_2lpt(prob, cosmo, [3], a, wa)
    cola.ic_2lpt(prob, cosmo, [3], b, wb)
    cola.step(prob, cosmo, a, 6, wa)
    cola.step(prob, cosmo, b, 2, wb)
    cola.step(prob, cosmo, b, 6, wb)
    assert rel_rms(b.x.cpu().numpy(), a.x.cpu().numpy()) < 1e-5
    assert rel_rms(b.p.cpu().numpy(), a.p.cpu().numpy()) < 1e-5
    # a resumed run with the force cache dropped re-evaluates the same force
    b.invalidate_force()
    cola.step(prob, cosmo, b, 7, wb)
    cola.step(prob, cosmo, a, 7, wa)
    assert rel_rms(b.x.cpu().numpy(), a.x.cpu().numpy()) < 1e-5


# ----------------------------------------------------------------------------- autotuned shapes

def test_autotuned_shapes_keep_parity(cola):
    """The autotuner changes only kernel shapes (values per thread, tile widths); every shape
    must give the same transform and force."""
    say("autotune")
    prob = cola.make_problem(256.0, 32, 3, 19.0, 10)
    ws = cola.Workspace(prob, n_pk=48)
    report = cola.autotune(prob, ws, n_pk=48)
    assert "n=96" in report and "x_green" in report
    for n in (32, 48, 96):
        x = W.random_field(n, seed=300 + n)
        xk = np.fft.rfftn(x)
        got = cola.fft_r2c(to_dev(x)).cpu().numpy()
        assert np.sqrt(np.mean(np.abs(got - xk) ** 2) / np.mean(np.abs(xk) ** 2)) < 2e-6 * math.log2(n)
        back = cola.fft_c2r(torch.as_tensor(xk.astype(np.complex64), device="cuda")).cpu().numpy()
        assert rel_rms(back, x * n ** 3) < 2e-6 * math.log2(n)
    disp = W.random_displacements(32, 6.0, seed=77).astype(np.float32)
    st = gpu_state_from_disp(cola, prob, disp)
    acc = cola.pm_force(prob, st, ws).cpu().numpy()
    op = ocola.Problem(256.0, 32, 3, 19.0, 10)
    ref = opm.pm_accel(ocola.positions(ocola.State(disp.astype(np.float64), None, None, None), op), 96, 256.0)
    assert rel_rms(acc, ref) < 1e-5
