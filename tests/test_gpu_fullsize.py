"""Parity at the full sizes of the benchmarked workloads, in the launch configuration the bench uses
(FFT kernel shapes from the autotuner).

  * 256^3 particles / 768^3 mesh, box 768, seed 1: one COLA step against the float64 oracle
    (relative RMS displacement <= 1e-5, the stated gate), and momentum conservation of the
    full-size force (sum of g over particles <= 1e-5 of the sum of |g|);
  * 768^3 r2c FFT: sampled modes against direct float64 sums (error <= 1e-4 of the rms mode
    amplitude), and c2r(r2c(x)) = n^3 x;
  * 1536^3 mesh (the largest supported): a plane wave transforms to a single mode of amplitude
    n^3 / 2, every other mode below 1e-4 of it;
  * learned correction on the 256^3 mesh with the trained weights: sampled voxels against the
    oracle network evaluated on the 5^3 neighbourhood that each output depends on (relative RMS
    <= 2e-2, the BF16 bound of the forward parity test).
The oracle's float64 step at 768^3 takes tens of seconds on the host (FFTs on all cores).
"""

import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, cosmology as ocosmo, learned as olc  # noqa: E402
from paper_1509_04685_amd import workloads as W  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def workers():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def test_fullsize_one_step_and_momentum(cola):
    from scipy import fft as sfft
    cfg = W.CONFIGS["plain_256_768"]
    say("full size: GPU ICs + one step (256^3 / 768^3)")
    prob = cola.make_problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=768)
    cola.autotune(prob, ws, n_pk=768, state=st)
    cola.ic_2lpt(prob, cosmo, [cfg["seeds"][0]], st, ws)
    cola.step(prob, cosmo, st, 1, ws)
    x = st.x.cpu().numpy()
    st.invalidate_force()
    acc = cola.pm_force(prob, st, ws).cpu().numpy().astype(np.float64)
    assert np.abs(acc.sum(1)).max() < 1e-5 * np.abs(acc).sum(1).max()
    del acc
    say("full size: oracle ICs + one step")
    with sfft.set_workers(workers()):
        op = ocola.Problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
        oc = ocosmo.Cosmology(**W.COSMOLOGY)
        ost = ocola.initial_state(op, oc, cfg["seeds"][0])
        ocola.step(ost, op, ocola.Schedule(op, oc), 1)
    err = rel_rms(x, ost.disp)
    say(f"  relative RMS displacement {err:.2e}")
    assert err < 1e-5


def test_fullsize_fft_768(cola):
    n = 768
    say("full size: 768^3 FFT")
    prob = cola.make_problem(768.0, 256, 3, 19.0, 40)
    ws = cola.Workspace(prob, n_pk=768)
    cola.autotune(prob, ws, n_pk=768)
    x = W.random_field(n, seed=2024, dtype=np.float32)
    xd = torch.as_tensor(x, device="cuda")
    got = cola.fft_r2c(xd)
    idx = np.arange(n)
    x64 = x.astype(np.float64)
    vals = []
    refs = []
    for (a, b, c) in ((0, 0, 1), (1, 2, 3), (n // 2, 7, n // 2), (n - 1, n // 3, 5), (100, 600, 250)):
        ez = np.exp(-2j * np.pi * c * idx / n)
        ey = np.exp(-2j * np.pi * b * idx / n)
        ex = np.exp(-2j * np.pi * a * idx / n)
        ref = ex @ (np.tensordot(x64, ez, axes=([2], [0])) @ ey)
        vals.append(complex(got[a, b, c].item()))
        refs.append(ref)
    scale = float(np.sqrt(x64.size) * np.sqrt(np.mean(x64 ** 2)))  # rms of |X_k| for white noise
    err = max(abs(v - r) for v, r in zip(vals, refs))
    say(f"  max sampled error {err:.3e} (rms |X| {scale:.3e})")
    assert err < 1e-4 * scale
    back = cola.fft_c2r(got)
    r = (back / float(n) ** 3 - xd)
    assert float(torch.sqrt(torch.mean(r.double() ** 2)).cpu()) < 2e-6 * 10 * float(np.sqrt(np.mean(x64 ** 2)))


def test_fullsize_fft_1536_plane_wave(cola):
    n = 1536
    say("full size: 1536^3 plane wave")
    a, b, c = 3, 700, 11
    i = torch.arange(n, device="cuda", dtype=torch.int32)
    m = (a * i[:, None, None] + b * i[None, :, None] + c * i[None, None, :]) % n  # exact phase index
    x = torch.cos(m.float() * (2 * np.pi / n))
    del m
    torch.cuda.empty_cache()
    out = cola.fft_r2c(x)
    del x
    peak = out[a, b, c].item()
    amp = 0.5 * float(n) ** 3
    assert abs(peak.real - amp) < 1e-5 * amp and abs(peak.imag) < 1e-5 * amp
    out[a, b, c] = 0
    rest = float(out.abs().max().cpu())
    say(f"  peak {peak.real:.6e} (expected {amp:.6e}), largest other mode {rest:.3e}")
    assert rest < 1e-4 * amp


def test_fullsize_learned_sampled_voxels(cola):
    from paper_1509_04685_amd import learned as L
    path = os.path.join(ROOT, "paper_1509_04685_amd", "lc_weights_c16.json")
    if not os.path.exists(path):
        pytest.skip("no trained weights")
    say("full size: learned forward on 256^3 with the trained weights")
    net, doc = L.load_net(path)
    n = 256
    rng = np.random.default_rng(77)
    delta = (W.random_field(n, seed=78) * 2.0).astype(np.float32)
    g = np.stack([(W.random_field(n, seed=79 + d) * 3.0).astype(np.float32) for d in range(3)])
    ws = cola.lc_workspace(n, net.channels)
    df = cola.lc_forward(net, torch.as_tensor(delta, device="cuda"), torch.as_tensor(g, device="cuda"), ws)
    df = df.cpu().numpy()
    onet = olc.Net(channels=net.channels, in_scale=net.in_scale, out_scale=net.out_scale)
    olc.set_flat_params(onet, np.asarray(doc["params"], dtype=np.float32).astype(np.float64))
    got, ref = [], []
    for _ in range(24):
        v = rng.integers(0, n, size=3)
        sl = [np.arange(v[d] - 2, v[d] + 3) % n for d in range(3)]
        pd = delta[np.ix_(*sl)].astype(np.float64)
        pg = np.stack([g[c][np.ix_(*sl)] for c in range(3)]).astype(np.float64)
        out, _ = olc.forward(onet, pd, pg)
        ref.append(out[:, 2, 2, 2])
        got.append(df[:, v[0], v[1], v[2]])
    got, ref = np.array(got), np.array(ref)
    err = rel_rms(got, ref)
    say(f"  sampled relative RMS {err:.3e}")
    assert err < 2e-2


def test_fullsize_multipoles_properties(cola):
    """Multipoles on the 1024^3 analysis mesh after one step of the headline workload: the
    real-space monopole is cola_power_spectrum's P(k); the real-space quadrupoles about the three
    axes sum to zero mode by mode (L_2(mu_x) + L_2(mu_y) + L_2(mu_z) = 0); the redshift-space
    monopole exceeds the real-space one at the largest scales (Kaiser)."""
    cfg = W.CONFIGS["plain_256_768"]
    say("full size: multipoles on 1024^3 after one step")
    prob = cola.make_problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=1024)
    cola.ic_2lpt(prob, cosmo, [cfg["seeds"][0]], st, ws)
    cola.step(prob, cosmo, st, 1, ws)
    a = float(cola.schedule_table(prob, cosmo)[1, 0])
    n_bins = 400
    p2s = []
    for los in (0, 1, 2):
        km, p0, p2, p4, nm = cola.power_multipoles(prob, cosmo, st, a, 1024, n_bins, ws, los=los,
                                                   redshift_space=False)
        p2s.append(p2.cpu().numpy()[0])
    p0 = p0.cpu().numpy()[0]
    km2, pk, nm2 = cola.power_spectrum(prob, cosmo, st, a, 1024, n_bins, ws)
    pk = pk.cpu().numpy()[0]
    sel = pk > 0
    assert np.allclose(p0[sel], pk[sel], rtol=1e-10, atol=0)
    total = np.abs(p2s[0] + p2s[1] + p2s[2])[sel]
    assert np.all(total < 1e-9 * p0[sel])
    red = cola.power_multipoles(prob, cosmo, st, a, 1024, n_bins, ws, los=2)
    r0 = red[1].cpu().numpy()[0]
    low = sel & (km2.cpu().numpy()[0] < 0.05)
    ratio = r0[low].sum() / p0[low].sum()
    say(f"  redshift/real monopole at k < 0.05: {ratio:.3f} (linear theory at f = 1: 1.867)")
    assert 1.5 < ratio < 2.2


def test_fullsize_pm_only_one_step(cola):
    from scipy import fft as sfft
    cfg = W.CONFIGS["plain_256_768"]
    say("full size: PM-only ICs + one step (256^3 / 768^3)")
    prob = cola.make_problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"], frame="pm")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob)
    cola.ic_2lpt(prob, cosmo, [cfg["seeds"][0]], st, ws)
    cola.step(prob, cosmo, st, 1, ws)
    x = st.x.cpu().numpy()
    p = st.p.cpu().numpy()
    say("full size: oracle PM-only step")
    with sfft.set_workers(workers()):
        op = ocola.Problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
        oc = ocosmo.Cosmology(**W.COSMOLOGY)
        sched = ocola.Schedule(op, oc)
        ost = ocola.initial_state(op, oc, cfg["seeds"][0])
        c1, c2 = ocola.lpt_momentum_coefficients(sched.a[0], oc.omega_m)
        ost.p_res = c1 * ost.psi1 + c2 * ost.psi2
        ocola.step_pm_only(ost, op, sched, 1)
    err = rel_rms(x, ost.disp)
    say(f"  relative RMS displacement {err:.2e}, momentum {rel_rms(p, ost.p_res):.2e}")
    assert err < 1e-5
    assert rel_rms(p, ost.p_res) < 1e-4
