"""Learned coarse-mesh force correction: BF16 matrix-core kernels against the float64 oracle.

Tolerances (BF16 storage of activations and weights, unit roundoff 2^-9, FP32 accumulation):
  * matrix-core self-test on BF16-exact inputs: relative 1e-6 (FP32 accumulation of exact
    products);
  * network output dF: relative RMS <= 1.5e-2 and cosine >= 0.9995 against float64;
  * parameter gradients: per tensor relative L2 error <= 2e-2 and cosine >= 0.999 (weights), for
    the bias sums a bound of 2e-2 of the L2 norm of that layer's weight gradient per element;
  * particle loss and its mesh adjoint (FP32, no BF16): relative 1e-5;
  * Adam (FP32): relative 1e-5;
  * mesh fields of arbitrary positions: as the PM force (relative RMS 1e-5);
  * corrected COLA run against the oracle with the same network: relative RMS displacement
    <= 2e-3, while the correction itself moves the particles by more than 10x that.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, cosmology as ocosmo, learned as olc, pm as opm  # noqa: E402
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


def cosine(a, b):
    a, b = a.ravel(), b.ravel()
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(a):
    u = np.asarray(bf16_round(a), dtype=np.float32).view(np.uint32) >> 16
    return torch.as_tensor(u.astype(np.int16), device="cuda")


def make_pair(c, seed, in_scale=(0.5, 2.0, 2.0, 2.0), out_scale=0.25):
    """Oracle net and GPU net with identical (float32-representable) parameters."""
    onet = olc.Net(channels=c, seed=seed, in_scale=in_scale, out_scale=out_scale)
    onet.w3 *= 10.0
    onet.b1[:] = np.random.default_rng(seed + 1).normal(0, 0.1, c)
    onet.b2[:] = np.random.default_rng(seed + 2).normal(0, 0.1, c)
    onet.b3[:] = np.random.default_rng(seed + 3).normal(0, 0.1, 3)
    flat = np.asarray(olc.flat_params(onet), dtype=np.float32)
    olc.set_flat_params(onet, flat.astype(np.float64))
    return onet, flat


def fields(n, seed):
    delta = f32(W.random_field(n, seed) * 1.5)
    g = np.stack([f32(W.random_field(n, seed + 10 + d) * 0.7) for d in range(3)])
    return delta, g


# ----------------------------------------------------------------------------- matrix cores

def test_mfma_selftest(cola):
    say("mfma self-test")
    rng = np.random.default_rng(1)
    a = bf16_round(rng.normal(size=(16, 32)))
    b = bf16_round(rng.normal(size=(32, 16)))
    d = cola.mfma_selftest(bf16_bits(a), bf16_bits(b)).cpu().numpy()
    ref = a @ b
    assert np.allclose(d, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())


# ----------------------------------------------------------------------------- forward / backward

@pytest.mark.parametrize("n,c", [(16, 16), (32, 16), (16, 32), (48, 32)])
def test_forward_matches_oracle(cola, n, c):
    say(f"lc forward n={n} C={c}")
    onet, flat = make_pair(c, seed=20 + c)
    delta, g = fields(n, seed=30 + n)
    ref, _ = olc.forward(onet, delta, g)
    net = cola.LcNet(c, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale)
    ws = cola.lc_workspace(n, c, 1, training=False)
    got = cola.lc_forward(net, to_dev(delta), to_dev(g), ws).cpu().numpy()
    assert rel_rms(got, ref) < 1.5e-2
    assert cosine(got, ref) > 0.9995
    # accumulate mode adds onto what is there
    base = np.random.default_rng(5).normal(size=got.shape).astype(np.float32)
    acc = to_dev(base)
    cola.lc_forward(net, to_dev(delta), to_dev(g), ws, df=acc, accumulate=True)
    assert np.allclose(acc.cpu().numpy() - base, got, rtol=0, atol=1e-5 * np.abs(got).max())


@pytest.mark.parametrize("n,c", [(32, 16), (48, 32)])
def test_band_weight_forward_and_backward_match_oracle(cola, n, c):
    say(f"lc band weight n={n} C={c}")
    band = 0.9
    onet, flat = make_pair(c, seed=70 + c)
    onet.band = band
    delta, g = fields(n, seed=80 + n)
    ref, cache = olc.forward(onet, delta, g)
    net = cola.LcNet(c, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale)
    net.set_scales(net.in_scale, net.out_scale, 0.0, band)
    ws = cola.lc_workspace(n, c, 1, training=True)
    got = cola.lc_forward(net, to_dev(delta), to_dev(g), ws, training=True).cpu().numpy()
    assert rel_rms(got, ref) < 1.5e-2
    assert cosine(got, ref) > 0.9995
    d_df = f32(np.random.default_rng(90 + n).normal(size=(3, n, n, n)))
    refg = olc.backward(onet, cache, d_df)
    cola.lc_backward(net, to_dev(d_df), ws)
    gg = net.grads.cpu().numpy().astype(np.float64)
    rr = np.concatenate([r.ravel() for r in refg])
    for lo, hi in ((0, refg[0].size), (refg[0].size + refg[1].size, refg[0].size + refg[1].size + refg[2].size)):
        assert np.linalg.norm(gg[lo:hi] - rr[lo:hi]) / np.linalg.norm(rr[lo:hi]) < 2e-2
    # accumulate mode through the band weight adds onto what is there
    base = np.random.default_rng(6).normal(size=got.shape).astype(np.float32)
    acc = to_dev(base)
    cola.lc_forward(net, to_dev(delta), to_dev(g), ws, df=acc, accumulate=True)
    assert np.allclose(acc.cpu().numpy() - base, got, rtol=0, atol=1e-5 * np.abs(got).max())
    # a bias-only network gives a constant dF, which the band-pass leaves unchanged
    zero = flat.copy()
    zero[:-3] = 0.0
    net0 = cola.LcNet(c, params=zero, in_scale=onet.in_scale, out_scale=onet.out_scale)
    net0.set_scales(net0.in_scale, net0.out_scale, 0.0, band)
    const = cola.lc_forward(net0, to_dev(delta), to_dev(g), ws).cpu().numpy()
    for d in range(3):
        assert np.allclose(const[d], zero[-3 + d] * onet.out_scale, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("n,c", [(16, 16), (32, 16), (16, 32), (32, 32)])
def test_backward_matches_oracle(cola, n, c):
    say(f"lc backward n={n} C={c}")
    onet, flat = make_pair(c, seed=40 + c)
    delta, g = fields(n, seed=50 + n)
    _, cache = olc.forward(onet, delta, g)
    d_df = f32(np.random.default_rng(60 + n).normal(size=(3, n, n, n)))
    ref = olc.backward(onet, cache, d_df)
    net = cola.LcNet(c, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale)
    ws = cola.lc_workspace(n, c, 1, training=True)
    cola.lc_forward(net, to_dev(delta), to_dev(g), ws, training=True)
    cola.lc_backward(net, to_dev(d_df), ws)
    got = net.grads.cpu().numpy().astype(np.float64)
    off = 0
    names = ["w1", "b1", "w2", "b2", "w3", "b3"]
    parts = {}
    for name, r in zip(names, ref):
        parts[name] = (got[off:off + r.size].reshape(r.shape), r)
        off += r.size
    for name in ("w1", "w2", "w3"):
        gg, rr = parts[name]
        err = np.linalg.norm(gg - rr) / np.linalg.norm(rr)
        say(f"  {name}: rel L2 {err:.2e} cos {cosine(gg, rr):.6f}")
        assert err < 2e-2, name
        assert cosine(gg, rr) > 0.999, name
    for name, wname in (("b1", "w1"), ("b2", "w2"), ("b3", "w3")):
        gg, rr = parts[name]
        bound = 2e-2 * np.linalg.norm(parts[wname][1])
        say(f"  {name}: max err {np.abs(gg - rr).max():.2e} bound {bound:.2e}")
        assert np.abs(gg - rr).max() < bound, name
    # a second backward adds the same gradient again
    cola.lc_backward(net, to_dev(d_df), ws)
    again = net.grads.cpu().numpy().astype(np.float64)
    assert np.allclose(again, 2 * got, rtol=1e-4, atol=1e-6 * np.abs(got).max())


def test_loss_and_adjoint_match_oracle(cola):
    say("lc loss")
    n, box, npart = 16, 48.0, 5003
    pos = f32(W.clustered_positions(npart, box, seed=71))
    rng = np.random.default_rng(72)
    df = f32(rng.normal(size=(3, n, n, n)) * 0.3)
    g1 = f32(rng.normal(size=(3, npart)))
    g3 = f32(g1 + rng.normal(size=(3, npart)) * 0.5)
    ref_l, ref_d = olc.particle_loss(df, pos, box, g1, g3)
    stats, d_df = cola.lc_loss(to_dev(pos), box, to_dev(df), to_dev(g1), to_dev(g3))
    st = stats.cpu().numpy()
    assert st[0] == pytest.approx(ref_l, rel=1e-5)
    assert st[1] == pytest.approx(float(np.sum((g3 - g1) ** 2)), rel=1e-6)
    got = d_df.cpu().numpy()
    assert np.abs(got - ref_d).max() < 1e-5 * np.abs(ref_d).max()


def test_adam_matches_oracle(cola):
    say("lc adam")
    c = 16
    count = cola.lc_param_count(c)
    rng = np.random.default_rng(80)
    p = f32(rng.normal(size=count))
    net = cola.LcNet(c, params=p)
    m = np.zeros(count)
    v = np.zeros(count)
    ref = p.copy()
    for t in range(1, 4):
        g = f32(rng.normal(size=count) * 10.0 ** rng.uniform(-3, 1, size=count))
        net.grads.copy_(to_dev(g))
        net.adam(1e-3)
        ref, m, v = olc.adam_step(ref, g, m, v, t, 1e-3)
        got = net.params.cpu().numpy()
        assert np.allclose(got, ref, rtol=1e-5, atol=1e-7), t
        assert float(net.grads.abs().max().cpu()) == 0.0


# ----------------------------------------------------------------------------- helpers of training

def test_pm_fields_match_oracle(cola):
    say("pm fields")
    n, box, npart = 32, 64.0, 20011
    pos = f32(W.clustered_positions(npart, box, seed=91))
    f = cola.pm_fields(to_dev(pos), n, box)
    delta = opm.density_contrast(pos, n, box)
    g = opm.force_mesh(delta, box)
    acc = opm.cic_gather(g, pos, box)
    assert np.abs(f["delta"].cpu().numpy() - delta).max() < 1e-7 * n * (np.abs(delta).max() + 1 + n ** 3 / npart)
    assert rel_rms(f["g"].cpu().numpy(), g) < 1e-5
    assert rel_rms(f["acc"].cpu().numpy(), acc) < 1e-5


def test_positions_match_oracle(cola):
    say("positions")
    prob = cola.make_problem(100.0, 16, 2, 9.0, 4, n_real=2)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob)
    cola.ic_2lpt(prob, cola.make_cosmology(**W.COSMOLOGY), [3, 4], st, ws)
    st.x.mul_(40.0)  # large displacements so that many particles wrap
    pos = cola.positions(prob, st).cpu().numpy()
    x = st.x.cpu().numpy().astype(np.float64)
    op = ocola.Problem(100.0, 16, 2, 9.0, 4)
    n = 16 ** 3
    for r in range(2):
        s = ocola.State(x[:, r * n:(r + 1) * n], None, None, None)
        ref = ocola.positions(s, op)
        d = np.abs(pos[:, r * n:(r + 1) * n] - ref)
        d = np.minimum(d, 100.0 - d)  # periodic distance
        assert d.max() < 2e-5 * 100.0
    assert pos.min() >= 0.0 and pos.max() < 100.0


# ----------------------------------------------------------------------------- corrected step

def _small_problem(cola, n_real=1):
    return cola.make_problem(64.0, 16, 1, 19.0, 5, n_real=n_real)


def test_zero_network_step_equals_plain_step(cola):
    say("step_lc with a zero network")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    prob = _small_problem(cola)
    flat = cola.lc_init_params(16, seed=3)
    o = olc.Net(channels=16)
    cut = sum(p.size for p in o.params()[:4])
    flat[cut:] = 0.0  # w3 = b3 = 0
    net = cola.LcNet(16, params=flat, training=False)
    a = cola.ParticleState(prob)
    b = cola.ParticleState(prob)
    ws_a, ws_b = cola.Workspace(prob), cola.Workspace(prob)
    lws = cola.lc_workspace(16, 16, 1)
    cola.ic_2lpt(prob, cosmo, [5], a, ws_a)
    cola.ic_2lpt(prob, cosmo, [5], b, ws_b)
    cola.step(prob, cosmo, a, 4, ws_a)
    cola.step_lc(prob, cosmo, b, 4, net, lws, ws_b)
    assert rel_rms(b.x.cpu().numpy(), a.x.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("n_real,band", [(1, 0.0), (2, 0.0), (2, 0.9)])
def test_corrected_run_matches_oracle(cola, n_real, band):
    say(f"corrected run vs oracle, n_real={n_real} band={band}")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    prob = _small_problem(cola, n_real)
    onet, flat = make_pair(16, seed=7, in_scale=(0.25, 1.0, 1.0, 1.0), out_scale=0.5)
    onet.band = band
    net = cola.LcNet(16, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale, training=False)
    net.set_scales(net.in_scale, net.out_scale, 0.0, band)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob)
    lws = cola.lc_workspace(16, 16, n_real)
    seeds = [11, 12][:n_real]
    cola.ic_2lpt(prob, cosmo, seeds, st, ws)
    cola.step_lc(prob, cosmo, st, 4, net, lws, ws)
    x = st.x.cpu().numpy()
    oc = ocosmo.Cosmology(**W.COSMOLOGY)
    op = ocola.Problem(64.0, 16, 1, 19.0, 5)
    op.accel = lambda pos, n_mesh, box: olc.corrected_accel(onet, pos, n_mesh, box)
    plain_p = ocola.Problem(64.0, 16, 1, 19.0, 5)
    n = 16 ** 3
    for r, seed in enumerate(seeds):
        ost, _ = ocola.run(op, oc, seed)
        pst, _ = ocola.run(plain_p, oc, seed)
        err = rel_rms(x[:, r * n:(r + 1) * n], ost.disp)
        effect = rel_rms(pst.disp, ost.disp)
        say(f"  seed {seed}: err {err:.2e}, effect of the correction {effect:.2e}")
        assert err < 2e-3
        assert effect > 10 * 2e-3


def test_schedule_equals_node_by_node_scales(cola):
    """A knot schedule in one call equals stepping one node at a time with the interpolated scale
    set by hand (knots constant below the first force nodes so both runs start alike)."""
    say("output-scale schedule")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    prob = cola.make_problem(64.0, 16, 1, 19.0, 6)
    a = cola.schedule_table(prob, cosmo)[:, 0]
    onet, flat = make_pair(16, seed=9, in_scale=(0.25, 1.0, 1.0, 1.0), out_scale=0.5)
    knot_a, knot_v = [0.3, 0.6, 0.9], [1.5, 0.7, 1.2]
    assert a[1] < knot_a[0]
    lws = cola.lc_workspace(16, 16, 1)
    xs = []
    for mode in ("schedule", "by hand"):
        net = cola.LcNet(16, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale, training=False)
        st = cola.ParticleState(prob)
        ws = cola.Workspace(prob)
        cola.ic_2lpt(prob, cosmo, [5], st, ws)
        if mode == "schedule":
            net.set_schedule(knot_a, knot_v)
            cola.step_lc(prob, cosmo, st, 5, net, lws, ws)
        else:
            for j in range(1, 6):
                net.set_scales(net.in_scale, onet.out_scale * float(np.interp(a[j], knot_a, knot_v)), 0.0)
                cola.step_lc(prob, cosmo, st, j, net, lws, ws)
        xs.append(st.x.cpu().numpy())
    assert rel_rms(xs[0], xs[1]) < 1e-6
    # the schedule changes the run
    net = cola.LcNet(16, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale, training=False)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob)
    cola.ic_2lpt(prob, cosmo, [5], st, ws)
    cola.step_lc(prob, cosmo, st, 5, net, lws, ws)
    assert rel_rms(st.x.cpu().numpy(), xs[0]) > 1e-4
