"""The corrected step's fused network kernels on a 128^3 mesh, against the float64 oracle.

In the corrected step the first convolution builds its periodic halo from the saved BF16 density
and the three force meshes, and the second ends with the 1x1x1 output layer that adds dF to the
force meshes.  On a 128^3 mesh there are 8 192 tiles of 4 x 4 x 16 voxels against a grid of at
most 4 096 blocks, and eight tiles along z, so the persistent multi-tile loop and the z-tile
decomposition run.  cola_pm_force_lc runs exactly those kernels (the step's force evaluation,
without the kick) on particles displaced from a 128^3 lattice (PM_grid 1, box 384, the learned
workload's 3 h^-1 Mpc cells), for
  * the trained C = 16 network of the learned workload (density input only), and
  * a random C = 16 network with the three force inputs switched on.
Reference: oracle.learned.corrected_accel.  Bounds: the mesh force part as the plain force
(relative RMS 1e-5 of g); the network's part, G[dF], to the BF16 forward bound, relative RMS
<= 1.5e-2 and cosine >= 0.9995 (the forward test's bounds).
"""

import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, learned as olc, pm as opm  # noqa: E402
from paper_1509_04685_amd import workloads as W  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N_PART, BOX = 128, 384.0


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


def check(cola, net, onet, seed, n_real=1):
    prob = cola.make_problem(BOX, N_PART, 1, 19.0, 40, n_real=n_real)
    n = N_PART ** 3
    disps = [W.random_displacements(N_PART, 2.0, seed=seed + r).astype(np.float32) for r in range(n_real)]
    st = cola.ParticleState(prob)
    st.x.copy_(torch.as_tensor(np.concatenate(disps, axis=1), device="cuda"))
    ws = cola.Workspace(prob)
    lws = cola.lc_workspace(N_PART, net.channels, n_real)
    got = cola.pm_force_lc(prob, st, net, lws, ws, a=1.0).cpu().numpy().astype(np.float64)
    plain = cola.pm_force(prob, st, ws).cpu().numpy().astype(np.float64)
    op = ocola.Problem(BOX, N_PART, 1, 19.0, 40)
    for r in range(n_real):
        pos = ocola.positions(ocola.State(disps[r].astype(np.float64), None, None, None), op)
        say(f"  oracle corrected force, realization {r}")
        ref = olc.corrected_accel(onet, pos, N_PART, BOX)
        ref_plain = opm.pm_accel(pos, N_PART, BOX)
        sl = slice(r * n, (r + 1) * n)
        e_plain = rel_rms(plain[:, sl], ref_plain)
        net_got, net_ref = got[:, sl] - plain[:, sl], ref - ref_plain
        e_net = rel_rms(net_got, net_ref)
        cos = cosine(net_got, net_ref)
        share = float(np.sqrt(np.mean(net_ref ** 2) / np.mean(ref_plain ** 2)))
        say(f"  plain {e_plain:.2e}; network part {e_net:.2e} (cos {cos:.6f}), "
            f"network/plain rms {share:.3f}")
        assert e_plain < 1e-5
        assert share > 1e-3  # the network does something
        assert e_net < 1.5e-2
        assert cos > 0.9995


def test_trained_network_128(cola):
    from paper_1509_04685_amd import learned as L
    path = os.path.join(ROOT, "paper_1509_04685_amd", "lc_weights_c16.json")
    if not os.path.exists(path):
        pytest.skip("no trained weights")
    say("corrected force, trained network, 128^3")
    net, doc = L.load_net(path)
    net.set_scales(net.in_scale, net.out_scale, 0.0, 0.0)
    net.set_schedule(None)  # output scale = out_scale, as in the oracle
    net.set_green_filter(None)  # the plain Green's function, as in the oracle's default
    onet = olc.Net(channels=net.channels, in_scale=net.in_scale, out_scale=net.out_scale)
    olc.set_flat_params(onet, np.asarray(doc["params"], dtype=np.float32).astype(np.float64))
    check(cola, net, onet, seed=1281)


def test_random_network_with_force_inputs_128(cola):
    say("corrected force, random network with force inputs, 128^3, two realizations")
    onet = olc.Net(channels=16, seed=128, in_scale=(0.5, 0.2, 0.2, 0.2), out_scale=0.3)
    onet.w3 *= 10.0
    rng = np.random.default_rng(129)
    onet.b1[:] = rng.normal(0, 0.1, 16)
    onet.b2[:] = rng.normal(0, 0.1, 16)
    flat = np.asarray(olc.flat_params(onet), dtype=np.float32)
    olc.set_flat_params(onet, flat.astype(np.float64))
    net = cola.LcNet(16, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale, training=False)
    check(cola, net, onet, seed=1290, n_real=2)


def test_green_filter_128(cola):
    """The Green's-function transfer T(u, a) of the corrected step: rows at the schedule's knots,
    evaluated between two knots (a = 0.6), against the oracle's corrected force with the same T
    interpolated in a by numpy and the schedule's output scale at a.  Bound: |got - ref| RMS <=
    1e-5 of the force plus 1.5e-2 of the network's part; the transfer moves the force by >1 %."""
    from paper_1509_04685_amd import learned as L
    path = os.path.join(ROOT, "paper_1509_04685_amd", "lc_weights_c16.json")
    if not os.path.exists(path):
        pytest.skip("no trained weights")
    say("corrected force with a Green's-function transfer, trained network, 128^3, a = 0.6")
    net, doc = L.load_net(path)
    knot_a = [0.05, 0.2, 0.35, 0.5, 0.65, 0.8, 1.0]
    knot_v = [0.9, 1.1, 1.0, 0.8, 1.2, 1.05, 1.0]
    u = [0.0, 0.2, 0.45, 0.7, 0.95, 1.3]
    rows = [[1.0 + 0.05 * i * np.sin(3.0 * uj + i) for uj in u] for i in range(len(knot_a))]
    net.set_scales(net.in_scale, net.out_scale, 0.0, 0.0)
    net.set_schedule(knot_a, knot_v)
    net.set_green_filter(u, rows)
    a = 0.6
    t_at = [float(np.interp(a, knot_a, [r[j] for r in rows])) for j in range(len(u))]
    scale = net.out_scale * float(np.interp(a, knot_a, knot_v))
    params = np.asarray(doc["params"], dtype=np.float32).astype(np.float64)
    onet = olc.Net(channels=net.channels, in_scale=net.in_scale, out_scale=scale)
    olc.set_flat_params(onet, params)
    onet0 = olc.Net(channels=net.channels, in_scale=net.in_scale, out_scale=0.0)
    olc.set_flat_params(onet0, params)
    prob = cola.make_problem(BOX, N_PART, 1, 19.0, 40)
    disp = W.random_displacements(N_PART, 2.0, seed=1301).astype(np.float32)
    st = cola.ParticleState(prob)
    st.x.copy_(torch.as_tensor(disp, device="cuda"))
    ws = cola.Workspace(prob)
    lws = cola.lc_workspace(N_PART, net.channels, 1)
    got = cola.pm_force_lc(prob, st, net, lws, ws, a=a).cpu().numpy().astype(np.float64)
    op = ocola.Problem(BOX, N_PART, 1, 19.0, 40)
    pos = ocola.positions(ocola.State(disp.astype(np.float64), None, None, None), op)
    say("  oracle corrected force with the transfer")
    ref = olc.corrected_accel(onet, pos, N_PART, BOX, transfer=(u, t_at))
    mesh_ref = olc.corrected_accel(onet0, pos, N_PART, BOX, transfer=(u, t_at))
    plain_ref = opm.pm_accel(pos, N_PART, BOX)
    rms = lambda x: float(np.sqrt(np.mean(x ** 2)))  # noqa: E731
    err = rms(got - ref)
    bound = 1e-5 * rms(ref) + 1.5e-2 * rms(ref - mesh_ref)
    effect = rms(mesh_ref - plain_ref) / rms(plain_ref)
    say(f"  |got - ref| {err:.3e} (bound {bound:.3e}); the transfer moves the mesh force by {effect:.3f}")
    assert effect > 1e-2
    assert err < bound
