"""The Jing (2005) aliasing correction of P(k) (Sec. 2.5) against the float64 oracle.

cola_power_spectrum_jing divides every mode by the CIC aliasing sum of its bin's local power law
(slope fitted to the current estimate, iterated); the oracle (power.bin_power_corrected) does the
same in float64 per mode, the GPU per class of sorted absolute mode integers in float32.
Two realizations (seeds 1 and 2) of the 32^3 / 96^3 case run to a = 1 on the GPU and in the
oracle; the corrected P(k) is compared on analysis meshes of 96^3, 48^3 (fewer bins asked for
than the mesh holds, and more) and 24^3 after 1 and 4 iterations.
Gate: n_modes equal to cola_power_spectrum's and the oracle's, k_mean to cola_power_spectrum's up to
the order of its float64 sums; per bin |P_gpu / P_oracle - 1| <= 1e-3 + the plain estimator's own error in that bin
(the correction is a smooth function of the same mode powers), and <= 1e-3 for k < 1 h/Mpc.
"""

import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, cosmology as ocosmo, power as opower  # noqa: E402
from paper_1509_04685_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04685_amd as c
    return c


@pytest.fixture(scope="module")
def runs(cola):
    cfg = W.CONFIGS["plain_32_96"]
    box, n_part, pm = cfg["box"], cfg["n_part"], cfg["pm_factor"]
    seeds = [1, 2]
    say("aliasing correction: 32^3 / 96^3 to a = 1, seeds 1 and 2")
    prob = cola.make_problem(box, n_part, pm, cfg["z_init"], cfg["n_steps"], n_real=2)
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=96)
    cola.ic_2lpt(prob, cosmo, seeds, st, ws)
    cola.step(prob, cosmo, st, cfg["n_steps"] - 1, ws)
    op = ocola.Problem(box, n_part, pm, cfg["z_init"], cfg["n_steps"])
    oc = ocosmo.Cosmology(**W.COSMOLOGY)
    sched = ocola.Schedule(op, oc)
    pos = []
    for s in seeds:
        ost = ocola.initial_state(op, oc, s)
        ocola.step(ost, op, sched, cfg["n_steps"] - 1)
        pos.append(ocola.positions(ost, op))
    return dict(prob=prob, cosmo=cosmo, st=st, ws=ws, pos=pos, box=box)


@pytest.mark.parametrize("n_pk,n_bins,iters", [(96, 64, 4), (48, 64, 4), (48, 30, 1), (24, 8, 4)])
def test_corrected_power_spectrum(cola, runs, n_pk, n_bins, iters):
    prob, cosmo, st, ws, box = runs["prob"], runs["cosmo"], runs["st"], runs["ws"], runs["box"]
    label = f"n_pk={n_pk} n_bins={n_bins} iterations={iters}"
    say(label)
    km0, pk0, nm0 = (t.cpu().numpy() for t in cola.power_spectrum(prob, cosmo, st, 1.0, n_pk, n_bins, ws))
    km, pk, nm = (t.cpu().numpy() for t in cola.power_spectrum_jing(prob, cosmo, st, 1.0, n_pk, n_bins, ws,
                                                                     iterations=iters))
    # k_mean: float64 atomic sums, equal up to their order
    assert np.allclose(km, km0, rtol=1e-12, atol=0) and np.array_equal(nm, nm0), label
    for r, pos in enumerate(runs["pos"]):
        ok_, opk, onm = opower.power_spectrum_corrected(pos, n_pk, box, n_bins, iterations=iters)
        _, opk0, _ = opower.power_spectrum(pos, n_pk, box, n_bins)
        assert np.array_equal(nm[r], onm), label
        sel = onm > 0
        err = np.abs(pk[r][sel] / opk[sel] - 1)
        err0 = np.abs(pk0[r][sel] / opk0[sel] - 1)
        effect = np.abs(opk[sel] / opk0[sel] - 1)
        tol = 1e-3 + err0
        say(f"  realization {r}: max |P/P_oracle - 1| = {err.max():.2e} (plain estimator {err0.max():.2e}); "
            f"the correction moves P by up to {effect.max():.2f}")
        assert np.all(err < tol), (label, r, err.max())
        low = ok_[sel] < 1.0
        assert np.all(err[low] < 1e-3), (label, r)
        # the correction does something: most near the Nyquist frequency, which 8 bins of 24^3 stop short of
        assert effect.max() > (0.02 if n_bins > n_pk // 2 else 2e-3)


def test_corrected_power_spectrum_rejects_bad_iterations(cola, runs):
    prob, cosmo, st, ws = runs["prob"], runs["cosmo"], runs["st"], runs["ws"]
    out = [torch.zeros((2, 16), dtype=torch.float64, device="cuda") for _ in range(3)]
    lib = cola._lib.lib()
    for iters in (0, 17):
        rc = lib.cola_power_spectrum_jing(ctypes.byref(prob), ctypes.byref(cosmo), ctypes.byref(st.c), 1.0, 48, 16,
                                          iters, ctypes.c_void_p(out[0].data_ptr()),
                                          ctypes.c_void_p(out[1].data_ptr()), ctypes.c_void_p(out[2].data_ptr()),
                                          ws.ptr, ws.nbytes, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == -1  # COLA_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert all(float(o.abs().sum()) == 0.0 for o in out)
