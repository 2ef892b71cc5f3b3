"""Training the learned correction on the GPU, and what it gains over the method without it.

Small case at the resolution of the learned workload (3 h^-1 Mpc coarse cells): 32^3 particles in
a 96 h^-1 Mpc box, fine mesh 96^3 (PM_grid 3), coarse mesh 32^3 (PM_grid 1), 20 nodes from z = 19.
Training pairs come from plain fine-mesh runs of seeds 4001-4003; the evaluation seed 4004 is
held out.  The test requires
  * the held-out particle loss to fall below 0.8 (1.0 without the network);
  * the final P(k) of the corrected 1x run to be closer to the plain 3x run than the plain 1x run
    is, by at least a third in the mean |P / P_3x - 1| over 0.2 < k < 1 h/Mpc.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1509_04685_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04685_amd as c
    return c


def test_training_gains_over_plain_coarse_mesh(cola):
    from paper_1509_04685_amd import learned as L
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    box, n_part, n_steps = 96.0, 32, 20
    say("lc training: samples")
    samples = L.make_samples(cosmo, box, n_part, 3, n_steps, 19.0, (4001, 4002, 4003), nodes=set(range(2, 20)))
    val = L.make_samples(cosmo, box, n_part, 3, n_steps, 19.0, (4004,), nodes=set(range(3, 20, 4)))
    net = L.new_net(samples[-1], channels=16, seed=1)
    tr = L.Trainer(net, n_part, box)
    v0 = tr.evaluate(val)
    for chunk in range(3):
        h = tr.train(samples, 200, 3e-3 * 0.3 ** chunk, batch=2, seed=chunk)
        say(f"  chunk {chunk}: training loss {h.mean():.4f}, validation {tr.evaluate(val):.4f}")
    v1 = tr.evaluate(val)
    say(f"  validation loss {v0:.4f} -> {v1:.4f}")
    assert v1 < 0.8
    n_pk, n_bins = 96, 48
    p3 = L.run_spectra(cola.make_problem(box, n_part, 3, 19.0, n_steps), cosmo, 4004, (1.0,), n_pk, n_bins)[0]
    prob1 = cola.make_problem(box, n_part, 1, 19.0, n_steps)
    p1 = L.run_spectra(prob1, cosmo, 4004, (1.0,), n_pk, n_bins)[0]
    plc = L.run_spectra(prob1, cosmo, 4004, (1.0,), n_pk, n_bins, net=net)[0]
    k = p3[0]
    sel = (k > 0.2) & (k < 1.0) & (p3[1] > 0)
    e1 = float(np.mean(np.abs(p1[1][sel] / p3[1][sel] - 1)))
    elc = float(np.mean(np.abs(plc[1][sel] / p3[1][sel] - 1)))
    say(f"  mean |P/P_3x - 1| for 0.2<k<1: plain 1x {e1:.4f}, learned 1x {elc:.4f}")
    assert elc < (2.0 / 3.0) * e1
