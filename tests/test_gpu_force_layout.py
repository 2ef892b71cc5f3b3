"""The step's force path with its interleaved force mesh, against the float64 oracle.

cola_pm_force (and every step) inverts the three force spectra in one z pass that writes
(F_x, F_y, F_z) of each cell next to each other, and the CIC gathers read a cell pair's three
components as 24 contiguous bytes (Sec. 2.2: the mesh force interpolated back with the deposit's
cloud-in-cell weights).  The pass has several kernel shapes (values per thread, lines per block,
compile-time or run-time plans; three thread groups per block, one per component): each admissible
one is pinned in turn and the accelerations compared with the oracle on identical positions
(relative RMS <= 1e-5, as the other force tests).  A batch of two realizations must give each
realization's force bit for bit (the force mesh of realization r sits fstride floats after r - 1).
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, pm as opm  # noqa: E402
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


def oracle_accel(disp, n_part, pm, box):
    op = ocola.Problem(box, n_part, pm, 19.0, 10)
    return opm.pm_accel(ocola.positions(ocola.State(disp.astype(np.float64), None, None, None), op), op.n_mesh, box)


# (n_part, pm, box, shapes): a 72^3 mesh (run-time plans only) and a 288^3 mesh (compile-time
# plans too); a shape is (values per thread, lines per block, compile-time plan)
CASES = [(24, 3, 120.0, [(6, 1, False), (6, 8, False), (12, 2, False), (12, 8, False)]),
         (96, 3, 300.0, [(6, 4, False), (12, 8, True), (12, 16, False), (24, 1, True), (24, 32, True)])]


@pytest.mark.parametrize("n_part,pm,box,shapes", CASES)
def test_interleaved_force_every_shape(cola, n_part, pm, box, shapes):
    n = n_part * pm
    disp = W.random_displacements(n_part, 4.0, seed=n_part + 7).astype(np.float32)
    ref = oracle_accel(disp, n_part, pm, box)
    prob = cola.make_problem(box, n_part, pm, 19.0, 10)
    ws = cola.Workspace(prob)
    st = cola.ParticleState(prob)
    st.x.copy_(torch.from_numpy(disp).cuda())
    for R, width, stat in shapes:
        cola.fft_set_shape(n, "z_c2r3", R, width, use_static=stat)
        say(f"interleaved force {n}^3: z_c2r3 R={R} width={width} static={stat}")
        acc = cola.pm_force(prob, st, ws).cpu().numpy()
        e = rel_rms(acc, ref)
        assert e < 1e-5, (R, width, stat, e)


def test_interleaved_force_batch_matches_single(cola):
    n_part, pm, box = 32, 3, 200.0
    disps = [W.random_displacements(n_part, 5.0, seed=s).astype(np.float32) for s in (11, 12)]
    prob2 = cola.make_problem(box, n_part, pm, 19.0, 10, n_real=2)
    st2 = cola.ParticleState(prob2)
    st2.x.copy_(torch.from_numpy(np.concatenate(disps, axis=1)).cuda())
    acc2 = cola.pm_force(prob2, st2, cola.Workspace(prob2)).cpu().numpy()
    prob1 = cola.make_problem(box, n_part, pm, 19.0, 10)
    ws1 = cola.Workspace(prob1)
    npr = n_part ** 3
    for r, d in enumerate(disps):
        st1 = cola.ParticleState(prob1)
        st1.x.copy_(torch.from_numpy(d).cuda())
        acc1 = cola.pm_force(prob1, st1, ws1).cpu().numpy()
        assert np.array_equal(acc2[:, r * npr:(r + 1) * npr], acc1), r
        assert rel_rms(acc1, oracle_accel(d, n_part, pm, box)) < 1e-5
