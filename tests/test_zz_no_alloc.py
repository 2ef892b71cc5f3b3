"""cola_pm_force_noalloc: the allocation-free form of cola_pm_force (its workspace is a fixed device
array of the library), called through the C ABI and compared with cola_pm_force on a caller
workspace.  Both run the same kernels on the same inputs with a deterministic deposit (fixed-point
sums) and FFT, so the accelerations must agree bit for bit.  Two calls in a row, the second on a
smaller problem, show that nothing left in the shared array from the first call leaks into the
second; a problem beyond the array's 96 MiB is rejected before any launch.
"""

import ctypes
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


def noalloc_force(cola, prob, st):
    from paper_1509_04685_amd import _lib
    acc = torch.empty((3, st.n), dtype=torch.float32, device="cuda")
    ptrs = (ctypes.c_void_p * 3)(*[acc[d].data_ptr() for d in range(3)])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.lib().cola_pm_force_noalloc(ctypes.byref(prob), ctypes.byref(st.c), ptrs, stream),
               "cola_pm_force_noalloc")
    return acc


def test_noalloc_matches_workspace_form(cola):
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    # first 64^3 particles on a 128^3 mesh (65 MiB of workspace), then a smaller batch of two
    # 24^3 / 72^3 realizations
    for box, n_part, pm, n_real, seeds in ((256.0, 64, 2, 1, [3]), (96.0, 24, 3, 2, [4, 5])):
        say(f"noalloc force: {n_real} x {n_part}^3 particles, {n_part * pm}^3 mesh")
        prob = cola.make_problem(box, n_part, pm, 19.0, 10, n_real=n_real)
        st = cola.ParticleState(prob)
        ws = cola.Workspace(prob)
        cola.ic_2lpt(prob, cosmo, seeds, st, ws)
        st.x.mul_(30.0)  # displacements of several cells, so the deposit sorts across tiles
        want = cola.pm_force(prob, st, ws)
        got = noalloc_force(cola, prob, st)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert float(want.abs().max()) > 0.0


def test_noalloc_rejects_beyond_its_array(cola):
    from paper_1509_04685_amd import _lib
    prob = cola.make_problem(256.0, 128, 1, 19.0, 10)  # 128 MiB of workspace
    assert cola.workspace_bytes(prob) > 64 << 20
    st = cola.ParticleState(prob)
    ptrs = (ctypes.c_void_p * 3)(*[st.p[d].data_ptr() for d in range(3)])
    s = _lib.lib().cola_pm_force_noalloc(ctypes.byref(prob), ctypes.byref(st.c), ptrs, None)
    assert s == -3  # COLA_ERR_WORKSPACE_TOO_SMALL
    assert float(st.p.abs().max()) == 0.0  # nothing was launched
