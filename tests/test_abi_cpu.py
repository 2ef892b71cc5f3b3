"""The C-ABI library on the host: it loads, exports every symbol the header declares, rejects
bad arguments before any launch, and its float64 host schedule matches the oracle.

No test here launches device work."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cola.h")

cola = pytest.importorskip("paper_1509_04685_amd")
from paper_1509_04685_amd import _lib  # noqa: E402
from oracle import cola as ocola, cosmology as ocosmo  # noqa: E402

LIB = _lib.lib()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cola_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(LIB, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_version_and_status_strings():
    assert b"gfx950" in LIB.cola_version()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert LIB.cola_status_string(s)


def prob(**kw):
    d = dict(box=256.0, n_part=32, pm_factor=3, z_init=19.0, n_steps=10, n_real=1)
    d.update(kw)
    return cola.make_problem(**d)


COSMO = cola.make_cosmology()


@pytest.mark.parametrize("bad", [dict(n_part=35), dict(pm_factor=5), dict(n_part=1),
                                 dict(n_part=770, pm_factor=1), dict(n_steps=1), dict(box=-1.0),
                                 dict(z_init=-1.5), dict(n_real=0), dict(pm_factor=0)])
def test_workspace_bytes_rejects_bad_problems(bad):
    assert cola.workspace_bytes(prob(**bad)) == 0


def test_workspace_bytes_scales():
    a = cola.workspace_bytes(prob())
    b = cola.workspace_bytes(prob(n_real=4))
    c = cola.workspace_bytes(prob(), n_pk=96)
    assert a > 0 and b > 3 * a and c > a
    assert cola.workspace_bytes(prob(), n_pk=97) == 0


def test_entry_points_validate_before_launch():
    p = prob()
    st = cola.Particles()
    seeds = (ctypes.c_uint64 * 1)(1)
    # NULL particle pointers
    assert LIB.cola_ic_2lpt(ctypes.byref(p), ctypes.byref(COSMO), seeds, ctypes.byref(st), None, 0, None) == -1
    fake = ctypes.c_void_p(0x1000)
    for d in range(3):
        st.x[d] = st.p[d] = st.psi1[d] = st.psi2[d] = 0x1000
    # workspace missing, then too small
    assert LIB.cola_ic_2lpt(ctypes.byref(p), ctypes.byref(COSMO), seeds, ctypes.byref(st), None, 0, None) == -1
    assert LIB.cola_ic_2lpt(ctypes.byref(p), ctypes.byref(COSMO), seeds, ctypes.byref(st), fake, 16, None) == -3
    # unsupported size: 770 = 2 5 7 11
    p2 = prob(n_part=770, pm_factor=1)
    assert LIB.cola_ic_2lpt(ctypes.byref(p2), ctypes.byref(COSMO), seeds, ctypes.byref(st), fake, 1 << 40, None) == -2
    # a_init >= a_final
    p3 = prob(z_init=0.0)
    assert LIB.cola_step(ctypes.byref(p3), ctypes.byref(COSMO), 0, 1, ctypes.byref(st), fake, 1 << 40, None) == -1
    # node range
    st.node = 2
    assert LIB.cola_step(ctypes.byref(p), ctypes.byref(COSMO), 0, 3, ctypes.byref(st), fake, 1 << 40, None) == -5
    assert LIB.cola_step(ctypes.byref(p), ctypes.byref(COSMO), 2, 10, ctypes.byref(st), fake, 1 << 40, None) == -5
    # bad cosmology
    bad = cola.make_cosmology(omega_m=0.0)
    st.node = 0
    assert LIB.cola_step(ctypes.byref(p), ctypes.byref(bad), 0, 1, ctypes.byref(st), fake, 1 << 40, None) == -1
    # P(k): a_out outside the current interval, bad n_pk
    out = ctypes.c_void_p(0x2000)
    assert LIB.cola_power_spectrum(ctypes.byref(p), ctypes.byref(COSMO), ctypes.byref(st), 0.9, 96, 48,
                                   out, out, out, fake, 1 << 40, None) == -5
    assert LIB.cola_power_spectrum(ctypes.byref(p), ctypes.byref(COSMO), ctypes.byref(st), 0.05, 100, 48,
                                   out, out, out, fake, 1 << 40, None) == -2
    assert LIB.cola_fft_r2c(14, fake, fake, fake, 1 << 30, None) == -2
    assert LIB.cola_fft_r2c(16, fake, fake, fake, 8, None) == -3


def test_host_schedule_matches_oracle():
    for n_steps, z_i in ((10, 19.0), (40, 19.0), (40, 39.0)):
        p = prob(n_steps=n_steps, z_init=z_i)
        tab = cola.schedule_table(p, COSMO)
        op = ocola.Problem(256.0, 32, 3, z_i, n_steps)
        sch = ocola.Schedule(op, ocosmo.Cosmology())
        assert np.allclose(tab[:, 0], sch.a, rtol=1e-14)
        assert np.allclose(tab[:, 1], sch.d1, rtol=1e-10)
        assert np.allclose(tab[:, 2], sch.d2, rtol=1e-10)
        assert np.allclose(tab[:-1, 3], sch.k_out, rtol=1e-11)
        assert np.allclose(tab[:-1, 4], sch.k_in, rtol=1e-11)
        assert np.allclose(tab[:-1, 5], sch.drift, rtol=1e-11)


def test_host_linear_power_matches_oracle():
    c = ocosmo.Cosmology()
    amp = ocosmo.linear_amplitude(c)
    for k in (1e-3, 0.01, 0.1, 0.5, 1.0, 3.0):
        assert cola.linear_power(COSMO, k) == pytest.approx(float(ocosmo.linear_power(k, c, amp)), rel=1e-8)


def test_host_schedule_samplings_match_oracle():
    """Eq. 3 with f = ln a and f = a^p (Sec. 4.2: 0.5 and 0.8), 40 nodes from z_i = 39."""
    for sampling, power in (("log", None), ("power", 0.5), ("power", 0.8)):
        p = cola.make_problem(256.0, 32, 3, 39.0, 40, sampling=sampling, sampling_power=power or 1.0)
        tab = cola.schedule_table(p, COSMO)
        op = ocola.Problem(256.0, 32, 3, 39.0, 40, sampling=sampling, sampling_power=power)
        sch = ocola.Schedule(op, ocosmo.Cosmology())
        assert np.allclose(tab[:, 0], sch.a, rtol=1e-13)
        assert np.allclose(tab[:, 1], sch.d1, rtol=1e-10)
        assert np.allclose(tab[:-1, 3], sch.k_out, rtol=1e-11)
        assert np.allclose(tab[:-1, 5], sch.drift, rtol=1e-11)


def test_problem_rejects_bad_sampling_and_frame():
    for kw in (dict(sampling=3), dict(sampling=2, sampling_power=0.0), dict(sampling=2, sampling_power=float("nan")),
               dict(frame=2)):
        p = cola.make_problem(256.0, 32, 3, 19.0, 10)
        for k, v in kw.items():
            setattr(p, k, v)
        assert LIB.cola_workspace_bytes(ctypes.byref(p), 0) == 0


def test_fof_and_multipole_entry_points_validate_before_launch():
    fake = ctypes.c_void_p(0x1000)
    P3 = ctypes.c_void_p * 3
    pos = P3(0x1000, 0x2000, 0x3000)
    assert LIB.cola_fof_workspace_bytes(0, 100.0, 1.0) == 0
    assert LIB.cola_fof_workspace_bytes(1000, -1.0, 1.0) == 0
    nb = LIB.cola_fof_workspace_bytes(1000, 100.0, 1.0)
    assert nb > 1000 * 20
    # linking length of half the box or more, NULL outputs, small workspace
    assert LIB.cola_fof(pos, 1000, 100.0, 50.0, fake, fake, fake, nb, None) == -1
    assert LIB.cola_fof(pos, 1000, 100.0, 1.0, None, fake, fake, nb, None) == -1
    assert LIB.cola_fof(pos, 1000, 100.0, 1.0, fake, fake, fake, 16, None) == -3
    # catalogue: room for fewer haloes than n / n_min
    com = P3(0x1000, 0x1000, 0x1000)
    assert LIB.cola_fof_catalogue(pos, 1000, 100.0, fake, fake, 100, 1.0, 9, fake, fake, fake, com, fake, fake,
                                  nb, None) == -1
    # mass histogram: edges not increasing, too many bins, non-positive particle mass
    edges = (ctypes.c_double * 3)(14.0, 13.0, 15.0)
    assert LIB.cola_fof_mass_histogram(fake, 1000, 101, 1e12, edges, 2, fake, None) == -1
    edges = (ctypes.c_double * 66)(*[12.0 + 0.1 * i for i in range(66)])
    assert LIB.cola_fof_mass_histogram(fake, 1000, 101, 1e12, edges, 65, fake, None) == -1
    assert LIB.cola_fof_mass_histogram(fake, 1000, 101, 0.0, edges, 3, fake, None) == -1
    # multipoles: line of sight out of range, output off the state's node
    p = prob()
    st = cola.Particles()
    for d in range(3):
        st.x[d] = st.p[d] = st.psi1[d] = st.psi2[d] = 0x1000
    st.node = 2
    a2 = float(cola.schedule_table(p, COSMO)[2, 0])
    args = (96, 48, fake, fake, fake, fake, fake, fake, 1 << 40, None)
    assert LIB.cola_power_multipoles(ctypes.byref(p), ctypes.byref(COSMO), ctypes.byref(st), a2, 3, 1, *args) == -1
    assert LIB.cola_power_multipoles(ctypes.byref(p), ctypes.byref(COSMO), ctypes.byref(st), a2 + 0.01, 2, 1,
                                     *args) == -5


def test_particle_mass_matches_oracle():
    for box, n in ((768.0, 256), (1536.0, 512), (300.0, 96)):
        got = cola.particle_mass(COSMO, box, n)
        ref = ocosmo.particle_mass(ocosmo.Cosmology(), box, n)
        assert got == pytest.approx(ref, rel=1e-14)
    assert cola.particle_mass(COSMO, -1.0, 8) == 0.0


def test_nonfinite_arguments_return_nonfinite():
    """COLA_ERR_NONFINITE (-6): a NaN or infinite floating-point argument is found by the host
    checks, before anything is launched (no device is touched; every pointer here is fake)."""
    nan, inf = float("nan"), float("inf")
    fake = ctypes.c_void_p(0x1000)
    st = cola.Particles()
    for d in range(3):
        st.x[d] = st.p[d] = st.psi1[d] = st.psi2[d] = 0x1000
    seeds = (ctypes.c_uint64 * 1)(1)
    for kw in (dict(box=nan), dict(z_init=inf), dict(a_final=nan)):
        p = prob()
        for k, v in kw.items():
            setattr(p, k, v)
        assert LIB.cola_ic_2lpt(ctypes.byref(p), ctypes.byref(COSMO), seeds, ctypes.byref(st), fake, 1 << 40,
                                None) == -6, kw
        assert LIB.cola_step(ctypes.byref(p), ctypes.byref(COSMO), 0, 1, ctypes.byref(st), fake, 1 << 40, None) == -6
    p = cola.make_problem(256.0, 32, 3, 19.0, 10, sampling="power", sampling_power=2.0)
    p.sampling_power = nan
    assert LIB.cola_step(ctypes.byref(p), ctypes.byref(COSMO), 0, 1, ctypes.byref(st), fake, 1 << 40, None) == -6
    for bad in (cola.make_cosmology(omega_m=nan), cola.make_cosmology(sigma_8=inf), cola.make_cosmology(n_s=nan)):
        assert LIB.cola_step(ctypes.byref(prob()), ctypes.byref(bad), 0, 1, ctypes.byref(st), fake, 1 << 40,
                             None) == -6
    out = ctypes.c_void_p(0x2000)
    assert LIB.cola_power_spectrum(ctypes.byref(prob()), ctypes.byref(COSMO), ctypes.byref(st), nan, 96, 48,
                                   out, out, out, fake, 1 << 40, None) == -6
    P3 = ctypes.c_void_p * 3
    pos = P3(0x1000, 0x2000, 0x3000)
    assert LIB.cola_cic_density(pos, 1000, 32, inf, fake, fake, 1 << 30, None) == -6
    assert LIB.cola_fof(pos, 1000, 100.0, nan, fake, fake, fake, 1 << 30, None) == -6
    edges = (ctypes.c_double * 3)(13.0, nan, 15.0)
    assert LIB.cola_fof_mass_histogram(fake, 1000, 101, 1e12, edges, 2, fake, None) == -6
    assert LIB.cola_mesh_force(32, nan, fake, P3(0x1000, 0x1000, 0x1000), fake, 1 << 30, None) == -6
    # the network's scales: a NaN output scale
    net = cola._lib.LcNet()
    net.channels = 16
    net.params = 0x1000
    net.packed = 0x1000
    net.out_scale = nan
    p1 = cola.make_problem(64.0, 16, 1, 19.0, 5)
    assert LIB.cola_step_lc(ctypes.byref(p1), ctypes.byref(COSMO), 0, 1, ctypes.byref(st), ctypes.byref(net), fake,
                            1 << 40, fake, 1 << 40, None) == -6
    assert LIB.cola_status_string(-6)


def test_fft_set_shape_fused_force_pass_host_checks():
    """The fused z pass of the force (z_c2r3: three thread groups per block, one per force
    component, sharing one LDS area) is admitted up to 1024 threads and 150 KB of LDS per block
    (host only: nothing is launched)."""
    f = LIB.cola_fft_set_shape
    assert f(768, b"z_c2r3", 24, 16, 1) == 0    # 3 x 16 x 16 threads, 3 x 16 x 385 x 8 B = 148 KB
    assert f(768, b"z_c2r3", 24, 32, 1) == -1   # 296 KB of LDS
    assert f(768, b"z_c2r3", 12, 16, 1) == -1   # 1536 threads
    assert f(1536, b"z_c2r3", 24, 8, 1) == 0
    assert f(1536, b"z_c2r3", 24, 16, 1) == -1
    assert f(768, b"z_c2r3", 24, 16, 2) == -1   # no split-exchange plan for z passes
    assert f(768, b"z_c2r", 12, 32, 0) == -1    # the single z pass keeps its 512-thread bound
    assert f(768, b"z_c2r3", 12, 8, 1) == 0     # restore the usual shape


def test_fft_set_shape_split_plans_host_checks():
    """Split-exchange plans are offered for the x-column kinds where compiled, nowhere else (host
    only: nothing is launched)."""
    f = LIB.cola_fft_set_shape
    assert f(768, b"x_green", 24, 16, 2) == 0
    assert f(1536, b"x_green", 24, 8, 2) == 0
    assert f(1536, b"x_green", 12, 8, 2) == 0   # 1024-thread blocks: split plans only
    assert f(1536, b"x_green", 12, 8, 1) == -1
    assert f(768, b"rows_y", 24, 8, 2) == -1
    assert f(512, b"x_green", 16, 8, 2) == -1
    assert f(768, b"x_green", 24, 16, 3) == -1
    assert f(768, b"x_green", 24, 8, 1) == 0  # restore a plain static plan
    assert f(768, b"x_green", 24, 16, 1) == 0
    assert f(1536, b"x_green", 24, 4, 1) == 0
