"""COLA particle-mesh step and 2LPT initial conditions on AMD MI355X (gfx950).

Method: Izard, Crocce & Fosalba, ICE-COLA (arXiv:1509.04685).  The computation lives in the
HIP library libcola.so (C ABI in include/cola.h); this package marshals torch tensors into it.
torch provides device memory and the HIP stream only.
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import ColaError, Cosmology, Problem, Particles  # noqa: F401

__all__ = ["Cosmology", "Problem", "ParticleState", "Workspace", "ic_2lpt", "pm_force", "step",
           "power_spectrum", "cic_density", "fft_r2c", "fft_c2r", "schedule_table",
           "linear_power", "workspace_bytes", "ColaError"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda_f32(t, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous device tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")


def make_cosmology(omega_m=0.25, omega_b=0.044, h=0.7, n_s=0.95, sigma_8=0.8):
    return Cosmology(omega_m, omega_b, h, n_s, sigma_8)


def make_problem(box, n_part, pm_factor, z_init, n_steps, a_final=1.0, n_real=1):
    return Problem(float(box), int(n_part), int(pm_factor), float(z_init), float(a_final),
                   int(n_steps), 0, int(n_real))


def workspace_bytes(prob, n_pk=0):
    return int(_lib.lib().cola_workspace_bytes(ctypes.byref(prob), int(n_pk)))


class Workspace:
    """Device workspace (a uint8 torch tensor) sized for a problem and P(k) mesh."""

    def __init__(self, prob, n_pk=0, device="cuda"):
        torch = _torch()
        nbytes = workspace_bytes(prob, n_pk)
        if nbytes == 0:
            raise ColaError(-1, "cola_workspace_bytes")
        self.tensor = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    @property
    def ptr(self):
        return ctypes.c_void_p(self.tensor.data_ptr())


class ParticleState:
    """Particle state of a batch: x, p, psi1, psi2 as (3, n_real * N_p^3) float32 device tensors."""

    def __init__(self, prob, device="cuda"):
        torch = _torch()
        n = prob.n_real * prob.n_part ** 3
        self.n = n
        self.x = torch.zeros((3, n), dtype=torch.float32, device=device)
        self.p = torch.zeros((3, n), dtype=torch.float32, device=device)
        self.psi1 = torch.zeros((3, n), dtype=torch.float32, device=device)
        self.psi2 = torch.zeros((3, n), dtype=torch.float32, device=device)
        self.c = Particles()
        for d in range(3):
            self.c.x[d] = self.x[d].data_ptr()
            self.c.p[d] = self.p[d].data_ptr()
            self.c.psi1[d] = self.psi1[d].data_ptr()
            self.c.psi2[d] = self.psi2[d].data_ptr()
        self.c.node = 0
        self.c.force_node = -1
        self.c.force_ws = None

    @property
    def node(self):
        return self.c.node

    def invalidate_force(self):
        self.c.force_node = -1


def ic_2lpt(prob, cosmo, seeds, state, ws):
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1))
    if seeds.size != prob.n_real:
        raise ValueError("need one seed per realization")
    arr = seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    _lib.check(_lib.lib().cola_ic_2lpt(ctypes.byref(prob), ctypes.byref(cosmo), arr,
                                       ctypes.byref(state.c), ws.ptr, ws.nbytes, _stream()),
               "cola_ic_2lpt")


def pm_force(prob, state, ws, acc=None):
    torch = _torch()
    if acc is None:
        acc = torch.empty((3, state.n), dtype=torch.float32, device=state.x.device)
    ptrs = (ctypes.c_void_p * 3)(*[acc[d].data_ptr() for d in range(3)])
    _lib.check(_lib.lib().cola_pm_force(ctypes.byref(prob), ctypes.byref(state.c), ptrs, ws.ptr,
                                        ws.nbytes, _stream()), "cola_pm_force")
    return acc


def step(prob, cosmo, state, j_end, ws):
    _lib.check(_lib.lib().cola_step(ctypes.byref(prob), ctypes.byref(cosmo), state.c.node, int(j_end),
                                    ctypes.byref(state.c), ws.ptr, ws.nbytes, _stream()),
               "cola_step")


def power_spectrum(prob, cosmo, state, a_out, n_pk, n_bins, ws, out=None):
    """Returns (k_mean, pk, n_modes), each (n_real, n_bins) float64 device tensors."""
    torch = _torch()
    if out is None:
        out = tuple(torch.empty((prob.n_real, n_bins), dtype=torch.float64, device=state.x.device)
                    for _ in range(3))
    km, pk, nm = out
    _lib.check(_lib.lib().cola_power_spectrum(ctypes.byref(prob), ctypes.byref(cosmo),
                                              ctypes.byref(state.c), float(a_out), int(n_pk),
                                              int(n_bins), _ptr(km), _ptr(pk), _ptr(nm), ws.ptr,
                                              ws.nbytes, _stream()), "cola_power_spectrum")
    return km, pk, nm


def cic_density(pos, n_mesh, box):
    """pos: (3, n) float32 device tensor of absolute positions -> (n_mesh,)*3 density contrast."""
    torch = _torch()
    _require_cuda_f32(pos, "pos")
    out = torch.empty((n_mesh, n_mesh, n_mesh), dtype=torch.float32, device=pos.device)
    ptrs = (ctypes.c_void_p * 3)(*[pos[d].data_ptr() for d in range(3)])
    _lib.check(_lib.lib().cola_cic_density(ptrs, pos.shape[1], int(n_mesh), float(box), _ptr(out), None, 0,
                                           _stream()), "cola_cic_density")
    return out


def _fft_ws(n, device):
    torch = _torch()
    nbytes = int(_lib.lib().cola_fft_workspace_bytes(int(n)))
    if nbytes == 0:
        raise ColaError(-2, "cola_fft_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def fft_r2c(x):
    """(n, n, n) float32 device tensor -> (n, n, n/2+1) complex64 (unnormalised forward)."""
    torch = _torch()
    _require_cuda_f32(x, "x")
    n = x.shape[0]
    out = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device=x.device)
    ws, nb = _fft_ws(n, x.device)
    _lib.check(_lib.lib().cola_fft_r2c(n, _ptr(x), _ptr(out), _ptr(ws), nb, _stream()), "cola_fft_r2c")
    return out


def fft_c2r(xk):
    """(n, n, n/2+1) complex64 device tensor -> (n, n, n) float32 (unnormalised inverse)."""
    torch = _torch()
    n = xk.shape[0]
    if xk.dtype != torch.complex64 or not xk.is_contiguous():
        raise ValueError("xk must be contiguous complex64")
    out = torch.empty((n, n, n), dtype=torch.float32, device=xk.device)
    ws, nb = _fft_ws(n, xk.device)
    _lib.check(_lib.lib().cola_fft_c2r(n, _ptr(xk), _ptr(out), _ptr(ws), nb, _stream()), "cola_fft_c2r")
    return out


def schedule_table(prob, cosmo):
    """Host-side float64 schedule: (n_steps, 6) array of a, D1, D2, K_out, K_in, Dr."""
    out = np.zeros((prob.n_steps, 6), dtype=np.float64)
    _lib.check(_lib.lib().cola_schedule_table(ctypes.byref(prob), ctypes.byref(cosmo),
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "cola_schedule_table")
    return out


def autotune(prob, ws, n_pk=0, state=None):
    """Pick the fastest FFT kernel shapes for this problem's sizes (destroys ws contents)."""
    buf = ctypes.create_string_buffer(4096)
    _lib.check(_lib.lib().cola_autotune(ctypes.byref(prob), int(n_pk), ws.ptr, ws.nbytes, _stream(), buf,
                                        len(buf)), "cola_autotune")
    if state is not None:
        state.invalidate_force()
    return buf.value.decode()


class Ensemble:
    """Shape classes of seeded realizations run together (cola_ensemble_run).

    classes: list of dicts with keys prob, seeds, a_out (tuple), n_pk, n_bins.  Allocates the
    particle states, workspaces and P(k) outputs of every class.
    """

    def __init__(self, classes, cosmo, device="cuda"):
        torch = _torch()
        self.cosmo = cosmo
        self.items = []
        arr = (_lib.EnsembleClass * len(classes))()
        for i, c in enumerate(classes):
            prob = c["prob"]
            st = ParticleState(prob, device)
            ws = Workspace(prob, n_pk=c["n_pk"], device=device)
            seeds = np.ascontiguousarray(np.asarray(c["seeds"], dtype=np.uint64))
            a_out = np.ascontiguousarray(np.asarray(c["a_out"], dtype=np.float64))
            n_out, n_bins = len(a_out), int(c["n_bins"])
            out = [torch.zeros((n_out, prob.n_real, n_bins), dtype=torch.float64, device=device)
                   for _ in range(3)]
            e = arr[i]
            e.prob = prob
            e.seeds = seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            e.parts = ctypes.pointer(st.c)
            e.ws = ws.ptr
            e.ws_bytes = ws.nbytes
            e.n_out = n_out
            e.a_out = a_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            e.n_pk = int(c["n_pk"])
            e.n_bins = n_bins
            e.k_mean, e.pk, e.n_modes = (_ptr(t) for t in out)
            self.items.append(dict(prob=prob, state=st, ws=ws, seeds=seeds, a_out=a_out, out=out))
        self.arr = arr

    def autotune(self):
        return "".join(autotune(it["prob"], it["ws"], n_pk=int(self.arr[i].n_pk), state=it["state"])
                       for i, it in enumerate(self.items))

    def run(self, graph=True):
        _lib.check(_lib.lib().cola_ensemble_run(len(self.items), self.arr, ctypes.byref(self.cosmo),
                                                1 if graph else 0, _stream()), "cola_ensemble_run")


def ensemble_release():
    _lib.check(_lib.lib().cola_ensemble_release(), "cola_ensemble_release")


def profiler_enable(on=True):
    _lib.check(_lib.lib().cola_profiler_enable(1 if on else 0), "cola_profiler_enable")


def profiler_read():
    """{kernel kind: (total ms, launches)} for the launches since the last read/enable."""
    n = int(_lib.lib().cola_profiler_num_kinds())
    ms = np.zeros(n, dtype=np.float64)
    cnt = np.zeros(n, dtype=np.int64)
    _lib.check(_lib.lib().cola_profiler_read(n, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               "cola_profiler_read")
    return {_lib.lib().cola_profiler_kind_name(i).decode(): (float(ms[i]), int(cnt[i]))
            for i in range(n) if cnt[i] > 0}


def copy(src, dst):
    """Device copy with the library's streaming kernel (counter yardstick)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    _lib.check(_lib.lib().cola_copy(_ptr(src), _ptr(dst), nbytes, _stream()), "cola_copy")


def linear_power(cosmo, k):
    return float(_lib.lib().cola_linear_power(ctypes.byref(cosmo), float(k)))
