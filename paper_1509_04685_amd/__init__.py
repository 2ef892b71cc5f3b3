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
           "power_spectrum", "power_spectrum_jing", "cic_density", "fft_r2c", "fft_c2r", "schedule_table",
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


SAMPLINGS = {"linear": 0, "log": 1, "power": 2}
FRAMES = {"cola": 0, "pm": 1}


def make_problem(box, n_part, pm_factor, z_init, n_steps, a_final=1.0, n_real=1, sampling="linear",
                 sampling_power=1.0, frame="cola"):
    """Run parameters (Table 1).  sampling: "linear" (f = a), "log" (f = ln a) or "power"
    (f = a^sampling_power) node spacing of Eq. 3; frame: "cola" (2LPT frame, Eq. 1-2) or "pm"
    (plain leapfrog, the LPT frame switched off)."""
    return Problem(float(box), int(n_part), int(pm_factor), float(z_init), float(a_final),
                   int(n_steps), SAMPLINGS[sampling], int(n_real), FRAMES[frame], float(sampling_power))


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


def power_multipoles(prob, cosmo, state, a_out, n_pk, n_bins, ws, los=2, redshift_space=True):
    """Multipoles about axis `los` at the state's node: (k_mean, p0, p2, p4, n_modes), each
    (n_real, n_bins) float64 device tensors; redshift_space maps positions with Eq. 5 first."""
    torch = _torch()
    out = tuple(torch.empty((prob.n_real, n_bins), dtype=torch.float64, device=state.x.device) for _ in range(5))
    _lib.check(_lib.lib().cola_power_multipoles(ctypes.byref(prob), ctypes.byref(cosmo), ctypes.byref(state.c),
                                                float(a_out), int(los), 1 if redshift_space else 0, int(n_pk),
                                                int(n_bins), *[_ptr(t) for t in out], ws.ptr, ws.nbytes, _stream()),
               "cola_power_multipoles")
    return out


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


def power_spectrum_jing(prob, cosmo, state, a_out, n_pk, n_bins, ws, iterations=4, out=None):
    """power_spectrum with the Jing (2005) aliasing correction: (k_mean, pk, n_modes)."""
    torch = _torch()
    if out is None:
        out = tuple(torch.empty((prob.n_real, n_bins), dtype=torch.float64, device=state.x.device)
                    for _ in range(3))
    km, pk, nm = out
    _lib.check(_lib.lib().cola_power_spectrum_jing(ctypes.byref(prob), ctypes.byref(cosmo),
                                                   ctypes.byref(state.c), float(a_out), int(n_pk),
                                                   int(n_bins), int(iterations), _ptr(km), _ptr(pk),
                                                   _ptr(nm), ws.ptr, ws.nbytes, _stream()),
               "cola_power_spectrum_jing")
    return km, pk, nm


def cic_density(pos, n_mesh, box, ws=None):
    """pos: (3, n) float32 device tensor of absolute positions -> (n_mesh,)*3 density contrast, by the
    step's sorted tile deposit."""
    torch = _torch()
    _require_cuda_f32(pos, "pos")
    n = int(pos.shape[1])
    nb = int(_lib.lib().cola_cic_workspace_bytes(n, int(n_mesh)))
    if nb == 0:
        raise ColaError(-1, "cola_cic_workspace_bytes")
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=pos.device)
    out = torch.empty((n_mesh, n_mesh, n_mesh), dtype=torch.float32, device=pos.device)
    ptrs = (ctypes.c_void_p * 3)(*[pos[d].data_ptr() for d in range(3)])
    _lib.check(_lib.lib().cola_cic_density(ptrs, n, int(n_mesh), float(box), _ptr(out), _ptr(ws), ws.numel(),
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

    classes: list of dicts with keys prob, seeds, a_out (tuple), n_pk, n_bins, and optionally net
    (an LcNet: the class runs the corrected steps).  Allocates the particle states, workspaces and
    P(k) outputs of every class.
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
            net = c.get("net")
            lws = None
            if net is not None:
                lws = lc_workspace(prob.n_part * prob.pm_factor, net.channels, prob.n_real, device=device)
                e.net = ctypes.cast(ctypes.pointer(net.c), ctypes.c_void_p)
                e.lc_ws = _ptr(lws)
                e.lc_ws_bytes = lws.numel()
            self.items.append(dict(prob=prob, state=st, ws=ws, seeds=seeds, a_out=a_out, out=out, net=net,
                                   lc_ws=lws))
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


def profiler_read_groups():
    """{(kernel kind, size tag): (total ms, launches)}; the tag is the mesh side for FFT passes."""
    cap = 512
    kinds = np.zeros(cap, dtype=np.int32)
    tags = np.zeros(cap, dtype=np.int64)
    ms = np.zeros(cap, dtype=np.float64)
    cnt = np.zeros(cap, dtype=np.int64)
    n = _lib.lib().cola_profiler_read_groups(cap, kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             tags.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                             ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if n < 0:
        raise ColaError(n, "cola_profiler_read_groups")
    name = _lib.lib().cola_profiler_kind_name
    return {(name(int(kinds[i])).decode(), int(tags[i])): (float(ms[i]), int(cnt[i])) for i in range(n)}


def copy(src, dst):
    """Device copy with the library's streaming kernel (counter yardstick)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    _lib.check(_lib.lib().cola_copy(_ptr(src), _ptr(dst), nbytes, _stream()), "cola_copy")


def linear_power(cosmo, k):
    return float(_lib.lib().cola_linear_power(ctypes.byref(cosmo), float(k)))


# ---------------------------------------------------------------- learned force correction

def _ptrs3(ts):
    return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])


def lc_param_count(channels):
    return int(_lib.lib().cola_lc_param_count(int(channels)))


def lc_init_params(channels, seed=0):
    """He-normal initial weights (zero biases, small output layer) as a flat float32 host array
    in the library's order w1 (C,4,27) b1 w2 (C,C,27) b2 w3 (3,C) b3."""
    rng = np.random.default_rng(seed)
    c = int(channels)
    parts = [rng.normal(0.0, np.sqrt(2.0 / 108.0), 108 * c), np.zeros(c),
             rng.normal(0.0, np.sqrt(2.0 / (27.0 * c)), 27 * c * c), np.zeros(c),
             rng.normal(0.0, np.sqrt(1.0 / c), 3 * c) * 0.1, np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


class LcNet:
    """The correction network on the device: FP32 parameters (and, for training, gradients and
    Adam moments) plus the BF16 weight copies the convolutions read."""

    def __init__(self, channels=16, params=None, in_scale=(1.0, 1.0, 1.0, 1.0), out_scale=1.0,
                 training=True, device="cuda"):
        torch = _torch()
        count = lc_param_count(channels)
        if count == 0:
            raise ColaError(-1, "cola_lc_param_count")
        self.channels = int(channels)
        self.params = torch.zeros(count, dtype=torch.float32, device=device)
        self.grads = torch.zeros(count, dtype=torch.float32, device=device) if training else None
        self.adam_m = torch.zeros(count, dtype=torch.float32, device=device) if training else None
        self.adam_v = torch.zeros(count, dtype=torch.float32, device=device) if training else None
        self.packed = torch.empty(int(_lib.lib().cola_lc_packed_bytes(self.channels)), dtype=torch.uint8,
                                  device=device)
        self.c = _lib.LcNet()
        self.c.channels = self.channels
        self.c.params = self.params.data_ptr()
        self.c.grads = self.grads.data_ptr() if training else None
        self.c.adam_m = self.adam_m.data_ptr() if training else None
        self.c.adam_v = self.adam_v.data_ptr() if training else None
        self.c.packed = self.packed.data_ptr()
        self.set_scales(in_scale, out_scale)
        self.set_params(lc_init_params(channels) if params is None else params)
        self.step_count = 0

    def set_scales(self, in_scale, out_scale, out_scale_slope=None, out_band=None):
        for i in range(4):
            self.c.in_scale[i] = float(in_scale[i])
        self.c.out_scale = float(out_scale)
        if out_scale_slope is not None:
            self.c.out_scale_slope = float(out_scale_slope)
        if out_band is not None:
            self.c.out_band = float(out_band)

    @property
    def out_scale_slope(self):
        return float(self.c.out_scale_slope)

    @property
    def out_band(self):
        return float(self.c.out_band)

    def set_schedule(self, knot_a=None, knot_v=None):
        """Piecewise-linear multiplier of the step's output scale over a (None: none)."""
        if knot_a is None:
            self.c.n_knots = 0
            return
        if len(knot_a) != len(knot_v) or not 2 <= len(knot_a) <= 8:
            raise ValueError("2 to 8 knots with one value each")
        self.c.n_knots = len(knot_a)
        for i, (a, v) in enumerate(zip(knot_a, knot_v)):
            self.c.knot_a[i] = float(a)
            self.c.knot_v[i] = float(v)

    def set_green_filter(self, u=None, rows=None):
        """Radial transfer T(u, a) of the corrected step's Green's function (see cola_lc_net): u the
        knots in |k| / k_Nyquist, rows[i][j] = T at the schedule's knot_a[i] and u[j] (one row without
        a schedule).  None: no filter."""
        if u is None:
            self.c.n_gknots = 0
            return
        if not 2 <= len(u) <= 10 or not 1 <= len(rows) <= 8 or any(len(r) != len(u) for r in rows):
            raise ValueError("2 to 10 knots in u and 1 to 8 rows of as many values")
        self.c.n_gknots = len(u)
        for j, v in enumerate(u):
            self.c.gknot_u[j] = float(v)
        for i in range(8):
            src = rows[min(i, len(rows) - 1)]
            for j in range(10):
                self.c.gknot_t[i][j] = float(src[j]) if j < len(u) else 0.0

    @property
    def green_filter(self):
        n = int(self.c.n_gknots)
        if not n:
            return None
        nr = max(1, int(self.c.n_knots))
        return ([float(self.c.gknot_u[j]) for j in range(n)],
                [[float(self.c.gknot_t[i][j]) for j in range(n)] for i in range(nr)])

    @property
    def schedule(self):
        n = int(self.c.n_knots)
        return ([float(self.c.knot_a[i]) for i in range(n)], [float(self.c.knot_v[i]) for i in range(n)]) if n else None

    @property
    def in_scale(self):
        return tuple(float(self.c.in_scale[i]) for i in range(4))

    @property
    def out_scale(self):
        return float(self.c.out_scale)

    def set_params(self, flat):
        torch = _torch()
        flat = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(-1))
        if flat.size != self.params.numel():
            raise ValueError("wrong parameter count")
        self.params.copy_(torch.from_numpy(flat))
        self.pack()

    def get_params(self):
        return self.params.cpu().numpy().copy()

    def pack(self):
        _lib.check(_lib.lib().cola_lc_pack(ctypes.byref(self.c), _stream()), "cola_lc_pack")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        _lib.check(_lib.lib().cola_lc_adam(ctypes.byref(self.c), self.step_count, float(lr), float(beta1),
                                           float(beta2), float(eps), _stream()), "cola_lc_adam")


def lc_workspace(n_mesh, channels, n_real=1, training=False, device="cuda"):
    torch = _torch()
    nbytes = int(_lib.lib().cola_lc_workspace_bytes(int(n_mesh), int(channels), int(n_real), 1 if training else 0))
    if nbytes == 0:
        raise ColaError(-2, "cola_lc_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def lc_forward(net, delta, g, ws, df=None, accumulate=False, training=False):
    """dF (3, n, n, n) of the network for delta (n, n, n) and g (3, n, n, n) device float32."""
    torch = _torch()
    _require_cuda_f32(delta, "delta")
    _require_cuda_f32(g, "g")
    n = delta.shape[0]
    if df is None:
        df = torch.empty((3, n, n, n), dtype=torch.float32, device=delta.device)
    _lib.check(_lib.lib().cola_lc_forward(ctypes.byref(net.c), n, _ptr(delta), _ptrs3(g), _ptrs3(df),
                                          1 if accumulate else 0, 1 if training else 0, _ptr(ws), ws.numel(),
                                          _stream()), "cola_lc_forward")
    return df


def lc_backward(net, d_df, ws):
    _require_cuda_f32(d_df, "d_df")
    n = d_df.shape[-1]
    _lib.check(_lib.lib().cola_lc_backward(ctypes.byref(net.c), n, _ptr(d_df), _ptr(ws), ws.numel(), _stream()),
               "cola_lc_backward")


def lc_loss(pos, box, df, g1, g3, stats=None, d_df=None):
    """(stats, d_df): stats = [L, denominator] float64 device tensor, d_df = dL/d(dF) (3, n, n, n)."""
    torch = _torch()
    n = df.shape[-1]
    if stats is None:
        stats = torch.empty(2, dtype=torch.float64, device=df.device)
    if d_df is None:
        d_df = torch.empty((3, n, n, n), dtype=torch.float32, device=df.device)
    _lib.check(_lib.lib().cola_lc_loss(n, float(box), _ptrs3(pos), pos.shape[1], _ptrs3(df), _ptrs3(g1),
                                       _ptrs3(g3), _ptr(stats), _ptr(d_df), _stream()), "cola_lc_loss")
    return stats, d_df


def step_lc(prob, cosmo, state, j_end, net, lc_ws, ws):
    _lib.check(_lib.lib().cola_step_lc(ctypes.byref(prob), ctypes.byref(cosmo), state.c.node, int(j_end),
                                       ctypes.byref(state.c), ctypes.byref(net.c), _ptr(lc_ws), lc_ws.numel(),
                                       ws.ptr, ws.nbytes, _stream()), "cola_step_lc")


def pm_force_lc(prob, state, net, lc_ws, ws, a=1.0, acc=None):
    """Corrected acceleration (3, n) of the state's positions: the step's mesh force plus the
    network's dF with the output scale of scale factor a."""
    torch = _torch()
    if acc is None:
        acc = torch.empty((3, state.n), dtype=torch.float32, device=state.x.device)
    _lib.check(_lib.lib().cola_pm_force_lc(ctypes.byref(prob), ctypes.byref(state.c), ctypes.byref(net.c), float(a),
                                           _ptr(lc_ws), lc_ws.numel(), _ptrs3(acc), ws.ptr, ws.nbytes, _stream()),
               "cola_pm_force_lc")
    return acc


def mesh_force(delta, box, ws=None, g=None):
    """Force meshes g (3, n, n, n) of a density-contrast mesh delta (n, n, n) float32 on the device."""
    torch = _torch()
    _require_cuda_f32(delta, "delta")
    n = int(delta.shape[0])
    nb = int(_lib.lib().cola_pm_fields_workspace_bytes(n))
    if nb == 0:
        raise ColaError(-2, "cola_pm_fields_workspace_bytes")
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=delta.device)
    if g is None:
        g = torch.empty((3, n, n, n), dtype=torch.float32, device=delta.device)
    _lib.check(_lib.lib().cola_mesh_force(n, float(box), _ptr(delta), _ptrs3(g), _ptr(ws), ws.numel(), _stream()),
               "cola_mesh_force")
    return g


def fft_set_shape(n, kind, values_per_thread, width, use_static=True, split=False):
    """Pin one FFT pass kind's kernel shape at mesh side n (see cola_fft_set_shape); split: the
    compile-time plan with real/imaginary LDS exchanges (x-column kinds)."""
    mode = 2 if split else (1 if use_static else 0)
    _lib.check(_lib.lib().cola_fft_set_shape(int(n), kind.encode(), int(values_per_thread), int(width), mode),
               "cola_fft_set_shape")


def pm_fields(pos, n_mesh, box, delta=True, g=True, acc=True, ws=None):
    """Mesh fields of absolute positions pos (3, n): dict with 'delta' (n_mesh^3), 'g' (3, n_mesh^3)
    and 'acc' (3, n) as requested."""
    torch = _torch()
    _require_cuda_f32(pos, "pos")
    dev = pos.device
    n = int(n_mesh)
    nb = int(_lib.lib().cola_pm_fields_workspace_bytes(n))
    if nb == 0:
        raise ColaError(-2, "cola_pm_fields_workspace_bytes")
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = {}
    if delta is True:
        delta = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    if g is True:
        g = torch.empty((3, n, n, n), dtype=torch.float32, device=dev)
    if acc is True:
        acc = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=dev)
    dp = _ptr(delta) if delta is not None and delta is not False else None
    gp = _ptrs3(g) if g is not None and g is not False else None
    ap = _ptrs3(acc) if acc is not None and acc is not False else None
    _lib.check(_lib.lib().cola_pm_fields(n, float(box), _ptrs3(pos), pos.shape[1], dp, gp, ap, _ptr(ws), ws.numel(),
                                         _stream()), "cola_pm_fields")
    if dp is not None:
        out["delta"] = delta
    if gp is not None:
        out["g"] = g
    if ap is not None:
        out["acc"] = acc
    return out


def positions(prob, state, out=None):
    """Absolute positions (3, n_real * N_p^3) of a state, wrapped into [0, box)."""
    torch = _torch()
    if out is None:
        out = torch.empty((3, state.n), dtype=torch.float32, device=state.x.device)
    _lib.check(_lib.lib().cola_positions(ctypes.byref(prob), ctypes.byref(state.c), _ptrs3(out), _stream()),
               "cola_positions")
    return out


def mfma_selftest(a_bits, b_bits):
    """a_bits (16, 32), b_bits (32, 16): int16 device tensors of BF16 bit patterns -> D (16, 16) float32."""
    torch = _torch()
    d = torch.empty((16, 16), dtype=torch.float32, device=a_bits.device)
    _lib.check(_lib.lib().cola_mfma_selftest(_ptr(a_bits), _ptr(b_bits), _ptr(d), _stream()),
               "cola_mfma_selftest")
    return d


# ---------------------------------------------------------------- friends-of-friends haloes

def linking_length(box, n_part, b=0.2):
    """b times the mean inter-particle separation box / N_p (Sec. 2.1)."""
    return b * float(box) / int(n_part)


def particle_mass(cosmo, box, n_part):
    return float(_lib.lib().cola_particle_mass(ctypes.byref(cosmo), float(box), int(n_part)))


def fof_workspace(n, box, link, device="cuda"):
    torch = _torch()
    nb = int(_lib.lib().cola_fof_workspace_bytes(int(n), float(box), float(link)))
    if nb == 0:
        raise ColaError(-1, "cola_fof_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def fof(pos, box, link, ws=None):
    """Friends-of-friends groups of positions pos (3, n) float32: (group, group_size) int32 (n,)
    device tensors; group[i] = smallest index in i's group, group_size[r] = members at a label r."""
    torch = _torch()
    _require_cuda_f32(pos, "pos")
    n = int(pos.shape[1])
    if ws is None:
        ws = fof_workspace(n, box, link, pos.device)
    group = torch.empty(n, dtype=torch.int32, device=pos.device)
    size = torch.empty(n, dtype=torch.int32, device=pos.device)
    _lib.check(_lib.lib().cola_fof(_ptrs3(pos), n, float(box), float(link), _ptr(group), _ptr(size), _ptr(ws),
                                   ws.numel(), _stream()), "cola_fof")
    return group, size


def fof_catalogue(pos, box, group, size, n_min, m_p, ws):
    """Haloes with at least n_min members, by label: dict of device tensors root, n (int32), mass
    and com (3, n_halo) (float64)."""
    torch = _torch()
    _require_cuda_f32(pos, "pos")
    n = int(pos.shape[1])
    cap = max(1, n // int(n_min))
    dev = pos.device
    root = torch.empty(cap, dtype=torch.int32, device=dev)
    cnt = torch.empty(cap, dtype=torch.int32, device=dev)
    mass = torch.empty(cap, dtype=torch.float64, device=dev)
    com = torch.empty((3, cap), dtype=torch.float64, device=dev)
    nh = torch.empty(1, dtype=torch.int64, device=dev)
    _lib.check(_lib.lib().cola_fof_catalogue(_ptrs3(pos), n, float(box), _ptr(group), _ptr(size), int(n_min),
                                             float(m_p), cap, _ptr(root), _ptr(cnt), _ptr(mass), _ptrs3(com),
                                             _ptr(nh), _ptr(ws), ws.numel(), _stream()), "cola_fof_catalogue")
    k = int(nh.item())
    return dict(root=root[:k], n=cnt[:k], mass=mass[:k], com=com[:, :k])


def fof_mass_histogram(size, n_min, m_p, log10_edges):
    """Groups with N >= n_min per Warren-mass bin [10^e_b, 10^e_{b+1}): int64 device tensor."""
    torch = _torch()
    e = [float(v) for v in log10_edges]
    counts = torch.empty(len(e) - 1, dtype=torch.int64, device=size.device)
    arr = (ctypes.c_double * len(e))(*e)
    _lib.check(_lib.lib().cola_fof_mass_histogram(_ptr(size), int(size.numel()), int(n_min), float(m_p), arr,
                                                  len(e) - 1, _ptr(counts), _stream()), "cola_fof_mass_histogram")
    return counts
