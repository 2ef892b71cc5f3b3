#!/usr/bin/env python
"""Throughput of the COLA particle-mesh method on one MI355X.

Workload (the paper's optimum of Sec. 4.5 scaled to one GPU): 256^3 particles, a 768^3 force
mesh (PM_grid = 3), box 768 h^-1 Mpc, 40 time nodes linear in a from z = 19 to 0, 2LPT Gaussian
initial conditions with a BBKS spectrum in the MICE-GC cosmology, P(k) on the 768^3 mesh at
z = 1, 0.5 and 0.  One benchmark step is one whole realization: initial conditions, the 40-node
COLA run (40 force evaluations) and the three spectra.  Inputs are synthetic and seeded.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Prints one JSON line.  value = particles x 40 nodes x K / wall time of the K timed steps
(particle-steps/s), timed between two device synchronisations with everything resident in HBM.
The roofline block reports the kernel with the largest share of the timed region: its
algorithmic bytes per launch over its mean launch duration, both from HIP events recorded on
the launch stream during the timed region.  cpu_baseline times the float64 oracle (test
infrastructure) on one COLA step of the same workload on the host cores.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1509_04685_amd import workloads as W  # noqa: E402

METRIC = "particle-steps/s at 256³ part/768³ mesh; learned vs plain at 1% P(k)"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plain_256_768")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 48-seed ensemble measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction measurement")
    ap.add_argument("--no-haloes", action="store_true", help="skip the friends-of-friends halo measurement")
    ap.add_argument("--no-multipoles", action="store_true", help="skip the redshift-space multipole measurement")
    ap.add_argument("--no-aliasing", action="store_true", help="skip the aliasing-corrected P(k) measurement")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 512^3-particle runs (1536^3 plain mesh and 512^3 learned mesh)")
    ap.add_argument("--no-stepping", action="store_true",
                    help="skip the PM-only / time-sampling comparison (needs the halo measurement)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default FFT kernel shapes")
    ap.add_argument("--profile-step", action="store_true",
                    help="for hardware counters: autotune, ICs, one COLA step, one 1 GiB copy; no timing")
    ap.add_argument("--no-profiler", action="store_true",
                    help="time without per-kernel events (roofline omitted)")
    return ap.parse_args()


def algorithmic_bytes(kind, tag, n_g, n_part):
    """Bytes one launch of a kernel kind must move at minimum (one read of its inputs, one
    write of its outputs), float32 fields, half spectra counted without padding.  FFT passes are
    tagged with their mesh side; the other kernels work on the force mesh n_g."""
    n = tag if tag else n_g
    G = n ** 3
    C = n * n * (n // 2 + 1)
    N = n_part ** 3
    table = {
        "cic_deposit": 32 * N,                  # binning: displacements in; tile key + cell record out
        "cic_sort": 36 * N,                     # scatter: key + record in, record out (scans: O(G/512))
        "cic_tile": 16 * N + 4 * G,             # sorted records in, density mesh out
        "fft_z_r2c": 4 * G + 8 * C,
        "fft_y_forward": 16 * C,
        "fft_x_forward": 16 * C,
        "fft_x_green": 8 * C + 16 * C,          # one spectrum in, two x-transformed outputs
        "fft_y_split": 8 * C + 16 * C,          # one in, two out
        "fft_y_inverse": 16 * C,
        "fft_z_c2r": 8 * C + 4 * G,
        "fft_z_c2r3": 24 * C + 12 * G,          # the three force spectra in; (F_x, F_y, F_z) out,
                                                # interleaved (ghost cells and row padding not counted)
        "gather_kick_drift": 12 * G + 92 * N,   # the force mesh; x,p,psi1,psi2 in; x,p out; key +
                                                # record of the next deposit out (binning fused in)
        "gather_kick": 12 * G + 60 * N,
        "pk_deposit": 12 * G + 68 * N,          # binning with the partial drift: x, p, psi1, psi2 and
                                                # the force meshes in; key + record out
    }
    return table.get(kind)


def floor_bytes(n_g, n_part):
    """Algorithmic bytes of one PM step in the floor model (every FFT one read and one write of
    the array, Green/gradient fused) and in the three-pass model (each 3D FFT three passes)."""
    G = n_g ** 3
    C = n_g * n_g * (n_g // 2 + 1)
    N = n_part ** 3
    dep, gkd = 12 * N + 4 * G, 12 * G + 72 * N
    fft = (4 * G + 8 * C) + 3 * (8 * C + 4 * G)
    return dep + fft + gkd, dep + 3 * fft + gkd


def step_loop_bench(cola, torch, prob, cosmo, st, ws, seed, n_steps, reps=5):
    """The step loop alone (ICs and P(k) outputs excluded): median over reps of the time from the
    first force to the last node, timed with events."""
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        cola.ic_2lpt(prob, cosmo, [seed], st, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cola.step(prob, cosmo, st, n_steps - 1, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def node_index(table, a_out):
    a = table[:, 0]
    j = int((a <= a_out * (1 + 1e-12)).sum()) - 1
    return max(0, min(j, len(a) - 1))


KERNEL_SOURCES = {"fft": ("fft.hip", "fft_core.h", "fft_kernels.h", "fft_static_1536.hip", "fft_static_768.hip",
                          "fft_static_512.hip", "fft_static_384.hip", "fft_static_288.hip", "fft_static_256.hip"), "cic": ("deposit_sorted.hip",),
                  "pk_deposit": ("deposit_sorted.hip", "force_gather.h"),
                  "gather_kick_drift": ("deposit_sorted.hip", "pm_kernels.hip", "force_gather.h"),
                  "gather": ("pm_kernels.hip", "force_gather.h"), "lc": ("lc_kernels.hip",),
                  "pk_alias": ("pk_kernels.hip",)}


def source_hash(kind):
    """Hash of the source files of a kernel kind: counters taken on other sources are stale."""
    files = next((v for k, v in KERNEL_SOURCES.items() if kind.startswith(k)), None)
    if files is None:
        return None
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1509_04685_amd", "csrc")
    for name in files:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kind, tag):
    """HBM bytes per launch from the committed counter summary of this kernel and mesh size, if it
    was taken on the current source of the kernel."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{tag}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash(kind):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, seed):
    """One COLA step of the workload by the float64 oracle on the host (test infrastructure)."""
    from scipy import fft as sfft
    from oracle import cola as ocola, cosmology as ocosmo
    try:
        workers = len(os.sched_getaffinity(0))
    except AttributeError:
        workers = os.cpu_count() or 1
    with sfft.set_workers(workers):
        op = ocola.Problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], cfg["z_init"], cfg["n_steps"])
        c = ocosmo.Cosmology(**W.COSMOLOGY)
        sched = ocola.Schedule(op, c)
        st = ocola.initial_state(op, c, seed)
        ocola.evaluate_force(st, op)
        t0 = time.perf_counter()
        ocola.step(st, op, sched, 1)
        dt = time.perf_counter() - t0
    n = cfg["n_part"] ** 3
    return {
        "value": n / dt,
        "unit": "particle-steps/s",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"one COLA step (kick, drift, PM force on the {op.n_mesh}^3 mesh, kick) of the "
                   f"{cfg['n_part']}^3 workload from its 2LPT state, float64 numpy/scipy; "
                   f"{dt:.1f} s; FFTs on {workers} threads, CIC and gather single-threaded"),
    }


def copy_ceiling(cola, torch):
    """Streaming-copy bandwidth of the library's copy kernel (2 GiB read + 2 GiB written), the
    practical HBM ceiling beside the 8 TB/s peak."""
    a = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    cola.copy(a, b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        cola.copy(a, b)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    torch.cuda.empty_cache()
    return round(2.0 * (1 << 31) / (ms / 1e3) / 1e9, 1)


def ensemble_bench(cola, torch, reps):
    """48-seed ensemble in two shape classes (96^3/288^3 in 300 h^-1 Mpc and 128^3/384^3 in 400),
    40 nodes each, P(k) at z = 0, replayed as one captured hipGraph."""
    spec = []
    total_ps = 0
    for name in ("ens_96_288", "ens_128_384"):
        c = W.CONFIGS[name]
        prob = cola.make_problem(c["box"], c["n_part"], c["pm_factor"], c["z_init"], c["n_steps"],
                                 n_real=len(c["seeds"]))
        n_g = c["n_part"] * c["pm_factor"]
        spec.append(dict(prob=prob, seeds=c["seeds"], a_out=(1.0,), n_pk=n_g, n_bins=n_g // 2))
        total_ps += len(c["seeds"]) * c["n_part"] ** 3 * c["n_steps"]
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    ens = cola.Ensemble(spec, cosmo)
    ens.autotune()
    t0 = time.perf_counter()
    ens.run(graph=True)  # capture, instantiate, first launch
    torch.cuda.synchronize()
    t_capture = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ens.run(graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    n_real = sum(len(x["seeds"]) for x in spec)
    pk = ens.items[0]["out"][1].cpu()
    if not bool(torch.isfinite(pk).all()):
        raise RuntimeError("non-finite ensemble spectra")
    out = {"realizations": n_real, "seconds_per_ensemble": sec,
           "realizations_per_hour": n_real * 3600.0 / sec,
           "particle_steps_per_s": total_ps / sec,
           "first_launch_with_capture_s": t_capture, "replays_timed": reps,
           "classes": "24 x (96^3 particles, 288^3 mesh, L 300) + 24 x (128^3, 384^3, L 400), 40 nodes, "
                      "P(k) at z=0, one hipGraph (classes on forked streams)"}
    # z = 0 spectra of every member (k, P) for the learned ensemble's comparison
    spectra = [(it["out"][0][0].cpu().numpy(), it["out"][1][0].cpu().numpy()) for it in ens.items]
    del ens
    cola.ensemble_release()
    torch.cuda.empty_cache()
    return out, spectra


def learned_ensemble_bench(cola, torch, reps, plain, plain_spectra):
    """The batched learned-correction form: the same 48 seeds on 1x meshes (96^3 and 128^3 cells, the
    trained network's 3 h^-1 Mpc resolution) with the network in every step, captured in one
    hipGraph, against the plain 3x ensemble above: realizations per hour, and max |P/P_3x - 1| for
    k < 1 of every member at z = 0 on the plain ensemble's analysis meshes (288^3, 384^3)."""
    import numpy as np
    from paper_1509_04685_amd import learned as L
    path = os.path.join(ROOT, "paper_1509_04685_amd", "lc_weights_c16.json")
    if not os.path.exists(path):
        return {"skipped": "no trained weights"}
    net, _ = L.load_net(path)
    spec = []
    total_ps = 0
    for name in ("ens_96_288", "ens_128_384"):
        c = W.CONFIGS[name]
        prob = cola.make_problem(c["box"], c["n_part"], 1, c["z_init"], c["n_steps"], n_real=len(c["seeds"]))
        n_pk = c["n_part"] * c["pm_factor"]
        spec.append(dict(prob=prob, seeds=c["seeds"], a_out=(1.0,), n_pk=n_pk, n_bins=n_pk // 2, net=net))
        total_ps += len(c["seeds"]) * c["n_part"] ** 3 * c["n_steps"]
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    ens = cola.Ensemble(spec, cosmo)
    ens.autotune()
    ens.run(graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ens.run(graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    n_real = sum(len(x["seeds"]) for x in spec)
    errs = []
    for it, (k3, p3) in zip(ens.items, plain_spectra):
        kk, pp = it["out"][0][0].cpu().numpy(), it["out"][1][0].cpu().numpy()
        for r in range(pp.shape[0]):
            errs.append(L.max_error(kk[r], pp[r], p3[r]))
    errs = np.array(errs)
    out = {"realizations": n_real, "seconds_per_ensemble": sec, "realizations_per_hour": n_real * 3600.0 / sec,
           "particle_steps_per_s": total_ps / sec,
           "speedup_vs_plain_3x_ensemble": round(plain["seconds_per_ensemble"] / sec, 3),
           "max_pk_error_k_lt_1": {"worst": round(float(errs.max()), 4), "median": round(float(np.median(errs)), 4),
                                   "members_within_1pct": int((errs <= 0.01).sum())},
           "classes": "24 x (96^3 particles, 96^3 mesh, L 300) + 24 x (128^3, 128^3, L 400) with the trained network "
                      "(cola_step_lc), 40 nodes, P(k) at z=0 on 288^3 / 384^3, one hipGraph; error of each member "
                      "against the plain 3x ensemble member of the same seed"}
    del ens
    cola.ensemble_release()
    torch.cuda.empty_cache()
    return out


HALO_N_MIN = 101  # haloes of more than 100 particles (Sec. 2.5)


def haloes(cola, torch, prob, st, cosmo, box, n_part):
    """Friends-of-friends (b = 0.2) on the state's positions and the Warren mass histogram of the
    haloes with more than 100 particles, in 0.2 dex bins from the 101-particle mass."""
    import numpy as np
    pos = cola.positions(prob, st)
    link = cola.linking_length(box, n_part)
    m_p = cola.particle_mass(cola.make_cosmology(**W.COSMOLOGY), box, n_part)
    e0 = np.log10(m_p * HALO_N_MIN * (1.0 - HALO_N_MIN ** -0.6))
    edges = e0 + 0.2 * np.arange(11)
    fws = cola.fof_workspace(pos.shape[1], box, link)
    cola.fof(pos, box, link, ws=fws)  # warm
    stream = torch.cuda.current_stream()
    e0v, e1v = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0v.record(stream)
    g, s = cola.fof(pos, box, link, ws=fws)
    e1v.record(stream)
    counts = cola.fof_mass_histogram(s, HALO_N_MIN, m_p, edges).cpu().numpy()
    ms = e0v.elapsed_time(e1v)
    largest = int(s.max().item())
    del pos, g, s, fws
    return {"counts": counts, "log10_edges": edges, "fof_ms": ms, "largest": largest, "particle_mass": m_p}


def abundance_error(counts, ref, min_count=20):
    """Largest |N / N_ref - 1| over mass bins where the reference has at least min_count haloes,
    and the ratio of the totals."""
    import numpy as np
    ok = ref >= min_count
    per_bin = np.abs(counts[ok] / ref[ok] - 1.0)
    return (float(per_bin.max()) if per_bin.size else float("nan"), float(counts.sum() / max(1, ref.sum())))


def stepping_bench(cola, torch, cfg, pk_ref, halo_ref):
    """What the 2LPT frame, the time sampling and the initial redshift buy (Sec. 4.1-4.3, Appendix B)
    on the headline workload and seed: COLA and PM-only runs with 10, 20 and 40 nodes, 40
    logarithmic / a^0.8 nodes, 40 linear nodes from z_i = 9, 39 and 100, and 10 nodes from z_i = 9,
    each against the timed 40-node linear COLA run from z_i = 19 (P(k) at z = 0 and haloes)."""
    import numpy as np
    from paper_1509_04685_amd import learned as L
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    n_pk = cfg["n_part"] * cfg["pm_factor"]
    z0 = cfg["z_init"]
    # (frame, sampling, nodes, z_i): step count and frame at the fiducial z_i, the samplings of
    # Eq. 3, the initial-redshift sweep of Sec. 4.3 (40 linear nodes) and the 10-node default
    runs = [("cola", "linear", 10, z0), ("cola", "linear", 20, z0), ("pm", "linear", 10, z0), ("pm", "linear", 20, z0),
            ("pm", "linear", 40, z0), ("cola", "log", 40, z0), ("cola", "power", 40, z0),
            ("cola", "linear", 40, 9.0), ("cola", "linear", 40, 39.0), ("cola", "linear", 40, 100.0),
            ("cola", "linear", 10, 9.0)]
    out = {}
    for frame, sampling, n_steps, z_init in runs:
        prob = cola.make_problem(cfg["box"], cfg["n_part"], cfg["pm_factor"], z_init, n_steps,
                                 sampling=sampling, sampling_power=0.8, frame=frame)
        st = cola.ParticleState(prob)
        ws = cola.Workspace(prob, n_pk=n_pk)
        cola.ic_2lpt(prob, cosmo, [cfg["seeds"][0]], st, ws)
        cola.step(prob, cosmo, st, n_steps - 1, ws)
        km, pk, _ = cola.power_spectrum(prob, cosmo, st, 1.0, n_pk, n_pk // 2, ws)
        k, pk = km.cpu().numpy()[0], pk.cpu().numpy()[0]
        h = haloes(cola, torch, prob, st, cosmo, cfg["box"], cfg["n_part"])
        worst, total = abundance_error(h["counts"], halo_ref["counts"])
        sel = (k > 0) & (k < 1.0)
        at = {f"{kk:g}": round(float(np.interp(kk, k[sel], pk[sel] / pk_ref[sel])) - 1.0, 4) for kk in (0.1, 0.3, 1.0)}
        name = f"{frame}_{sampling if sampling != 'power' else 'a0.8'}_{n_steps}"
        if z_init != z0:
            name += f"_zi{z_init:g}"
        out[name] = {"max_pk_error_k_lt_1": round(L.max_error(k, pk, pk_ref), 4), "pk_ratio_minus_1": at,
                     "haloes_gt_100": int(h["counts"].sum()), "halo_total_ratio": round(total, 4),
                     "max_halo_abundance_error": round(worst, 4)}
        del st, ws
        torch.cuda.empty_cache()
    out["reference"] = "COLA, 40 nodes linear in a from z = 19, the timed headline run (same seed, same mesh)"
    return out


def multipoles_bench(cola, torch, prob, st, cfg, n_pk=1024):
    """Redshift-space multipoles (Sec. 6: Eq. 5, 6) of the headline run's z = 0 particles on the
    paper's 1024^3 analysis mesh, line of sight z: time per call and P_2 / P_0 at large scales
    against the linear (Kaiser) value (4f/3 + 4f^2/7) / (1 + 2f/3 + f^2/5)."""
    import numpy as np
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    tab = cola.schedule_table(prob, cosmo)
    a = float(tab[-1, 0])
    # f = dln D1 / dln a at the last node from a three-point one-sided difference on the nodes
    a3, d3 = tab[-3:, 0], tab[-3:, 1]
    h = a3[2] - a3[1]
    dd = (3.0 * d3[2] - 4.0 * d3[1] + d3[0]) / (2.0 * h) if abs((a3[1] - a3[0]) - h) < 1e-9 * h else None
    f = a * dd / d3[2] if dd is not None else float("nan")
    ws = cola.Workspace(prob, n_pk=n_pk)
    n_bins = n_pk // 2
    cola.power_multipoles(prob, cosmo, st, a, n_pk, n_bins, ws)  # warm (plans, twiddles)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    km, p0, p2, p4, nm = cola.power_multipoles(prob, cosmo, st, a, n_pk, n_bins, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    km, p0, p2, p4, nm = (t.cpu().numpy()[0] for t in (km, p0, p2, p4, nm))
    real = cola.power_multipoles(prob, cosmo, st, a, n_pk, n_bins, ws, redshift_space=False)
    r0 = real[1].cpu().numpy()[0]
    lo = (nm > 0) & (km < 0.05)
    kaiser = (4 * f / 3 + 4 * f * f / 7) / (1 + 2 * f / 3 + f * f / 5)
    pick = {f"{kk:g}": [round(float(np.interp(kk, km[nm > 0], v[nm > 0])), 1) for v in (p0, p2, p4)]
            for kk in (0.05, 0.1, 0.2, 0.5)}
    del ws
    torch.cuda.empty_cache()
    return {"ms_per_call": round(e0.elapsed_time(e1), 3), "analysis_mesh": n_pk, "los": "z",
            "growth_rate_f": round(f, 4), "p2_over_p0_k_lt_0.05": round(float(p2[lo].sum() / p0[lo].sum()), 4),
            "kaiser_p2_over_p0": round(kaiser, 4),
            "p0_over_real_k_lt_0.05": round(float(p0[lo].sum() / r0[lo].sum()), 4),
            "kaiser_p0_over_real": round(1 + 2 * f / 3 + f * f / 5, 4),
            "p0_p2_p4_at_k": pick,
            "what": "plane-parallel redshift space (Eq. 5) at z = 0, multipoles in the P(k) shells (Eq. 6); "
                    "mode-weighted sums over k < 0.05 h/Mpc against linear theory"}


def aliasing_bench(cola, torch, prob, cosmo, st, ws, n_pk, n_bins, reps=3, iterations=4):
    """P(k) of the state at a = 1 with and without the Jing (2005) aliasing correction (Sec. 2.5):
    the time of each estimate and what the correction changes."""
    import numpy as np
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    ms0, (km, p0, nm) = timed(lambda: cola.power_spectrum(prob, cosmo, st, 1.0, n_pk, n_bins, ws))
    ms1, (_, p1, _) = timed(lambda: cola.power_spectrum_jing(prob, cosmo, st, 1.0, n_pk, n_bins, ws,
                                                             iterations=iterations))
    cola.profiler_enable(True)
    cola.power_spectrum_jing(prob, cosmo, st, 1.0, n_pk, n_bins, ws, iterations=iterations)
    groups = cola.profiler_read_groups()
    cola.profiler_enable(False)
    k, p0, p1 = km.cpu().numpy()[0], p0.cpu().numpy()[0], p1.cpu().numpy()[0]
    sel = (k > 0) & (p0 > 0)
    r = p1[sel] / p0[sel] - 1.0
    k_nyq = np.pi * n_pk / prob.box
    at = {f"{kk:g}": round(float(np.interp(kk, k[sel], r)), 5) for kk in (0.5, 1.0, 2.0) if kk < k[sel].max()}
    at["k_nyquist"] = round(float(np.interp(k_nyq, k[sel], r)), 5)
    passes = {f"{name}@{tag}": {"ms_per_launch": round(ms / cnt, 4), "launches": cnt}
              for (name, tag), (ms, cnt) in groups.items() if name == "pk_alias"}
    return {"ms_plain": round(ms0, 3), "ms_corrected": round(ms1, 3), "iterations": iterations,
            "corrected_over_plain_minus_1": at, "k_nyquist": round(k_nyq, 4), "passes": passes,
            "what": f"P(k) of the z = 0 state on the {n_pk}^3 mesh ({n_bins} bins): plain CIC-deconvolved "
                    f"estimator vs the Jing (2005) aliasing correction; passes: @1 slopes + aliasing table "
                    f"(one evaluation per class of sorted |m|), @2 rebinning, per iteration"}


def large_bench(cola, torch):
    """The 512^3-particle workload: plain COLA on the 1536^3 mesh (PM_grid 3), one realization after
    a warm-up, then the learned form on the 512^3 mesh beside it (same seed, P(k) at z = 0 on the
    1536^3 analysis mesh)."""
    cfg = W.CONFIGS["plain_512_1536"]
    box, n_part, pm = cfg["box"], cfg["n_part"], cfg["pm_factor"]
    n_g, n_steps, seed = n_part * pm, cfg["n_steps"], cfg["seeds"][0]
    n_pk, n_bins = n_g, n_g // 2
    prob = cola.make_problem(box, n_part, pm, cfg["z_init"], n_steps)
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=n_pk)
    t_at = time.perf_counter()
    report = cola.autotune(prob, ws, n_pk=n_pk, state=st)
    t_at = time.perf_counter() - t_at
    print(f"[bench] large: FFT autotune ({t_at:.1f} s):\n" + report.rstrip(), file=sys.stderr, flush=True)
    out = tuple(torch.empty((1, n_bins), dtype=torch.float64, device="cuda") for _ in range(3))

    def realization():
        cola.ic_2lpt(prob, cosmo, [seed], st, ws)
        cola.step(prob, cosmo, st, n_steps - 1, ws)
        cola.power_spectrum(prob, cosmo, st, 1.0, n_pk, n_bins, ws, out=out)

    realization()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    realization()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    pk_plain = out[1].cpu().numpy()[0]
    res = {"plain_512_1536": {"ms_per_realization": round(ms, 1),
                              "particle_steps_per_s": round(n_part ** 3 * n_steps / (ms / 1e3), 1),
                              "realizations_per_hour": round(3.6e6 / ms, 1), "autotune_s": round(t_at, 1)}}
    del st, ws, out
    torch.cuda.empty_cache()
    print(f"[bench] large: plain 512^3 / 1536^3 {ms:.0f} ms per realization", file=sys.stderr, flush=True)
    res["learned_512_512"] = learned_bench(cola, torch, "plain_512_1536", [pk_plain], (1.0,), n_pk, n_bins, ms,
                                           reps=1)
    res["workload"] = (f"plain_512_1536: {n_part}^3 particles, {n_g}^3 mesh (PM_grid {pm}), box {box:g} h^-1 Mpc, "
                       f"{n_steps} nodes linear in a from z={cfg['z_init']:g}, seed {seed}, P(k) at z = 0 on "
                       f"{n_pk}^3; learned_512_512: the same particles on the {n_part}^3 mesh with the network")
    return res


def learned_bench(cola, torch, cfg_name, pk_plain3, a_outs, n_pk, n_bins, ms_plain3, reps, halo3=None,
                  holdout_seeds=()):
    """The learned-correction form: 256^3 particles on the 256^3 (PM_grid = 1) mesh with the trained
    network, against the plain 3x realization timed above (same seed, same outputs) and the plain
    1x run without the network."""
    from paper_1509_04685_amd import learned as L
    path = os.path.join(ROOT, "paper_1509_04685_amd", "lc_weights_c16.json")
    if not os.path.exists(path):
        return {"skipped": "no trained weights (run paper_1509_04685_amd/train_lc.py)"}
    net, doc = L.load_net(path)
    lname = {"plain_256_768": "learned_256_256", "plain_512_1536": "learned_512_512"}.get(cfg_name)
    if lname is None:
        return {"skipped": f"no learned workload beside {cfg_name}"}
    c = W.CONFIGS[lname]
    prob = cola.make_problem(c["box"], c["n_part"], c["pm_factor"], c["z_init"], c["n_steps"])
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    table = cola.schedule_table(prob, cosmo)
    plan = [(a, node_index(table, a)) for a in sorted(a_outs)]
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=n_pk)
    lws = cola.lc_workspace(c["n_part"] * c["pm_factor"], net.channels, 1)
    outs = [tuple(torch.empty((1, n_bins), dtype=torch.float64, device="cuda") for _ in range(3))
            for _ in a_outs]

    def realization(use_net):
        cola.ic_2lpt(prob, cosmo, [c["seeds"][0]], st, ws)

        def adv(j):
            if use_net:
                cola.step_lc(prob, cosmo, st, j, net, lws, ws)
            else:
                cola.step(prob, cosmo, st, j, ws)
        for i, (a, j) in enumerate(plan):
            adv(j)
            cola.power_spectrum(prob, cosmo, st, a, n_pk, n_bins, ws, out=outs[i])
        adv(c["n_steps"] - 1)

    res = {}
    stream = torch.cuda.current_stream()
    for name, use_net in (("plain_1x", False), ("learned_1x", True)):
        cola.autotune(prob, ws, n_pk=n_pk, state=st)
        realization(use_net)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            realization(use_net)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        cola.profiler_enable(True)
        realization(use_net)
        groups = cola.profiler_read_groups()
        cola.profiler_enable(False)
        for (kname, tag), (kms, cnt) in sorted(groups.items(), key=lambda kv: -kv[1][0])[:10]:
            label = f"{kname}@{tag}" if tag else kname
            print(f"[bench]   {name:10s} {label:22s} {kms:8.2f} ms/realization  {cnt:5d} launches  "
                  f"{kms / cnt:7.3f} ms/launch", file=sys.stderr, flush=True)
        by_a = {}
        for (a, _), o, ref in zip(plan, outs, pk_plain3):
            by_a[f"{a:.3f}"] = round(L.max_error(o[0].cpu().numpy()[0], o[1].cpu().numpy()[0], ref), 4)
        res[name] = {"ms_per_realization": round(ms, 2), "realizations_per_hour": round(3.6e6 / ms, 1),
                     "max_pk_error_k_lt_1": max(by_a.values()), "max_pk_error_k_lt_1_by_a": by_a}
        if halo3 is not None:  # the state now holds this form's z = 0 particles
            h = haloes(cola, torch, prob, st, cosmo, c["box"], c["n_part"])
            worst, total = abundance_error(h["counts"], halo3["counts"])
            res[name]["haloes_gt_100"] = int(h["counts"].sum())
            res[name]["halo_counts"] = [int(v) for v in h["counts"]]
            res[name]["max_halo_abundance_error"] = round(worst, 4)
            res[name]["halo_total_ratio"] = round(total, 4)
    res["plain_3x"] = {"ms_per_realization": round(ms_plain3, 2), "realizations_per_hour": round(3.6e6 / ms_plain3, 1)}
    if halo3 is not None:
        res["plain_3x"]["haloes_gt_100"] = int(halo3["counts"].sum())
        res["plain_3x"]["halo_counts"] = [int(v) for v in halo3["counts"]]
        res["halo_bins_log10_mass"] = [round(float(v), 3) for v in halo3["log10_edges"]]
    res["speedup_vs_plain_3x"] = round(ms_plain3 / res["learned_1x"]["ms_per_realization"], 3)
    if holdout_seeds:
        # seeds never used for training, calibration or any choice of the method
        prob3 = cola.make_problem(c["box"], c["n_part"], 3, c["z_init"], c["n_steps"])
        worst = {}
        for s in holdout_seeds:
            ref = L.run_spectra(prob3, cosmo, s, sorted(a_outs), n_pk, n_bins)
            got = L.run_spectra(prob, cosmo, s, sorted(a_outs), n_pk, n_bins, net=net)
            worst[str(s)] = round(max(L.max_error(k, pl, p3) for (k, p3), (_, pl) in zip(ref, got)), 4)
        vals = sorted(worst.values())
        res["holdout"] = {"seeds": list(holdout_seeds), "max_pk_error_k_lt_1": worst,
                          "worst": vals[-1], "median": vals[len(vals) // 2],
                          "seeds_within_1pct": sum(v <= 0.01 for v in vals),
                          "what": "per seed: max over 0<k<1 h/Mpc and over the outputs of |P_learned1x / P_plain3x - 1|"}
    rec = doc.get("recipe", {})
    seeds = rec.get("calib_seeds", (3001, 3002))
    inputs = "density and force" if rec.get("force_input", True) else "density only"
    res["network"] = (f"C={net.channels}: two 3x3x3 conv layers + SiLU, 1x1x1 output, input {inputs}; BF16 matrix "
                      f"cores, FP32 accumulation; trained on 128^3/384^3 pairs in 384 h^-1 Mpc (seeds 3001-3006), "
                      f"validation loss {doc['val_loss_initial']:.3f} -> {doc['val_loss_trained']:.3f}; output "
                      f"scale calibrated on training seeds {seeds[0]}-{seeds[-1]} at every output: factor "
                      f"{net.out_scale / doc.get('out_scale_fitted', net.out_scale):.2f}, slope "
                      f"{net.out_scale_slope:+.2f} in (1 - a)"
                      + (f", schedule {[round(v, 3) for v in net.schedule[1]]} at a = {[round(v, 3) for v in net.schedule[0]]}"
                         if net.schedule else "")
                      + (f"; Green's-function transfer T(|k|/k_N, a): cubic in |k|/k_N on {len(net.green_filter[0])} "
                         f"knots, rows at the schedule's knots, calibrated with the schedule at trajectory level in "
                         f"{len(doc['green_filter']['passes'])} passes on training seeds "
                         + ", ".join(f"{p['seeds'][0]}-{p['seeds'][-1]}" for p in doc['green_filter']['passes'])
                         + f" ({doc['green_filter']['passes'][-1]['n_part']}^3 particles)" if net.green_filter else "")
                      + f"; evaluation seed {c['seeds'][0]} held out")
    res["workload"] = (f"{lname}: {c['n_part']}^3 particles, {c['n_part']}^3 mesh (PM_grid 1), box {c['box']:g}, "
                       f"40 nodes from z=19, seed {c['seeds'][0]}, P(k) on {n_pk}^3 at the same outputs; error = "
                       f"max over 0<k<1 h/Mpc and over the outputs of |P/P_plain3x - 1| (by_a: per output); haloes: FoF b=0.2 at z=0, "
                       f"Warren masses, > 100 particles, 0.2 dex bins; halo error = max over bins with >= 20 "
                       f"plain-3x haloes of |N/N_plain3x - 1|")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(an ensemble shards one realization per GPU with no communication).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1509_04685_amd as cola

    cfg = W.CONFIGS[args.workload]
    box, n_part, pm = cfg["box"], cfg["n_part"], cfg["pm_factor"]
    n_g = n_part * pm
    n_steps = cfg["n_steps"]
    a_outs = cfg.get("a_out", (1.0,))
    n_pk = n_g
    n_bins = n_pk // 2
    seed = cfg["seeds"][0]

    torch.cuda.set_device(0)
    prob = cola.make_problem(box, n_part, pm, cfg["z_init"], n_steps)
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    table = cola.schedule_table(prob, cosmo)
    st = cola.ParticleState(prob)
    ws = cola.Workspace(prob, n_pk=n_pk)
    outs = [tuple(torch.empty((1, n_bins), dtype=torch.float64, device="cuda") for _ in range(3))
            for _ in a_outs]
    plan = [(a, node_index(table, a)) for a in sorted(a_outs)]

    def realization():
        cola.ic_2lpt(prob, cosmo, [seed], st, ws)
        for i, (a, j) in enumerate(plan):
            cola.step(prob, cosmo, st, j, ws)
            cola.power_spectrum(prob, cosmo, st, a, n_pk, n_bins, ws, out=outs[i])
        cola.step(prob, cosmo, st, n_steps - 1, ws)

    if args.profile_step:
        print(cola.autotune(prob, ws, n_pk=n_pk, state=st).rstrip(), file=sys.stderr, flush=True)
        cola.ic_2lpt(prob, cosmo, [seed], st, ws)
        cola.step(prob, cosmo, st, 1, ws)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        cola.copy(a, b)  # 1 GiB read + 1 GiB write: the counter yardstick
        del a, b
        path = os.path.join(ROOT, "paper_1509_04685_amd", "lc_weights_c16.json")
        if os.path.exists(path):  # one step of the learned 1x form
            from paper_1509_04685_amd import learned as L
            net, _ = L.load_net(path)
            c = W.CONFIGS["learned_256_256"]
            p1 = cola.make_problem(c["box"], c["n_part"], c["pm_factor"], c["z_init"], c["n_steps"])
            s1 = cola.ParticleState(p1)
            w1 = cola.Workspace(p1)
            lws = cola.lc_workspace(c["n_part"] * c["pm_factor"], net.channels, 1)
            cola.ic_2lpt(p1, cosmo, [c["seeds"][0]], s1, w1)
            cola.step_lc(p1, cosmo, s1, 1, net, lws, w1)
        torch.cuda.synchronize()
        print("[bench] profile step done", file=sys.stderr, flush=True)
        return
    print(f"[bench] {args.workload}: {n_part}^3 particles, {n_g}^3 mesh, {n_steps} nodes; "
          f"warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    if not args.no_autotune:
        t_at = time.perf_counter()
        report = cola.autotune(prob, ws, n_pk=n_pk, state=st)
        print(f"[bench] FFT autotune ({time.perf_counter() - t_at:.1f} s):\n" + report.rstrip(),
              file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        realization()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if not args.no_profiler:
        cola.profiler_enable(True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        realization()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    kernels = cola.profiler_read_groups() if not args.no_profiler else {}
    cola.profiler_enable(False)
    pk_final = outs[-1][1].cpu().numpy()[0]
    if not np.all(np.isfinite(pk_final)):
        raise RuntimeError("non-finite power spectrum")

    ms_per_step = ms_total / args.steps
    particles = n_part ** 3
    value = particles * n_steps * args.steps / (ms_total / 1e3)
    print(f"[bench] {ms_per_step:.1f} ms per realization ({wall:.2f} s wall for {args.steps}); "
          f"{value:.3e} particle-steps/s", file=sys.stderr, flush=True)

    roofline = None
    if kernels:
        ranked = sorted(kernels.items(), key=lambda kv: -kv[1][0])
        for (name, tag), (ms, cnt) in ranked:
            b = algorithmic_bytes(name, tag, n_g, n_part)
            gbs = (b / (ms / cnt / 1e3) / 1e9) if b else float("nan")
            label = f"{name}@{tag}" if tag else name
            print(f"[bench]   {label:22s} {ms / args.steps:9.2f} ms/step  {cnt / args.steps:7.1f} launches/step"
                  f"  {ms / cnt:8.3f} ms/launch  {gbs:8.1f} GB/s", file=sys.stderr, flush=True)
        dom = next((kv for kv in ranked if algorithmic_bytes(kv[0][0], kv[0][1], n_g, n_part)), None)
        if dom:
            (name, tag), (ms, cnt) = dom
            b = algorithmic_bytes(name, tag, n_g, n_part)
            achieved = b / (ms / cnt / 1e3) / 1e9
            traffic = read_traffic(name, tag or n_g)
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": traffic, "kernel": name, "mesh": tag or n_g, "bytes_per_launch": b,
                        "ms_per_launch": round(ms / cnt, 4), "launches_per_step": cnt / args.steps,
                        "share_of_step": round(ms / ms_total, 4)}
            # every kernel with at least 5% of the realization, against the same byte model
            roofline["kernels"] = []
            for (kname, ktag), (kms, kcnt) in ranked:
                if kms / ms_total < 0.05:
                    continue
                kb = algorithmic_bytes(kname, ktag, n_g, n_part)
                kach = kb / (kms / kcnt / 1e3) / 1e9 if kb else None
                roofline["kernels"].append({
                    "kernel": kname, "mesh": ktag or n_g, "share_of_step": round(kms / ms_total, 4),
                    "ms_per_launch": round(kms / kcnt, 4), "bytes_per_launch": kb,
                    "achieved": round(kach, 1) if kach else None,
                    "frac": round(kach / HBM_PEAK_GBS, 4) if kach else None,
                    "traffic": read_traffic(kname, ktag or n_g)})

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n_part}^3 particles, {n_g}^3 mesh (PM_grid {pm}), "
                               f"box {box:g} h^-1 Mpc, {n_steps} nodes linear in a from z={cfg['z_init']:g}, "
                               f"2LPT ICs, P(k) at a={','.join(f'{a:.3f}' for a in sorted(a_outs))}",
                   "particles": particles, "mesh": n_g, "nodes": n_steps, "seed": seed,
                   "step_unit": "one realization (ICs + all nodes + P(k) outputs)"},
        "roofline": roofline,
    }
    if roofline is not None:
        roofline["copy_ceiling_gbs"] = copy_ceiling(cola, torch)
    ms_loop = step_loop_bench(cola, torch, prob, cosmo, st, ws, seed, n_steps)
    fb, fb3 = floor_bytes(n_g, n_part)
    ms_node = ms_loop / n_steps
    result["step_loop"] = {
        "particle_steps_per_s": round(particles * n_steps / (ms_loop / 1e3), 1),
        "ms_per_realization": round(ms_loop, 2), "ms_per_node": round(ms_node, 3),
        "floor_bytes_per_step": fb, "three_pass_bytes_per_step": fb3,
        "floor_ms_at_peak": round(fb / HBM_PEAK_GBS / 1e6, 3), "three_pass_ms_at_peak": round(fb3 / HBM_PEAK_GBS / 1e6, 3),
        "floor_fraction": round(fb / HBM_PEAK_GBS / 1e6 / ms_node, 4),
        "three_pass_fraction": round(fb3 / HBM_PEAK_GBS / 1e6 / ms_node, 4),
        "what": "ICs and P(k) outputs excluded: the first force to the last node (40 forces, 39 drifts), "
                "median of 5; fractions = step time at 8 TB/s of the floor / three-pass byte models over "
                "the measured time per node"}
    print(f"[bench] step loop: {json.dumps(result['step_loop'])}", file=sys.stderr, flush=True)
    if not args.no_multipoles:
        print("[bench] redshift-space multipoles on the 1024^3 analysis mesh", file=sys.stderr, flush=True)
        result["multipoles"] = multipoles_bench(cola, torch, prob, st, cfg)
        print(f"[bench] multipoles: {json.dumps(result['multipoles'])}", file=sys.stderr, flush=True)
    if not args.no_aliasing:
        result["aliasing"] = aliasing_bench(cola, torch, prob, cosmo, st, ws, n_pk, n_bins)
        print(f"[bench] aliasing: {json.dumps(result['aliasing'])}", file=sys.stderr, flush=True)
    halo3 = None
    if not args.no_haloes:
        # the state holds the last timed realization at z = 0
        halo3 = haloes(cola, torch, prob, st, cosmo, box, n_part)
        result["haloes"] = {"fof_ms": round(halo3["fof_ms"], 3),
                            "fof_particles_per_s": round(particles / (halo3["fof_ms"] / 1e3), 1),
                            "haloes_gt_100": int(halo3["counts"].sum()), "largest_halo": halo3["largest"],
                            "particle_mass": halo3["particle_mass"],
                            "what": "friends-of-friends (b = 0.2 of the mean separation) of the z = 0 particles, "
                                    "Warren-mass histogram of haloes with more than 100 particles"}
        print(f"[bench] haloes: {json.dumps(result['haloes'])}", file=sys.stderr, flush=True)
    if halo3 is not None and not args.no_stepping:
        print("[bench] time stepping: COLA vs PM only, 10/20/40 nodes, log and a^0.8 samplings", file=sys.stderr,
              flush=True)
        result["stepping"] = stepping_bench(cola, torch, cfg, outs[-1][1].cpu().numpy()[0], halo3)
        print(f"[bench] stepping: {json.dumps(result['stepping'])}", file=sys.stderr, flush=True)
    if not args.no_learned:
        print("[bench] learned correction: 256^3 on the 256^3 mesh vs the plain runs", file=sys.stderr, flush=True)
        result["learned"] = learned_bench(cola, torch, args.workload, [o[1].cpu().numpy()[0] for o in outs], a_outs, n_pk,
                                          n_bins, ms_per_step, reps=2, halo3=halo3, holdout_seeds=(41, 42, 43, 44, 45))
        print(f"[bench] learned: {json.dumps(result['learned'])}", file=sys.stderr, flush=True)
    if not args.no_ensemble:
        del st, ws, outs
        torch.cuda.empty_cache()
        print("[bench] ensemble: 48 seeds in two shape classes, hipGraph", file=sys.stderr, flush=True)
        result["ensemble"], plain_spectra = ensemble_bench(cola, torch, reps=2)
        print(f"[bench] ensemble: {result['ensemble']['seconds_per_ensemble']:.2f} s per 48 realizations, "
              f"{result['ensemble']['realizations_per_hour']:.0f} realizations/hour", file=sys.stderr, flush=True)
        if not args.no_learned:
            print("[bench] learned ensemble: the same 48 seeds on 1x meshes with the network", file=sys.stderr,
                  flush=True)
            result["learned_ensemble"] = learned_ensemble_bench(cola, torch, 2, result["ensemble"], plain_spectra)
            print(f"[bench] learned ensemble: {json.dumps(result['learned_ensemble'])}", file=sys.stderr, flush=True)
    if not args.no_large and args.workload == "plain_256_768":
        print("[bench] large: 512^3 particles, plain 1536^3 mesh and learned 512^3 mesh", file=sys.stderr, flush=True)
        result["large"] = large_bench(cola, torch)
        print(f"[bench] large: {json.dumps(result['large'])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline: float64 oracle, one step", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(cfg, seed)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
