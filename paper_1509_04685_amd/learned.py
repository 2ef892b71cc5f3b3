"""Training and use of the learned coarse-mesh force correction (cola_lc_* in include/cola.h).

Sec. 4.4 finds that a force mesh coarser than PM_grid = 3 biases haloes through the force
resolution; this module trains the library's correction network so that a PM_grid = 1 run
approaches the PM_grid = 3 one.  Training pairs come from the method itself: at every chosen node
of a plain fine-mesh run, the particle positions and the fine-mesh acceleration there (the
target); the coarse-mesh fields of the same positions are the network's input.  The loss is the
particle-level relative residual

    L = sum_p |g1_p + G[dF]_p - g3_p|^2 / sum_p |g3_p - g1_p|^2

(1 without the network).  Every computation runs in libcola's kernels; this module only chooses
samples, holds device buffers and reads back scalars.  The input and output scales are set once
from the first sample on the host (root mean squares).
"""

import numpy as np

from . import (LcNet, ParticleState, Workspace, ic_2lpt, lc_backward, lc_forward, lc_loss, lc_workspace,
               make_problem, pm_fields, positions, power_spectrum, schedule_table, step, step_lc)


def _torch():
    import torch
    return torch


class Sample:
    """One training pair: positions, fine-mesh acceleration, and the coarse-mesh fields."""

    def __init__(self, pos, acc_fine, n_coarse, box, ws=None):
        f = pm_fields(pos, n_coarse, box, ws=ws)
        self.pos = pos
        self.acc_fine = acc_fine
        self.delta = f["delta"]
        self.g = f["g"]
        self.acc = f["acc"]


def make_samples(cosmo, box, n_part, pm_fine, n_steps, z_init, seeds, nodes=None, net=None):
    """A Sample (coarse mesh = N_p cells) at each node in `nodes` (default: all) of one run per
    seed.  The runs are plain fine-mesh runs, or with `net` the corrected coarse runs (PM_grid 1
    with the network): the positions are then the ones the corrected form visits, and the targets
    stay the fine-mesh accelerations at those positions."""
    prob = make_problem(box, n_part, 1 if net is not None else pm_fine, z_init, n_steps)
    st = ParticleState(prob)
    ws = Workspace(prob)
    lws = lc_workspace(n_part, net.channels, 1) if net is not None else None
    out = []
    for seed in seeds:
        ic_2lpt(prob, cosmo, [int(seed)], st, ws)
        for j in range(n_steps):
            if j > st.node:
                if net is None:
                    step(prob, cosmo, st, j, ws)
                else:
                    step_lc(prob, cosmo, st, j, net, lws, ws)
            if nodes is None or j in nodes:
                pos = positions(prob, st)
                acc_fine = pm_fields(pos, n_part * pm_fine, box, delta=False, g=False)["acc"]
                out.append(Sample(pos, acc_fine, n_part, box))
    return out


def scales_from(sample):
    """Input scales 1/rms of delta and of each force component, output scale rms(g_fine - g)."""
    d = sample.delta.cpu().numpy().astype(np.float64)
    g = sample.g.cpu().numpy().astype(np.float64)
    r = sample.acc_fine.cpu().numpy().astype(np.float64) - sample.acc.cpu().numpy().astype(np.float64)
    ins = [1.0 / max(np.sqrt(np.mean(d ** 2)), 1e-30)]
    ins += [1.0 / max(np.sqrt(np.mean(g[c] ** 2)), 1e-30) for c in range(3)]
    return tuple(float(np.float32(s)) for s in ins), float(np.float32(np.sqrt(np.mean(r ** 2))))


class Trainer:
    """Adam on mini-batches of samples (gradients summed over the batch)."""

    def __init__(self, net, n_coarse, box):
        torch = _torch()
        self.net = net
        self.n = int(n_coarse)
        self.box = float(box)
        n = self.n
        self.ws = lc_workspace(n, net.channels, 1, training=True)
        self.df = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        self.d_df = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        self.stats = torch.empty(2, dtype=torch.float64, device="cuda")

    def loss(self, s, training=False):
        lc_forward(self.net, s.delta, s.g, self.ws, df=self.df, training=training)
        lc_loss(s.pos, self.box, self.df, s.acc, s.acc_fine, self.stats, self.d_df)
        return self.stats

    def train(self, samples, iters, lr, batch=1, seed=0, lr_final=None):
        """Returns the per-iteration mean batch loss (host array)."""
        rng = np.random.default_rng(seed)
        hist = np.zeros(iters)
        for it in range(iters):
            for _ in range(batch):
                s = samples[int(rng.integers(len(samples)))]
                st = self.loss(s, training=True)
                lc_backward(self.net, self.d_df, self.ws)
                hist[it] += float(st.cpu()[0]) / batch
            rate = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(1, iters - 1))
            self.net.adam(rate)
        return hist

    def evaluate(self, samples):
        """Mean loss over samples (no parameter change)."""
        vals = []
        for s in samples:
            vals.append(float(self.loss(s).cpu()[0]))
        return float(np.mean(vals))


def new_net(sample, channels=16, seed=0, force_input=True):
    """A network with initial weights and scales from `sample`.  force_input=False zeroes the input
    scales of the three force channels: the network then sees only the density, so its response to
    a long-wavelength mode is a local stencil of the density (of order k^2 g at small k) and
    cannot rescale the large-scale force itself."""
    from . import lc_init_params
    ins, outs = scales_from(sample)
    if not force_input:
        ins = (ins[0], 0.0, 0.0, 0.0)
    return LcNet(channels, params=lc_init_params(channels, seed), in_scale=ins, out_scale=outs)


def run_spectra(prob, cosmo, seed, a_out, n_pk, n_bins, net=None):
    """One realization from its 2LPT ICs to the last node, with the network's correction when
    `net` is given; returns the P(k) (k_mean, pk) at each a_out as host arrays."""
    st = ParticleState(prob)
    ws = Workspace(prob, n_pk=n_pk)
    lws = lc_workspace(prob.n_part * prob.pm_factor, net.channels, prob.n_real) if net is not None else None
    ic_2lpt(prob, cosmo, [int(seed)], st, ws)
    tab = schedule_table(prob, cosmo)
    out = []

    def advance(j):
        if j > st.node:
            if net is None:
                step(prob, cosmo, st, j, ws)
            else:
                step_lc(prob, cosmo, st, j, net, lws, ws)

    for a in a_out:
        j = int((tab[:, 0] <= a * (1 + 1e-12)).sum()) - 1
        advance(j)
        km, pk, _ = power_spectrum(prob, cosmo, st, a, n_pk, n_bins, ws)
        out.append((km.cpu().numpy()[0], pk.cpu().numpy()[0]))
    advance(prob.n_steps - 1)
    return out


def load_net(path, training=False):
    """A network from a weights file written by train_lc.py."""
    import json
    with open(path) as fh:
        doc = json.load(fh)
    net = LcNet(int(doc["channels"]), params=np.asarray(doc["params"], dtype=np.float32),
                in_scale=doc["in_scale"], out_scale=doc["out_scale"], training=training)
    net.set_scales(net.in_scale, net.out_scale, doc.get("out_scale_slope", 0.0), doc.get("out_band", 0.0))
    sched = doc.get("schedule")
    net.set_schedule(*(sched if sched else (None, None)))
    gfil = doc.get("green_filter")
    if gfil:
        net.set_green_filter(gfil["u"], gfil["t"])
    return net, doc


def max_error(k, pk, pk_ref, k_max=1.0):
    """max over bins with 0 < k < k_max of |pk / pk_ref - 1| (host arrays)."""
    sel = (k > 0) & (k < k_max) & (pk_ref > 0)
    return float(np.abs(pk[sel] / pk_ref[sel] - 1.0).max())


def calibrate_out_scale(net, cosmo, box, n_part, z_init, n_steps, seeds, factors, slopes=(0.0,), n_pk=None,
                        k_max=1.0, log=None, bands=None, a_outs=(1.0,)):
    """Trajectory-level calibration of the output scale on training realizations.  For each factor
    f, slope s (and band weight b, when `bands` is given) the step uses out_scale * f * (1 + s (1 - a))
    at a node of scale factor a (and the band-pass weight b); every seed's corrected PM_grid = 1
    realization is compared with the plain PM_grid = 3 run of the same seed at every output scale
    factor in a_outs, by max over 0 < k < k_max of |P / P_3x - 1|, and the combination with the
    smallest worst case over seeds and outputs wins.  A network fitted to noisy force residuals
    underestimates the correction (regression dilution); this picks the scale on the training
    seeds only.  Sets the best values on the network and returns (out_scale, slope, table of
    (f, s, error)), or of (f, s, b, error) with bands."""
    n_pk = n_pk or n_part * 3
    n_bins = n_pk // 2
    base = net.out_scale
    prob1 = make_problem(box, n_part, 1, z_init, n_steps)
    prob3 = make_problem(box, n_part, 3, z_init, n_steps)
    refs = [run_spectra(prob3, cosmo, s, a_outs, n_pk, n_bins) for s in seeds]
    table = []
    for b in (bands if bands is not None else (None,)):
        for f in factors:
            for sl in slopes:
                net.set_scales(net.in_scale, base * f, sl, b)
                worst = 0.0
                for s, ref in zip(seeds, refs):
                    got = run_spectra(prob1, cosmo, s, a_outs, n_pk, n_bins, net=net)
                    for (k, p3), (_, plc) in zip(ref, got):
                        worst = max(worst, max_error(k, plc, p3, k_max))
                table.append((float(f), float(sl), worst) if b is None else (float(f), float(sl), float(b), worst))
                if log:
                    tag = "" if b is None else f" band {b:.2f}"
                    log(f"[calibrate] factor {f:.3f} slope {sl:+.2f}{tag}: worst max |P/P_3x - 1| {worst:.4f}")
    best = min(table, key=lambda x: x[-1])
    net.set_scales(net.in_scale, base * best[0], best[1], None if bands is None else best[2])
    return net.out_scale, net.out_scale_slope, table


def calibrate_schedule(net, cosmo, box, n_part, z_init, n_steps, seeds, knot_a, a_outs=(1.0,), n_pk=None,
                       k_max=1.0, rounds=5, log=None):
    """Refines the step's output scale into a piecewise-linear schedule over a: starting from the
    network's out_scale (1 + slope (1 - a)) sampled at the knots, each knot value in turn is
    multiplied by a few factors and the change is kept when the worst max |P / P_3x - 1| over the
    training seeds and outputs a_outs drops (coordinate descent; coarse factors first, then fine).
    Sets the schedule on the network (with the slope folded in) and returns (knot values, worst
    error, log of accepted moves)."""
    n_pk = n_pk or n_part * 3
    n_bins = n_pk // 2
    prob1 = make_problem(box, n_part, 1, z_init, n_steps)
    prob3 = make_problem(box, n_part, 3, z_init, n_steps)
    refs = [run_spectra(prob3, cosmo, s, a_outs, n_pk, n_bins) for s in seeds]
    knot_a = [float(a) for a in knot_a]
    vals = [1.0 + net.out_scale_slope * (1.0 - a) for a in knot_a]
    net.set_scales(net.in_scale, net.out_scale, 0.0)

    def worst(v):
        net.set_schedule(knot_a, v)
        w = 0.0
        for s, ref in zip(seeds, refs):
            got = run_spectra(prob1, cosmo, s, a_outs, n_pk, n_bins, net=net)
            for (k, p3), (_, plc) in zip(ref, got):
                w = max(w, max_error(k, plc, p3, k_max))
        return w

    best = worst(vals)
    moves = []
    for rnd in range(rounds):
        improved = False
        for i in range(len(knot_a)):
            for m in ((0.8, 0.9, 1.1, 1.25) if rnd < 2 else (0.93, 0.97, 1.03, 1.07)):
                trial = list(vals)
                trial[i] *= m
                w = worst(trial)
                if w < best - 1e-5:
                    best, vals, improved = w, trial, True
                    moves.append((rnd, i, m, w))
                    if log:
                        log(f"[schedule] round {rnd} knot a={knot_a[i]:.2f} x{m}: worst {w:.4f}")
        if not improved and rnd >= 2:
            break
    net.set_schedule(knot_a, vals)
    return vals, best, moves


def calibrate_green_filter(net, cosmo, box, n_part, z_init, n_steps, seeds, u_knots, a_outs=(1.0,), n_pk=None,
                           k_max=1.0, p_norms=(2, 2, 4, 4, 4, 6, 6, 6), h=0.04, smooth=0.1, n_fixed=1,
                           seed_mean=False, mean_weight=0.0, log=None):
    """Trajectory-level calibration of the corrected step's Green's-function transfer T(u, a)
    together with the output-scale schedule, on training realizations.  Parameters: T at every
    (schedule knot a_i, u_j) beyond the first n_fixed knots and the schedule's knot values; T = 1 at
    the first n_fixed knots (the first one is u = 0): the long-wavelength force, and with it the
    linear growth, stays the PM force's; residuals: P / P_3x - 1 in every bin
    with 0 < k < k_max at every output of every seed.  One Levenberg-Marquardt step per entry of
    p_norms on the p-norm of the residuals (iteratively reweighted least squares, weights
    (|r| / max |r|)^(p - 2): least squares first, then larger p, which approaches the worst case
    that the target bounds), with a forward-difference Jacobian (step h) and a second-difference
    penalty in u and in a (weight `smooth`) that keeps T smooth.  A step is taken when it lowers
    that p-norm; the parameters with the smallest worst |P / P_3x - 1| seen are kept.  seed_mean:
    the residuals are the errors averaged over the seeds bin by bin (the systematic part, which a
    transfer can remove; each realization adds its own scatter of a few per mille near k_max);
    mean_weight > 0: every seed's residuals and, appended with that weight, the seed-averaged ones.  Sets the filter and schedule on the network and returns (u_knots, rows, knot_v,
    worst error, history)."""
    n_pk = n_pk or n_part * 3
    n_bins = n_pk // 2
    prob1 = make_problem(box, n_part, 1, z_init, n_steps)
    prob3 = make_problem(box, n_part, 3, z_init, n_steps)
    refs = [run_spectra(prob3, cosmo, s, a_outs, n_pk, n_bins) for s in seeds]
    sched = net.schedule
    if sched is None:
        raise ValueError("the network needs an output-scale schedule (its knots carry T's rows)")
    knot_a, knot_v = [float(v) for v in sched[0]], [float(v) for v in sched[1]]
    if float(u_knots[0]) != 0.0:
        raise ValueError("the first knot of the transfer is u = 0")
    na, nu = len(knot_a), len(u_knots) - n_fixed  # free values per row
    theta = np.concatenate([np.ones(na * nu), np.asarray(knot_v)])
    start = net.green_filter
    if start is not None and list(start[0]) == [float(np.float32(u)) for u in u_knots]:
        theta[:na * nu] = np.asarray([r[n_fixed:] for r in start[1][:na]]).ravel()

    def rows_of(th):
        return [[1.0] * n_fixed + list(th[i * nu:(i + 1) * nu]) for i in range(na)]

    def apply(th):
        net.set_green_filter(list(u_knots), rows_of(th))
        net.set_schedule(knot_a, list(th[na * nu:]))

    def resid(th):
        apply(th)
        out = []
        for s, ref in zip(seeds, refs):
            got = run_spectra(prob1, cosmo, s, a_outs, n_pk, n_bins, net=net)
            for (k, p3), (_, pl) in zip(ref, got):
                sel = (k > 0) & (k < k_max) & (p3 > 0)
                out.append(pl[sel] / p3[sel] - 1.0)
        per_seed = np.asarray(out).reshape(len(seeds), len(a_outs), -1)
        if seed_mean:
            return per_seed.mean(axis=0).ravel()
        if mean_weight > 0.0:
            return np.concatenate([per_seed.ravel(), mean_weight * per_seed.mean(axis=0).ravel()])
        return per_seed.ravel()

    def pnorm(r, p):
        m = np.abs(r).max()
        return float(m * np.mean((np.abs(r) / m) ** p) ** (1.0 / p))

    # second differences of T along u (within each row) and along a (within each column)
    rows_d = []
    for i in range(na):
        for j in range(1, nu - 1):
            e = np.zeros(theta.size)
            e[i * nu + j - 1], e[i * nu + j], e[i * nu + j + 1] = 1.0, -2.0, 1.0
            rows_d.append(e)
    for j in range(nu):
        for i in range(1, na - 1):
            e = np.zeros(theta.size)
            e[(i - 1) * nu + j], e[i * nu + j], e[(i + 1) * nu + j] = 1.0, -2.0, 1.0
            rows_d.append(e)
    D = np.asarray(rows_d)
    n_seed_res = None

    def worst_of(rv):
        # the worst error of the realizations themselves (not of the appended weighted means)
        return float(np.abs(rv[:n_seed_res]).max()) if n_seed_res else float(np.abs(rv).max())

    r = resid(theta)
    if mean_weight > 0.0 and not seed_mean:
        n_seed_res = r.size * len(seeds) // (len(seeds) + 1)
    best_theta, best = theta.copy(), worst_of(r)
    history = [(0, best)]
    if log:
        log(f"[green] start: worst {best:.4f}, rms {np.sqrt(np.mean(r ** 2)):.4f}")
    for it, p_norm in enumerate(p_norms):
        J = np.empty((r.size, theta.size))
        for q in range(theta.size):
            tp = theta.copy()
            tp[q] += h
            J[:, q] = (resid(tp) - r) / h
        w = (np.abs(r) / np.abs(r).max()) ** (p_norm - 2.0)
        w = w / float(np.mean(w))  # mean weight 1: the penalty keeps its weight across p
        JW = J * w[:, None]
        JtJ = JW.T @ J
        lm = float(np.mean(np.diag(JtJ)))
        taken = False
        for mu in (1e-3, 1e-2, 1e-1, 1.0):
            A = JtJ + smooth * (D.T @ D) + mu * lm * np.eye(theta.size)
            step = np.linalg.solve(A, -(JW.T @ r + smooth * (D.T @ (D @ theta))))
            trial = theta + step
            rt = resid(trial)
            wt = worst_of(rt)
            if log:
                log(f"[green] step {it} (p = {p_norm}) damping {mu:g}: worst {wt:.4f}, "
                    f"rms {np.sqrt(np.mean(rt ** 2)):.4f}")
            if pnorm(rt, p_norm) < pnorm(r, p_norm):
                theta, r, taken = trial, rt, True
                if wt < best:
                    best_theta, best = trial.copy(), wt
                history.append((it + 1, wt))
                break
        if not taken and p_norm == p_norms[-1]:
            break
    apply(best_theta)
    return list(u_knots), rows_of(best_theta), list(best_theta[na * nu:]), best, history
