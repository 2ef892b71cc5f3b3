"""Train the learned coarse-mesh force correction and write its weights (needs a GPU).

    python paper_1509_04685_amd/train_lc.py [--channels 16] [--out paper_1509_04685_amd/lc_weights_c16.json]

Training pairs: plain PM_grid = 3 runs of 128^3 particles in a 384 h^-1 Mpc box (the resolution,
3 h^-1 Mpc per coarse cell, of the 256^3 / 768 h^-1 Mpc learned workload), 40 nodes from z = 19,
seeds 3001-3006 for training and 3007 for validation, every other node.  The network sees the
density only (the force channels' input scales are zero): its response to a long-wavelength mode
is then a local stencil of the density, of order k^2 g, so it cannot rescale the large-scale force
and bias the growth of large scales (with the force as input it did, by 1-2 % in P(k) at
k ~ 0.2-0.3 h/Mpc).  After the force-level fit, the output scale is calibrated at trajectory level
on training seeds 3001-3004 against the plain 3x runs at every output (a = 0.5, 2/3, 1): first a
factor and slope on a grid, then a piecewise-linear schedule over a (seven knots, coordinate
descent), each minimising the worst max |P / P_3x - 1| for k < 1 over seeds and outputs.
Optional on-policy rounds (--onpolicy-rounds): the calibrated network runs the
coarse form on the training seeds, the positions it visits get fine-mesh targets, the network is
fine-tuned on the old and new samples together and calibrated again.  The weights file holds the flat
FP32 parameters in the library's order, the input and output scales (fitted and calibrated), the
validation loss before and after training, the calibration table and the recipe.

    python paper_1509_04685_amd/train_lc.py --calibrate-filter paper_1509_04685_amd/lc_weights_c16.json

calibrates, for an existing weights file, a radial transfer T(|k| / k_Nyquist, a) of the corrected
step's Green's function together with the schedule (damped Gauss-Newton on the p-norm, p = 8, of
the errors of every P(k) bin with k < 1 h/Mpc of the training seeds 3001-3004 at every output) and
writes it into the file.
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

RECIPE = dict(box=384.0, n_part=128, pm_fine=3, n_steps=40, z_init=19.0,
              train_seeds=(3001, 3002, 3003, 3004, 3005, 3006), val_seeds=(3007,),
              train_nodes=tuple(range(4, 40, 2)), val_nodes=tuple(range(5, 40, 6)),
              iters=3000, batch=2, lr=3e-3, lr_decay=0.3, chunks=5, init_seed=1, force_input=False,
              calib_seeds=(3001, 3002, 3003, 3004), calib_factors=tuple(round(0.3 + 0.1 * i, 2) for i in range(14)),
              calib_slopes=tuple(round(-0.8 + 0.2 * i, 1) for i in range(9)),
              calib_a=(0.5, 2.0 / 3.0, 1.0), knot_a=(0.05, 0.2, 0.35, 0.5, 0.65, 0.8, 1.0), knot_rounds=5,
              onpolicy_rounds=0, onpolicy_iters=1500, onpolicy_lr=1e-3,
              onpolicy_factors=tuple(round(0.9 + 0.05 * i, 2) for i in range(13)),
              onpolicy_slopes=tuple(round(-0.2 + 0.2 * i, 1) for i in range(6)))


# knots of the Green's-function transfer in |k| / k_Nyquist of the coarse mesh (the last one covers
# the mesh corners)
FILTER_U = (0.0, 0.12, 0.25, 0.38, 0.5, 0.62, 0.74, 0.86, 0.98, 1.3)
FILTER_FIXED = 1  # T = 1 (with zero slope) at u = 0: the large-scale force stays the PM force


def train(channels, recipe=RECIPE, log=print):
    import paper_1509_04685_amd as cola
    from paper_1509_04685_amd import learned as L, workloads as W
    r = recipe
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    t0 = time.time()
    samples = L.make_samples(cosmo, r["box"], r["n_part"], r["pm_fine"], r["n_steps"], r["z_init"],
                             r["train_seeds"], nodes=set(r["train_nodes"]))
    val = L.make_samples(cosmo, r["box"], r["n_part"], r["pm_fine"], r["n_steps"], r["z_init"],
                         r["val_seeds"], nodes=set(r["val_nodes"]))
    log(f"[train_lc] {len(samples)} training and {len(val)} validation samples ({time.time() - t0:.1f} s)")
    net = L.new_net(samples[-1], channels=channels, seed=r["init_seed"], force_input=r["force_input"])
    tr = L.Trainer(net, r["n_part"], r["box"])
    v0 = tr.evaluate(val)
    per = r["iters"] // r["chunks"]
    for c in range(r["chunks"]):
        h = tr.train(samples, per, r["lr"] * r["lr_decay"] ** c, batch=r["batch"], seed=c)
        log(f"[train_lc] chunk {c}: mean training loss {h.mean():.4f}, validation {tr.evaluate(val):.4f} "
            f"({time.time() - t0:.1f} s)")
    fitted = net.out_scale
    v1 = tr.evaluate(val)
    best, slope, table = L.calibrate_out_scale(net, cosmo, r["box"], r["n_part"], r["z_init"], r["n_steps"],
                                               r["calib_seeds"], r["calib_factors"], r["calib_slopes"], log=log,
                                               a_outs=r["calib_a"])
    log(f"[train_lc] output scale {fitted:.5g} -> {best:.5g} (factor {best / fitted:.3f}), slope {slope:+.2f}; "
        f"worst training-seed error {min(t[2] for t in table):.4f}")
    for rd in range(r["onpolicy_rounds"]):
        onp = L.make_samples(cosmo, r["box"], r["n_part"], r["pm_fine"], r["n_steps"], r["z_init"],
                             r["train_seeds"], nodes=set(r["train_nodes"]), net=net)
        net.set_scales(net.in_scale, fitted, 0.0)  # fine-tune at the fitted scale, calibrate again after
        data = samples + onp
        per = r["onpolicy_iters"] // 3
        for c in range(3):
            h = tr.train(data, per, r["onpolicy_lr"] * 0.3 ** c, batch=r["batch"], seed=1000 * (rd + 1) + c)
            log(f"[train_lc] on-policy round {rd} chunk {c}: mean training loss {h.mean():.4f}, validation "
                f"{tr.evaluate(val):.4f} ({time.time() - t0:.1f} s)")
        v1 = tr.evaluate(val)
        del onp, data
        best, slope, table = L.calibrate_out_scale(net, cosmo, r["box"], r["n_part"], r["z_init"], r["n_steps"],
                                                   r["calib_seeds"], r["onpolicy_factors"], r["onpolicy_slopes"],
                                                   log=log, a_outs=r["calib_a"])
        log(f"[train_lc] on-policy round {rd}: factor {best / fitted:.3f}, slope {slope:+.2f}; worst training-seed "
            f"error {min(t[2] for t in table):.4f}")
    del samples, val
    if r["knot_rounds"] > 0:
        vals, worst, _ = L.calibrate_schedule(net, cosmo, r["box"], r["n_part"], r["z_init"], r["n_steps"],
                                              r["calib_seeds"], r["knot_a"], a_outs=r["calib_a"],
                                              rounds=r["knot_rounds"], log=log)
        log(f"[train_lc] schedule {[round(v, 3) for v in vals]} at a = {list(r['knot_a'])}: worst training-seed "
            f"error {worst:.4f}")
    return net, v0, v1, fitted, table


def calibrate_filter_file(path, recipe=RECIPE, log=print, n_part=None, seeds=None, p_norms=None, seed_mean=False,
                          mean_weight=0.0):
    """The Green's-function transfer of the corrected step (T at the schedule's knots in a and at
    FILTER_U in |k| / k_Nyquist), calibrated with the schedule by damped Gauss-Newton on the
    training seeds' trajectories (every output a), written into the weights file."""
    import paper_1509_04685_amd as cola
    from paper_1509_04685_amd import learned as L, workloads as W
    r = recipe
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    net, doc = L.load_net(path)
    t0 = time.time()
    # the same 3 h^-1 Mpc cells as the training pairs, in a box scaled with the particle count
    n_part = n_part or r["n_part"]
    box = r["box"] * n_part / r["n_part"]
    seeds = tuple(seeds or r["calib_seeds"])
    extra = {} if p_norms is None else {"p_norms": tuple(p_norms)}
    u, rows, knot_v, worst, hist = L.calibrate_green_filter(
        net, cosmo, box, n_part, r["z_init"], r["n_steps"], seeds, FILTER_U,
        a_outs=r["calib_a"], n_fixed=FILTER_FIXED, seed_mean=seed_mean, mean_weight=mean_weight, log=log, **extra)
    log(f"[train_lc] Green's-function transfer calibrated: worst training-seed error {worst:.4f} "
        f"({time.time() - t0:.1f} s)")
    prev = doc.get("green_filter") or {}
    passes = prev.get("passes", []) if list(prev.get("u", [])) == list(u) else []
    passes.append({"seeds": list(seeds), "n_part": n_part, "box": box, "seed_mean": seed_mean,
                   "mean_weight": mean_weight,
                   "worst_training_error": worst, "history": hist})
    doc["green_filter"] = {"u": u, "t": rows, "worst_training_error": worst, "a_outs": list(r["calib_a"]),
                           "passes": passes}
    doc["schedule"] = [net.schedule[0], knot_v]
    with open(path, "w") as fh:
        json.dump(doc, fh)
    log(f"[train_lc] wrote {path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--channels", type=int, default=16)
    ap.add_argument("--out", default=None)
    ap.add_argument("--iters", type=int, default=RECIPE["iters"])
    ap.add_argument("--onpolicy-rounds", type=int, default=RECIPE["onpolicy_rounds"])
    ap.add_argument("--force-input", action="store_true", help="the network also sees the three force components")
    ap.add_argument("--calibrate-filter", metavar="WEIGHTS", default=None,
                    help="calibrate the Green's-function transfer (and the schedule) of an existing weights "
                         "file on the training seeds and write it back (no training)")
    ap.add_argument("--calib-n-part", type=int, default=None,
                    help="particles per side of the filter calibration runs (box scaled to keep 3 h^-1 Mpc cells)")
    ap.add_argument("--calib-seeds", type=int, nargs="*", default=None,
                    help="training seeds of the filter calibration (default: the recipe's calibration seeds)")
    ap.add_argument("--calib-p", type=float, nargs="*", default=None,
                    help="p of the p-norm of each calibration step (default 2 2 4 4 4 6 6 6)")
    ap.add_argument("--calib-seed-mean", action="store_true",
                    help="fit the errors averaged over the calibration seeds (their systematic part)")
    ap.add_argument("--calib-mean-weight", type=float, default=0.0,
                    help="also fit the seed-averaged errors, with this weight, beside every seed's")
    args = ap.parse_args()
    if args.calibrate_filter:
        calibrate_filter_file(args.calibrate_filter, log=lambda m: print(m, flush=True), n_part=args.calib_n_part,
                              seeds=args.calib_seeds, p_norms=args.calib_p, seed_mean=args.calib_seed_mean,
                              mean_weight=args.calib_mean_weight)
        return
    out = args.out or os.path.join(HERE, f"lc_weights_c{args.channels}.json")
    recipe = dict(RECIPE, iters=args.iters, onpolicy_rounds=args.onpolicy_rounds,
                  force_input=args.force_input)
    net, v0, v1, fitted, table = train(args.channels, recipe=recipe, log=lambda m: print(m, flush=True))
    doc = dict(channels=net.channels, in_scale=list(net.in_scale), out_scale=net.out_scale,
               out_scale_slope=net.out_scale_slope, out_scale_fitted=fitted, calibration=table,
               schedule=net.schedule,
               val_loss_initial=v0, val_loss_trained=v1, recipe=recipe,
               params=[float(x) for x in net.get_params()])
    with open(out, "w") as fh:
        json.dump(doc, fh)
    print(f"[train_lc] wrote {out}: validation loss {v0:.4f} -> {v1:.4f}", flush=True)


if __name__ == "__main__":
    main()
