"""Train the learned coarse-mesh force correction and write its weights (needs a GPU).

    python paper_1509_04685_amd/train_lc.py [--channels 16] [--out paper_1509_04685_amd/lc_weights_c16.json]

Training pairs: plain PM_grid = 3 runs of 128^3 particles in a 384 h^-1 Mpc box (the resolution,
3 h^-1 Mpc per coarse cell, of the 256^3 / 768 h^-1 Mpc learned workload), 40 nodes from z = 19,
seeds 3001-3006 for training and 3007 for validation, every other node.  After the force-level
fit, the output scale is calibrated at trajectory level on training seeds 3001-3002 (the factor
that minimises the worst max |P / P_3x - 1| for k < 1 at z = 0).  The weights file holds the flat
FP32 parameters in the library's order, the input and output scales (fitted and calibrated), the
validation loss before and after training, the calibration table and the recipe.
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
              iters=1500, batch=2, lr=3e-3, lr_decay=0.3, chunks=5, init_seed=1,
              calib_seeds=(3001, 3002), calib_factors=tuple(round(1.2 + 0.05 * i, 2) for i in range(11)),
              calib_slopes=tuple(round(-0.6 + 0.2 * i, 1) for i in range(7)))


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
    net = L.new_net(samples[-1], channels=channels, seed=r["init_seed"])
    tr = L.Trainer(net, r["n_part"], r["box"])
    v0 = tr.evaluate(val)
    per = r["iters"] // r["chunks"]
    for c in range(r["chunks"]):
        h = tr.train(samples, per, r["lr"] * r["lr_decay"] ** c, batch=r["batch"], seed=c)
        log(f"[train_lc] chunk {c}: mean training loss {h.mean():.4f}, validation {tr.evaluate(val):.4f} "
            f"({time.time() - t0:.1f} s)")
    v1 = tr.evaluate(val)
    del samples, val
    fitted = net.out_scale
    best, slope, table = L.calibrate_out_scale(net, cosmo, r["box"], r["n_part"], r["z_init"], r["n_steps"],
                                               r["calib_seeds"], r["calib_factors"], r["calib_slopes"], log=log)
    log(f"[train_lc] output scale {fitted:.5g} -> {best:.5g} (factor {best / fitted:.3f}), slope {slope:+.2f}; "
        f"worst training-seed error {min(t[2] for t in table):.4f}")
    return net, v0, v1, fitted, table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--channels", type=int, default=16)
    ap.add_argument("--out", default=None)
    ap.add_argument("--iters", type=int, default=RECIPE["iters"])
    args = ap.parse_args()
    out = args.out or os.path.join(HERE, f"lc_weights_c{args.channels}.json")
    recipe = dict(RECIPE, iters=args.iters)
    net, v0, v1, fitted, table = train(args.channels, recipe=recipe, log=lambda m: print(m, flush=True))
    doc = dict(channels=net.channels, in_scale=list(net.in_scale), out_scale=net.out_scale,
               out_scale_slope=net.out_scale_slope, out_scale_fitted=fitted, calibration=table,
               val_loss_initial=v0, val_loss_trained=v1, recipe=recipe,
               params=[float(x) for x in net.get_params()])
    with open(out, "w") as fh:
        json.dump(doc, fh)
    print(f"[train_lc] wrote {out}: validation loss {v0:.4f} -> {v1:.4f}", flush=True)


if __name__ == "__main__":
    main()
