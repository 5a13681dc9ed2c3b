"""Surrogate experiment: train the MLP on Monte Carlo runs of the device and
measure its heat-map error and time per bias point against the plain MC.

    python -m paper_1707_09073_amd.surrogate_experiment --train 12000 --val 200 --out result.json

Training inputs are seeded bias points (Vgs ~ U[-3,0] V, Vds ~ U[1,10] V,
doping log-uniform in [1e17, 1e19] cm^-3) with random drain-side hot spots;
each target is the MC's window-averaged heat and density map.  Held-out
references use `--ref-seeds` independent MC runs averaged, so that their own
noise is below the tolerance.  Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=12000)
    ap.add_argument("--val", type=int, default=200)
    ap.add_argument("--particles", type=int, default=200_000)
    ap.add_argument("--warm", type=int, default=1000, help="intervals (10 fs) before the window")
    ap.add_argument("--window", type=int, default=1000, help="intervals (10 fs) averaged")
    ap.add_argument("--ref-seeds", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=1400)
    ap.add_argument("--width", type=int, default=1024)
    ap.add_argument("--depth", type=int, default=4)
    ap.add_argument("--ensemble", type=int, default=4)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--weight-decay", type=float, default=0.0)
    ap.add_argument("--lognorm-weight", type=float, default=1.0)
    ap.add_argument("--per-cell-scale", action="store_true",
                    help="z-score every output on its own (default: one scale per map)")
    ap.add_argument("--tol", type=float, default=0.02)
    ap.add_argument("--save-data", default="", help="write the Monte Carlo data (.npz) for later fits")
    ap.add_argument("--load-data", default="", help="fit on Monte Carlo data written by --save-data")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)

    import torch
    from . import surrogate as S
    from . import workloads as W

    def log(*x):
        print(*x, file=sys.stderr, flush=True)

    if a.load_data:
        d = np.load(a.load_data)
        X, Y, Xv, Yv, Yv_single = d["X"], d["Y"], d["Xv"], d["Yv"], d["Yv_single"]
        t_train, mc_time_per_point = float(d["t_train"]), float(d["mc_time_per_point"])
        a.train, a.val = X.shape[0], Xv.shape[0]
        a.ref_seeds, a.warm, a.window, a.particles = (int(d[k]) for k in ("ref_seeds", "warm", "window", "particles"))
        log(f"MC data from {a.load_data}: {a.train} training and {a.val} held-out points")
    else:
        train_cfgs = W.surrogate_inputs(a.train, seed=11)
        val_cfgs = W.surrogate_inputs(a.val, seed=23)
        for c in train_cfgs + val_cfgs:
            c["n_particles"] = a.particles
            c["capacity"] = int(a.particles * 1.3)
        log(f"MC training data: {a.train} bias points x {a.particles} electrons, {a.warm}+{a.window} intervals")
        X, Y, t_train = S.generate(train_cfgs, a.warm, a.window, log=log)
        log(f"MC held-out references: {a.val} bias points x {a.ref_seeds} seeds")
        Xv = np.stack([S.features(c) for c in val_cfgs])
        Yv = np.zeros((a.val, 2 * S.N_CELL), np.float32)
        Yv_single = None
        t_ref = 0.0
        for r in range(a.ref_seeds):
            cfgs = [dict(c, seed=c["seed"] + 100003 * (r + 1)) for c in val_cfgs]
            _, Yr, tr = S.generate(cfgs, a.warm, a.window, log=log)
            t_ref += tr
            Yv += Yr / a.ref_seeds
            if Yv_single is None:
                Yv_single = Yr
        mc_time_per_point = t_ref / (a.ref_seeds * a.val)
        if a.save_data:
            np.savez(a.save_data, X=X, Y=Y, Xv=Xv, Yv=Yv, Yv_single=Yv_single, t_train=t_train,
                     mc_time_per_point=mc_time_per_point, ref_seeds=a.ref_seeds, warm=a.warm, window=a.window,
                     particles=a.particles)
    # noise of one MC run against the averaged reference (an estimate of
    # the MC's own error at this ensemble size and window)
    mc_err = S.rel_l2(Yv_single, Yv).max(axis=1) * np.sqrt(a.ref_seeds / max(1, a.ref_seeds - 1))

    sur = S.Surrogate(width=a.width, depth=a.depth, ensemble=a.ensemble, max_batch=256, tol=a.tol,
                      weight_decay=a.weight_decay, lognorm_weight=a.lognorm_weight,
                      shared_scale=not a.per_cell_scale)
    t0 = time.perf_counter()
    losses = sur.fit(X, Y, epochs=a.epochs, batch=128, lr=a.lr, log=log)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    # calibrate the spread on half of the held-out points, evaluate on the other half
    h = a.val // 2
    calib = sur.calibrate(Xv[:h], Yv[:h])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        m, sp = sur.predict(Xv[h:])
    torch.cuda.synchronize()
    t_pred = (time.perf_counter() - t0) / (reps * (a.val - h))
    # single-point latency
    t0 = time.perf_counter()
    for i in range(20):
        sur.predict(Xv[h + (i % (a.val - h)):h + (i % (a.val - h)) + 1])
    torch.cuda.synchronize()
    t_pred1 = (time.perf_counter() - t0) / 20
    err = S.rel_l2(m, Yv[h:])
    perr = sur.calib * sp
    accept = (perr <= a.tol) & sur.in_box(Xv[h:])
    # accuracy / time trade-off of the hybrid (surrogate where the calibrated
    # predicted error is within tolerance, Monte Carlo elsewhere)
    tradeoff = []
    for tol in (0.02, 0.05, 0.10):
        acc = (perr <= tol) & sur.in_box(Xv[h:])
        t_hyb = acc.mean() * t_pred1 + (1 - acc.mean()) * mc_time_per_point
        emax = err[acc].max(axis=1) if acc.any() else np.zeros(0)
        tradeoff.append({"tol": tol, "accepted_fraction": float(acc.mean()),
                         "accepted_within_tol_fraction": float(np.mean(emax <= tol)) if acc.any() else None,
                         "hybrid_seconds_per_point": float(t_hyb),
                         "hybrid_speedup": float(mc_time_per_point / t_hyb)})
    res = {
        "train_points": a.train, "val_points": a.val, "particles": a.particles,
        "warm_intervals": a.warm, "window_intervals": a.window, "ref_seeds": a.ref_seeds,
        "mlp": {"width": a.width, "depth": a.depth, "ensemble": a.ensemble, "epochs": a.epochs, "lr": a.lr,
                "weight_decay": a.weight_decay, "lognorm_weight": a.lognorm_weight,
                "shared_scale": not a.per_cell_scale},
        "mc_seconds_per_bias_point": mc_time_per_point,
        "mc_train_data_seconds": t_train,
        "surrogate_fit_seconds": t_fit,
        "surrogate_seconds_per_point_batched": t_pred,
        "surrogate_seconds_single_point": t_pred1,
        "speedup_batched": mc_time_per_point / t_pred,
        "speedup_single_point": mc_time_per_point / t_pred1,
        "heat_rel_l2_median": float(np.median(err[:, 0])), "heat_rel_l2_p90": float(np.quantile(err[:, 0], 0.9)),
        "density_rel_l2_median": float(np.median(err[:, 1])),
        "density_rel_l2_p90": float(np.quantile(err[:, 1], 0.9)),
        "mc_single_run_rel_l2_median": float(np.median(mc_err)),
        "calibration_factor": calib,
        "accepted_fraction": float(np.mean(accept)),
        "accepted_heat_rel_l2_max": float(err[accept, 0].max()) if accept.any() else None,
        "accepted_within_tol_fraction": float(np.mean(err[accept].max(axis=1) <= a.tol)) if accept.any() else None,
        "fallback_fraction": float(1 - np.mean(accept)),
        "tradeoff": tradeoff,
        "train_loss_curve": losses,
    }
    txt = json.dumps(res)
    print(txt, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
