"""Surrogate runtime: data from the Monte Carlo, training, error calibration
and the predict-or-Monte-Carlo decision.

The thermal side of the paper's hybrid iteration (coupling paragraph) needs
the electron MC's per-subcell heat generation for every new lattice
temperature field.  The surrogate learns that map from runs of the MC itself
and hands the query back to the MC whenever its own predicted error exceeds
the tolerance or the query leaves the training box.  The Monte Carlo runs
and the network's forward, backward and Adam steps run in libgfmc.so
(batched MC contexts, BF16 MFMA kernels).  Around them this module does the
batch bookkeeping in NumPy on the host: the target encoding (unit shape and
log-norm per map) and its decoding, the predicted error from the ensemble
spread, its calibration on held-out points, the training-box check and the
data statistics for z-scoring.  The decoding and the predicted error follow
the same definitions as the library's one-query entry point
sg_predict_or_mc, and are checked against the oracle's.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import gfmc
from . import workloads as W

N_CELL = 1800


def features(cfg: dict) -> np.ndarray:
    """(Vgs, Vds, log10 doping [cm^-3], per-subcell lattice temperature)."""
    T = cfg.get("T_cells")
    T = np.full(N_CELL, cfg["T0_K"]) if T is None else np.asarray(T, np.float64)
    return np.concatenate([[cfg["Vgs"], cfg["Vds"], math.log10(cfg["N_D_m3"] * 1e-6)], T]).astype(np.float32)


def generate(cfgs: list[dict], warm_intervals: int, window_intervals: int, max_instances: int = 64,
             log=print) -> tuple[np.ndarray, np.ndarray, float]:
    """Run the MC for every bias point (batched contexts of up to
    `max_instances` instances; each instance keeps its own seed, doping, bias
    and temperature map) and return the inputs, the window-averaged maps
    (heat W/m^3, then electron density m^-3) and the GPU seconds spent."""
    import torch
    X = np.stack([features(c) for c in cfgs])
    Y = np.zeros((len(cfgs), 2 * N_CELL), np.float32)
    t0 = time.perf_counter()
    for s in range(0, len(cfgs), max_instances):
        chunk = [dict(c, instance=i) for i, c in enumerate(cfgs[s:s + max_instances])]
        K = chunk[0]["substeps"]
        ens = gfmc.Ensemble(chunk)
        ens.mc_step(warm_intervals * K)
        for i in range(len(chunk)):
            ens.mc_tally(i, reset_window=(i == len(chunk) - 1))
        ens.mc_step(window_intervals * K)
        for i in range(len(chunk)):
            m = ens.mc_maps(i)
            Y[s + i, :N_CELL] = m["heat_Wm3"]
            Y[s + i, N_CELL:] = m["density_m3"]
        ens.close()
        torch.cuda.synchronize()
        log(f"  generated {min(s + max_instances, len(cfgs))}/{len(cfgs)} bias points "
            f"({time.perf_counter() - t0:.1f} s)")
    return X, Y, time.perf_counter() - t0


def rel_l2(pred: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Relative L2 error per row of each map (heat, density): shape [n, 2]."""
    pred, ref = np.asarray(pred, np.float64), np.asarray(ref, np.float64)
    out = np.zeros((pred.shape[0], 2))
    for k, sl in enumerate((slice(0, N_CELL), slice(N_CELL, 2 * N_CELL))):
        out[:, k] = np.linalg.norm(pred[:, sl] - ref[:, sl], axis=1) / np.maximum(
            np.linalg.norm(ref[:, sl], axis=1), 1e-300)
    return out


# Target encoding.  Across bias points and doping the maps span orders of
# magnitude, while the accuracy asked for is relative per map: each map is
# learned as its unit-norm shape (1800 values) and the logarithm of its norm,
# so that a squared error in the shape is a relative error of the map.
N_ENC = 2 * N_CELL + 2
# the two log-norms' scale is divided by this in the loss (loss weight = its square)
LOGNORM_WEIGHT = 1.0


def encode(Y: np.ndarray) -> np.ndarray:
    Y = np.asarray(Y, np.float64)
    out = np.zeros((Y.shape[0], N_ENC))
    for k, sl in enumerate((slice(0, N_CELL), slice(N_CELL, 2 * N_CELL))):
        nrm = np.maximum(np.linalg.norm(Y[:, sl], axis=1), 1e-300)
        out[:, sl] = Y[:, sl] / nrm[:, None]
        out[:, 2 * N_CELL + k] = np.log(nrm)
    return out


def decode(T: np.ndarray) -> np.ndarray:
    T = np.asarray(T, np.float64)
    Y = np.zeros((T.shape[0], 2 * N_CELL))
    for k, sl in enumerate((slice(0, N_CELL), slice(N_CELL, 2 * N_CELL))):
        Y[:, sl] = T[:, sl] * np.exp(T[:, 2 * N_CELL + k])[:, None]
    return Y


def encoded_spread(mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    """Raw predicted relative error per row from the ensemble spread of the
    encoded outputs: shape spread over shape norm combined with the spread
    of the log-norm, the larger of the two maps."""
    mean, std = np.asarray(mean, np.float64), np.asarray(std, np.float64)
    out = np.zeros(mean.shape[0])
    for k, sl in enumerate((slice(0, N_CELL), slice(N_CELL, 2 * N_CELL))):
        rs = np.linalg.norm(std[:, sl], axis=1) / np.maximum(np.linalg.norm(mean[:, sl], axis=1), 1e-300)
        out = np.maximum(out, np.hypot(rs, std[:, 2 * N_CELL + k]))
    return out


class Surrogate:
    """Ensemble MLP on the library's BF16 MFMA kernels, with calibrated
    predicted error and Monte Carlo fallback."""

    def __init__(self, width=1024, depth=4, ensemble=4, max_batch=256, seed=1707_09073, tol=0.02,
                 weight_decay=0.0, lognorm_weight=LOGNORM_WEIGHT, shared_scale=True):
        self.net = gfmc.SurrogateNet(3 + N_CELL, N_ENC, width=width, depth=depth, ensemble=ensemble,
                                     max_batch=max_batch, seed=seed, weight_decay=weight_decay)
        self.lognorm_weight = lognorm_weight
        # shared_scale: one scale per map for its shape block and its log-norm
        # (the latter divided by lognorm_weight), so that the squared error
        # of each map's block is its squared relative L2 error; per-cell
        # z-scores instead up-weight the noisy near-zero cells of the heat map
        # and overfit
        self.shared_scale = shared_scale
        self.ensemble = ensemble
        self.max_batch = max_batch
        self.tol = tol
        self.calib = 1.0
        self.box = None

    def fit(self, X: np.ndarray, Y: np.ndarray, epochs: int = 2000, batch: int = 128, lr: float = 3e-4,
            seed: int = 0, log=print) -> list[float]:
        import torch
        T = encode(Y)
        # statistics in FP64 (densities ~1e24 m^-3 would overflow FP32 squared)
        X64 = X.astype(np.float64)
        xm, xs = X64.mean(0), X64.std(0)
        xs = np.where(xs > 1e-6 * np.maximum(1.0, np.abs(xm)), xs, 1.0)
        ym, ys = T.mean(0), T.std(0)
        ys = np.where(ys > 1e-9, ys, 1.0)
        if self.shared_scale:
            for k, sl in enumerate((slice(0, N_CELL), slice(N_CELL, 2 * N_CELL))):
                s_map = float(np.sqrt(np.mean(T[:, sl].var(axis=0))))
                ys[sl] = s_map
                ys[2 * N_CELL + k] = s_map
        ys[2 * N_CELL:] /= self.lognorm_weight
        self.net.sg_set_normalization(xm, xs, ym, ys)
        self.box = (X.min(0), X.max(0))
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        batch = min(batch, self.max_batch, n)
        Td = torch.tensor(T.astype(np.float32), device="cuda")
        Xd_all = torch.tensor(X, device="cuda")
        losses = []
        for ep in range(epochs):
            # cosine learning-rate schedule
            lr_e = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))
            for e in range(self.ensemble):
                perm = torch.tensor(rng.permutation(n), device="cuda")
                Xd, Yd = Xd_all[perm], Td[perm]
                for s in range(0, n - batch + 1, batch):
                    self.net.sg_train_step(e, Xd[s:s + batch], Yd[s:s + batch], lr_e, want_loss=False)
            if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
                losses.append(float(np.mean([self.net.sg_backward(e, Xd_all[:batch], Td[:batch])
                                             for e in range(self.ensemble)])))
                log(f"  epoch {ep}: train loss {losses[-1]:.4g}")
        return losses

    def predict_encoded(self, X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        import torch
        means, stds = [], []
        for s in range(0, X.shape[0], self.max_batch):
            xd = torch.tensor(X[s:s + self.max_batch], device="cuda")
            m = torch.empty((xd.shape[0], N_ENC), device="cuda")
            sd = torch.empty_like(m)
            self.net.sg_predict(xd, m, sd)
            means.append(m.cpu().numpy())
            stds.append(sd.cpu().numpy())
        return np.concatenate(means), np.concatenate(stds)

    def predict(self, X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        """Maps (heat W/m^3, density m^-3) and the raw predicted relative
        error of each row."""
        m, s = self.predict_encoded(X)
        return decode(m), encoded_spread(m, s)

    def calibrate(self, Xv: np.ndarray, Yv: np.ndarray) -> float:
        """Scale the spread so that it bounds the observed validation error
        for 90% of the points."""
        maps, sp = self.predict(Xv)
        err = rel_l2(maps, Yv).max(axis=1)
        self.calib = float(np.quantile(err / np.maximum(sp, 1e-12), 0.9))
        return self.calib

    def in_box(self, X: np.ndarray) -> np.ndarray:
        lo, hi = self.box
        pad = 1e-6 * np.maximum(1.0, np.abs(hi - lo))
        return np.all((X >= lo - pad) & (X <= hi + pad), axis=1)

    def predict_or_mc(self, cfgs: list[dict], warm_intervals: int, window_intervals: int, log=print):
        """Surrogate maps where the calibrated predicted error is within
        tolerance and the query is inside the training box; the Monte Carlo
        for the rest.  Returns (maps, used_mc mask, predicted error)."""
        X = np.stack([features(c) for c in cfgs])
        maps, sp = self.predict(X)
        perr = self.calib * sp
        use_mc = (perr > self.tol) | ~self.in_box(X)
        if np.any(use_mc):
            idx = np.nonzero(use_mc)[0]
            _, Ymc, _ = generate([cfgs[i] for i in idx], warm_intervals, window_intervals, log=log)
            maps[idx] = Ymc
        return maps, use_mc, perr
