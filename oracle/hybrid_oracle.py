"""FP64 reference of the electro-thermal iteration of the coupling paragraph
(Hao, Zhao, Xiao and Kronenfeld, arXiv:1707.09073) and of the device
thermal resistance of the thermal-resistance passage.

TEST INFRASTRUCTURE ONLY: used by the tests; the GPU product path never
imports it.  It composes the reference electron Monte Carlo (emc_oracle),
the reference phonon tables (phonon_oracle) and the reference phonon packet
run (emc_oracle.phonon_mc) in the paper's order:

  1. electrons at the current lattice temperature: settle, then a window;
     its net phonon-emission map is the heat generated per subcell;
  2. phonon packets from that heat (tables linearised at T_lin) give the
     temperature rise dT per subcell over the isothermal faces' T_sink;
  3. T_new = T_sink + dT; the lattice temperature moves to
     T + relax (T_new - T) and sets the electron rates again;

until no subcell moves by more than tol_K or after max_iterations.  The
thermal resistance of an iteration is max dT over the emitted phonon power
(emission only) of its window.  The phonon domain of an instance is its own
box and subcells.

With a chip (the Fourier's-law stage of the coupling paragraph), every
wire of the array takes the instance's heat map, the chip's steady
conduction problem is solved (fourier_oracle), and the chip's temperature
below each subcell column replaces T_sink in step 3.
"""
from __future__ import annotations

import numpy as np

from oracle import emc_oracle as E
from oracle import fourier_oracle as F
from oracle import phonon_oracle as P


def _mean(x) -> float:
    s = 0.0
    for v in x:
        s += float(v)
    return s / len(x)


def hybrid(mc_cfgs: list[dict], hy: dict, heat0_Wm3=None, threads: int = 0, chip: dict | None = None) -> dict:
    """mc_cfgs: device-mode instance configurations (emc_oracle.make_config
    keys; a T_cells entry sets the starting temperature); hy: mat (Table II
    dict), electrons (dict or None), n_bins, faces, max_events, n_packets,
    seed, T_sink_K, T_lin_K (<= 0: the instance's mean subcell temperature
    at the iteration's start), warmup_intervals, window_intervals,
    max_iterations, relax, tol_K.  heat0_Wm3 ([n_inst][ncell] or None): a
    warm-start heat map for the first iteration.  chip (or None): fo (n,
    dirichlet, k_interface, R_K_m2KW), edges, material, src_index,
    base_index, kappa_by_material, half_wires.  Returns the records (one per
    instance and iteration, as the library's hy_record), the iterations
    done, the final temperatures, and per record the dT map."""
    ors = [E.Oracle(c) for c in mc_cfgs]
    n = len(ors)
    nc = ors[0].ncell
    T = []
    for c in mc_cfgs:
        t0 = c.get("T_cells")
        T.append(np.array(t0, dtype=np.float64) if t0 is not None else np.full(nc, float(c["T0_K"])))
    records, maps = [], []
    done = 0
    for it in range(int(hy["max_iterations"])):
        warm = it == 0 and heat0_Wm3 is not None
        if not warm:
            for o in ors:
                o.run(int(hy["warmup_intervals"]), threads)
                o.reset_window()
                o.run(int(hy["window_intervals"]), threads)
        worst = 0.0
        for i, o in enumerate(ors):
            cfg = mc_cfgs[i]
            L = np.asarray(cfg["L_nm"], float)
            ncl = np.asarray(cfg["n_cells"], int)
            vc_m3 = (L[0] / ncl[0]) * (L[1] / ncl[1]) * (L[2] / ncl[2]) * 1e-27
            r = dict(iteration=it, instance=i, source=0, steady=0, drain_current_A=0.0, emit_W=0.0)
            if warm:
                r["source"] = 1
                heat = np.asarray(heat0_Wm3, np.float64).reshape(n, nc)[i]
            else:
                ob = o.observables()
                heat, _, _ = o.power_maps()
                r.update(steady=ob["steady"], drain_current_A=ob["I_D"], emit_W=ob["P_emit_W"])
            q = heat * vc_m3
            r["heat_W"] = float(q.sum())
            tl = float(hy.get("T_lin_K", 0.0))
            if not tl > 0.0:
                tl = _mean(T[i])
            r["T_lin_K"] = tl
            w, v, Cb, inv_tau = P.bin_tables(hy["mat"], tl, int(hy["n_bins"]), electrons=hy.get("electrons"))
            pcfg = dict(L_nm=list(L), n_cells=list(ncl), faces=hy["faces"], seed=hy["seed"], instance=i,
                        max_events=int(hy.get("max_events", 1 << 22)))
            ph = E.phonon_mc(pcfg, q, v, inv_tau, Cb, int(hy["n_packets"]), threads)
            dT = ph["dT"]
            base = np.full(nc, float(hy["T_sink_K"]))
            if chip is not None:
                kap = np.asarray(chip["kappa_by_material"], np.float64)[np.asarray(chip["material"])]
                si = np.asarray(chip["src_index"])
                qc = np.where(si >= 0, q[np.maximum(si, 0)], 0.0)
                fcfg = dict(chip["fo"], T_sink_K=hy["T_sink_K"])
                T_chip = F.solve(fcfg, chip["edges"], kap, qc)
                base = T_chip[np.asarray(chip["base_index"])]
            rise = (base - hy["T_sink_K"]) + dT
            T_new = base + dT
            change = float(np.abs(T_new - T[i]).max())
            T[i] = T[i] + hy["relax"] * (T_new - T[i])
            o.set_temperature(T[i])
            mx = float(rise.max())
            r.update(dT_max_K=mx, dT_mean_K=_mean(rise), hot_cell=int(np.argmax(rise)), change_K=change,
                     R_th_KW=mx / r["emit_W"] if r["emit_W"] > 0 else 0.0,
                     packets_absorbed=int(ph["absorbed"].sum()), packets_dropped=int(ph["dropped"]))
            if chip is not None:
                P_dev = chip["half_wires"] * r["emit_W"]
                fmax = float(T_chip.max()) - hy["T_sink_K"]
                r.update(dT_junction_max_K=max(0.0, float((base - hy["T_sink_K"]).max())), dT_fourier_max_K=fmax,
                         R_th_device_KW=mx / P_dev if P_dev > 0 else 0.0,
                         R_th_fourier_KW=fmax / P_dev if P_dev > 0 else 0.0)
            records.append(r)
            maps.append(dT)
            worst = max(worst, change)
        done = it + 1
        if worst <= hy.get("tol_K", 0.0):
            break
    return dict(records=records, iterations=done, T_cells=np.array(T), dT_maps=maps)
