"""GPU parity of the electro-thermal iteration (coupling paragraph) and the
thermal resistance (thermal-resistance passage) against the FP64 reference
iteration, and the iteration at the full device size."""
import sys

import numpy as np
import pytest

from oracle import hybrid_oracle as H
from oracle import phonon_oracle as P
from paper_1707_09073_amd import workloads as W

pytestmark = pytest.mark.gpu

GAN = P.table2("GaN")
ELEC = dict(n_m3=1e24, m_dos=0.21, D_a_eV=8.3, rho=6095.0, v_g=3338.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1707_09073_amd import gfmc
    gfmc.lib()
    return gfmc


def _hy(**kw):
    h = dict(mat=GAN, electrons=ELEC, n_bins=256, faces=W.WIRE_FACES, n_packets=20000, seed=21, T_sink_K=300.0,
             T_lin_K=0.0, warmup_intervals=6, window_intervals=14, max_iterations=2, relax=0.7, tol_K=0.0)
    h.update(kw)
    return h


EXACT = ("iteration", "instance", "source", "steady", "hot_cell", "packets_absorbed", "packets_dropped")


def _compare(g, o, rel_mc=1e-12, rel_ph=1e-9):
    assert len(g["records"]) == len(o["records"])
    for a, b in zip(g["records"], o["records"]):
        for k in EXACT:
            assert a[k] == b[k], (k, a, b)
        for k in ("drain_current_A", "emit_W", "heat_W", "T_lin_K"):
            assert a[k] == pytest.approx(b[k], rel=rel_mc, abs=1e-30), (k, a[k], b[k])
        for k in ("dT_max_K", "dT_mean_K", "change_K", "R_th_KW"):
            assert a[k] == pytest.approx(b[k], rel=rel_ph, abs=1e-12), (k, a[k], b[k])
    rise_g, rise_o = g["T_cells"] - 300.0, o["T_cells"] - 300.0
    assert np.abs(rise_g - rise_o).max() <= rel_ph * np.abs(rise_o).max()


def test_hybrid_iteration_matches_the_reference(G):
    """Two bias points in one context (Vds = 3 V and 1.5 V), FP64, two
    iterations with under-relaxation and tables re-linearised at the mean
    temperature, Eq. (1) in the relaxation rates.  Integer counts behind
    every window are identical, so currents and powers agree to rounding;
    the packet runs use tables computed on each side (equal to 1e-11), so the
    temperature maps agree to 1e-9."""
    cfgs = [W.device_config(n_particles=4000, precision="fp64", Vds=3.0, seed=101),
            dict(W.device_config(n_particles=3000, precision="fp64", Vds=1.5, seed=102), instance=1)]
    hy = _hy()
    _say("hybrid parity: 2 instances, 2 iterations of 6 + 14 intervals, 20000 packets")
    e = G.Ensemble(cfgs)
    g = G.hy_run(e, hy)
    o = H.hybrid(cfgs, hy)
    assert g["iterations"] == o["iterations"] == 2
    _compare(g, o)
    r = g["records"]
    assert r[0]["emit_W"] > r[1]["emit_W"] > 0 and r[0]["dT_max_K"] > 0


def test_hybrid_warm_start_matches_the_reference(G):
    """The first iteration's source is a given heat map (a surrogate's, say)
    instead of an electron window; then one electron window."""
    cfg = W.device_config(n_particles=4000, precision="fp64", Vds=3.0, seed=103)
    q = np.zeros((100, 18))
    q[68:80] = 3e17
    q[10:14, 9:] = -5e16
    hy = _hy(T_lin_K=330.0, relax=1.0, electrons=None)
    _say("hybrid warm start: 1 instance, warm map then one window")
    e = G.Ensemble(cfg)
    g = G.hy_run(e, hy, heat0_Wm3=q.reshape(1, -1))
    o = H.hybrid([cfg], hy, heat0_Wm3=q.reshape(1, -1))
    _compare(g, o)
    assert g["records"][0]["source"] == 1 and 68 <= g["records"][0]["hot_cell"] // 18 < 80


def test_hybrid_rejects_what_it_cannot_couple(G):
    e = G.Ensemble(W.device_config(n_particles=2000, precision="fp64", seed=104))
    assert G.hy_workspace_bytes(e, _hy()) > 0
    for bad in (dict(relax=0.0), dict(relax=1.5), dict(window_intervals=0), dict(max_iterations=0),
                dict(n_bins=0), dict(n_packets=0), dict(T_sink_K=0.0)):
        assert G.hy_workspace_bytes(e, _hy(**bad)) == 0, bad
        with pytest.raises(G.MCError):
            G.hy_run(e, _hy(**bad))
    b = G.Ensemble(W.bulk_config(n_particles=1000, precision="fp64"))
    assert G.hy_workspace_bytes(b, _hy()) == 0


def test_hybrid_full_device(G):
    """The device at 2e5 electrons, FP32 state: three iterations from 300 K.
    The hot subcell sits on the drain side of the gate, the heat leaves
    through the isothermal faces, the thermal resistance is the largest rise
    over the emitted power, and heating lowers the drain current: the second
    window's current is below that of the same ensemble (same seed, same
    random streams) kept at 300 K over the same intervals (the windows are
    still in the start-up transient, so the currents of successive
    iterations alone do not show it)."""
    cfg = W.device_config(n_particles=200_000, precision="fp32", Vds=5.0, Vgs=0.0, seed=105)
    hy = _hy(n_packets=400_000, warmup_intervals=40, window_intervals=80, max_iterations=3, relax=1.0)
    _say("hybrid full device: 2e5 electrons, 3 iterations of 40 + 80 intervals, 4e5 packets")
    e = G.Ensemble(cfg)
    g = G.hy_run(e, hy)
    recs = g["records"]
    for r in recs:
        _say({k: (float("%.5g" % v) if isinstance(v, float) else v) for k, v in r.items()})
        assert r["packets_absorbed"] == 400_000 and r["packets_dropped"] == 0
        assert r["R_th_KW"] == pytest.approx(r["dT_max_K"] / r["emit_W"], rel=1e-12)
        assert r["emit_W"] > r["heat_W"] > 0
        assert 500 <= (r["hot_cell"] // 18) * 10 < 1000
    assert recs[0]["dT_max_K"] > 20
    c = G.Ensemble(cfg)                                  # the control: never heated
    K = cfg["substeps"]
    c.mc_step(K * (40 + 80 + 40))
    c.mc_tally(reset_window=True)
    c.mc_step(K * 80)
    i_cold = c.mc_observables()["drain_current_A"]
    _say("second window: heated", recs[1]["drain_current_A"], "A, at 300 K", i_cold, "A")
    assert recs[1]["drain_current_A"] < i_cold


def test_hybrid_with_the_chip_matches_the_reference(G):
    """The iteration with the Fourier's-law stage on a small array (five
    wires over a 200 nm channel): each window's heat map heats every wire,
    the chip's junction temperature lifts the packets' rise; records and
    temperatures against the reference iteration (direct chip solves).
    Counts exact; what the chip's temperature enters to 2e-7: the
    conjugate gradients stop at a relative residual of 1e-13, and the error
    of the temperature is that times the operator's condition number (3e-8
    of the rise measured here)."""
    dev = W.device_config(n_particles=3000, precision="fp64", Vds=3.0, n_cells=(20, 3, 6), L_nm=(200.0, 60.0, 120.0),
                          seed=107)
    g = W.chip_geometry(dev, n_wires=5, margin_x_um=0.4, margin_y_um=0.3, film_um=0.3, substrate_um=1.0)
    chip = dict(fo=dict(n=g["n"], dirichlet=[0, 0, 0, 0, 1, 0], k_interface=g["k_interface"], R_K_m2KW=2.3e-8,
                        rtol=1e-13, max_iterations=50000),
                edges=g["edges"], material=g["material"], src_index=g["src_index"], base_index=g["base_index"],
                kappa_by_material=[0.0, 350.0, 125.0, 35.6], half_wires=5)
    hy = _hy(faces=W.WIRE_FACES_ON_CHIP, n_packets=10000, warmup_intervals=4, window_intervals=10)
    _say("hybrid with chip: small device and array, 2 iterations")
    e = G.Ensemble(dev)
    g_run = G.hy_run(e, hy, chip=chip)
    o = H.hybrid([dev], hy, chip=chip)
    _compare(g_run, o, rel_ph=2e-7)
    for a, b in zip(g_run["records"], o["records"]):
        for k in ("dT_junction_max_K", "dT_fourier_max_K", "R_th_device_KW", "R_th_fourier_KW"):
            assert a[k] == pytest.approx(b[k], rel=2e-7), (k, a[k], b[k])
        assert a["fo_iterations"] > 0 and a["dT_junction_max_K"] > 0
