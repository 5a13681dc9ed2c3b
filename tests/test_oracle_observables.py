"""Pins of the reference's window observables: drain and source current,
the per-subcell net and emission-only phonon power maps, the electron
density map, and the steady-state test of the electron MC paragraph (the
current and the field no longer change).

Each conversion from counts to physical units is checked against something
the counts do not contain: energies the oracle tallies electron by electron
(work of the field in free flight, energy carried through the contacts,
energy taken from absorbed phonons, the ensemble's own energy), the drift
velocity of the bulk Monte Carlo, and charge neutrality."""
import math

import numpy as np
import pytest

from paper_1707_09073_amd import workloads as W

QE = 1.602176634e-19


def _small_device(Vds, n=20000, nx=50, Lx=500.0, gate=True, seed=None):
    c = W.device_config(n_particles=n, precision="fp64", Vds=Vds, n_cells=(nx, 3, 6), L_nm=(Lx, 60.0, 120.0),
                        seed=seed)
    if not gate:
        c["gate_x_nm"] = [-1.0, -1.0]
    return c


@pytest.fixture(scope="module")
def biased(oracle_mod):
    cfg = _small_device(2.0)
    o = oracle_mod.Oracle(cfg)
    o.run(100)
    o.reset_window()
    o.run(300)
    return cfg, o


def test_heat_map_equals_energy_balance_of_the_electrons(biased):
    """Every electron's energy is followed on its own: kinetic energy gained in
    free flight (the field's work), energy carried out through and brought in
    at the contacts, the change of the ensemble's total energy.  What is left
    went into phonons, and must equal the net phonon power map integrated over
    the subcells and the window (exact up to rounding)."""
    cfg, o = biased
    ob = o.observables()
    qn, qe, _ = o.power_maps()
    Vc = 1e-27 * 10.0 * 20.0 * 20.0
    t = ob["t_window_s"]
    to_phonons = ob["W_field_J"] - ob["dE_ens_J"] - ob["E_out_J"].sum() + ob["E_in_J"].sum()
    assert ob["W_field_J"] > 0.0 and to_phonons > 0.0
    assert qn.sum() * Vc * t == pytest.approx(to_phonons, rel=1e-10)
    assert ob["P_heat_W"] * t == pytest.approx(to_phonons, rel=1e-10)
    # emission only: the net exchange plus the energy taken from absorbed
    # phonons (tallied from the electrons' energy change in each absorption)
    assert qe.sum() * Vc * t == pytest.approx(to_phonons + ob["E_abs_J"], rel=1e-10)
    assert ob["P_emit_W"] * t == pytest.approx(to_phonons + ob["E_abs_J"], rel=1e-10)
    assert np.all(qe >= 0.0) and np.all(qe >= qn - 1e-6 * np.abs(qn).max())


def test_drain_current_equals_bulk_drift_current(oracle_mod):
    """An ungated 1 um channel at 1 V is a uniform 10 kV/cm bar of neutral
    doped GaN: its drain current must be e n v_d A with the drift velocity of
    the bulk Monte Carlo at the same field, doping and temperature."""
    cfgb = W.bulk_config(n_particles=20000, field_V_per_nm=1e-3, doping_cm3=1e18, substeps=10)
    b = oracle_mod.Oracle(cfgb)
    b.run(100)
    b.reset_window()
    b.run(400)
    vz = b.observables()["v_drift_ms"][2]
    assert vz < 0.0                                      # electrons drift against the field
    cfgd = W.device_config(n_particles=40000, precision="fp64", Vds=1.0)
    cfgd["gate_x_nm"] = [-1.0, -1.0]
    d = oracle_mod.Oracle(cfgd)
    d.run(200)
    d.reset_window()
    d.run(600)
    od = d.observables()
    A = 60e-9 * 120e-9
    want = QE * 1e24 * (-vz) * A
    assert od["I_D"] == pytest.approx(want, rel=0.03)
    # continuity: what enters at the source leaves at the drain
    se = math.hypot(*od["half_se"][0]) / 2
    assert abs(od["I_D"] + od["I_S"]) < 0.02 * od["I_D"] + 3 * se
    assert od["steady"] == 1


def test_density_map_is_the_doping_in_a_neutral_channel(oracle_mod):
    """Zero bias, no gate: the channel stays neutral, so the mean electron
    density over the window is N_D everywhere."""
    cfg = W.device_config(n_particles=40000, precision="fp64", Vds=0.0, n_cells=(20, 3, 6),
                          L_nm=(200.0, 60.0, 120.0))
    cfg["gate_x_nm"] = [-1.0, -1.0]
    o = oracle_mod.Oracle(cfg)
    o.run(20)
    o.reset_window()
    o.run(100)
    _, _, n = o.power_maps()
    ND = cfg["N_D_m3"]
    assert n.mean() == pytest.approx(ND, rel=0.01)
    # per channel slice: counting noise of 18 cells x 100 refreshes
    sl = n.reshape(20, 18).mean(1)
    per_slice = ND * 20 * 20 * 10e-27 * 18 / o.weight     # electrons per slice
    sigma = ND / math.sqrt(per_slice * 100 / 10)            # refreshes correlated over ~10 intervals
    assert np.all(np.abs(sl - ND) < 6 * sigma), (sl / ND, sigma / ND)
    ob = o.observables()
    assert abs(ob["I_D"]) < 3 * math.hypot(*ob["half_se"][0]) / 2 + 1e-12


def test_maps_from_counts_by_hand(oracle_mod):
    """A units check on one subcell from the integer counts: net heat
    w e (hw_LO (em - ab) + hw_iv (em - ab)) / (V_c t), emission alone, and
    the density w <count> / V_c."""
    cfg = _small_device(1.0, n=3600, nx=10, Lx=100.0)
    o = oracle_mod.Oracle(cfg)
    o.reset_window()
    o.run(7)
    heat, dens = o.maps()
    qn, qe, n = o.power_maps()
    w, Vc, t = o.weight, 10 * 20 * 20 * 1e-27, 7 * 10e-15
    q = int(np.argmax(heat[:, 0]))
    h = heat[q].astype(float)
    assert h[0] > 0
    assert qn[q] == pytest.approx(w * QE * (0.0912 * (h[0] - h[1]) + 0.0912 * (h[2] - h[3])) / (Vc * t), rel=1e-14)
    assert qe[q] == pytest.approx(w * QE * 0.0912 * (h[0] + h[2]) / (Vc * t), rel=1e-14)
    assert n[q] == pytest.approx(w * dens[q] / 7 / Vc, rel=1e-14)


def test_steady_state_test_on_synthetic_series(oracle_mod):
    rng = np.random.default_rng(5)
    noise = 3.0 + rng.normal(0.0, 1.0, 400)
    f, out = oracle_mod.steady_test(noise)
    assert f == 1
    # batch means of 20 values: the standard error of a half's mean is 1/sqrt(200)
    assert out[2] == pytest.approx(1 / math.sqrt(200), rel=0.35)
    assert out[0] == pytest.approx(noise[:200].mean(), rel=1e-12)
    assert out[1] == pytest.approx(noise[200:].mean(), rel=1e-12)
    ramp = noise + np.linspace(0.0, 2.0, 400)
    assert oracle_mod.steady_test(ramp)[0] == 0
    assert oracle_mod.steady_test(np.full(40, 2.5))[0] == 1          # constant: no change, no spread
    assert oracle_mod.steady_test(noise[:19])[0] == -1               # halves of fewer than 10 values
    # an odd length drops the first value
    f, out = oracle_mod.steady_test(noise[:41])
    assert out[0] == pytest.approx(noise[1:21].mean(), rel=1e-12)


def test_steady_state_of_the_bulk_transient(oracle_mod):
    """From a 300 K Maxwellian switched on at 100 kV/cm the drift velocity and
    mean energy rise over a few hundred fs: a window over the first 100 fs is
    not steady, a window after 3 ps is."""
    cfg = W.bulk_config(n_particles=10000, field_V_per_nm=1e-2)
    o = oracle_mod.Oracle(cfg)
    o.run(100)
    assert o.observables()["steady"] == 0
    o.run(3000)
    o.reset_window()
    o.run(1000)
    ob = o.observables()
    assert ob["steady"] == 1
    assert ob["valley_frac"].sum() == pytest.approx(1.0, rel=1e-12)
