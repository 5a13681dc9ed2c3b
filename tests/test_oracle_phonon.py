"""Pins of the phonon-side reference: the sine dispersion and its density of
states against the paper's own definitions (q0 = (6 pi^2 N)^(1/3), so the
states of a branch number N per volume), the classical heat capacity, the
bulk conductivities Table II was fitted to, the limits of Eq. (1) and the
Fermi level, and the closed forms and symmetries of Eqs. (2) and (3)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import phonon_oracle as P

GAN, SIC = P.table2("GaN"), P.table2("6H-SiC")


@pytest.mark.parametrize("m", [GAN, SIC])
def test_dispersion_and_group_velocity(m):
    w = np.linspace(0.01, 0.99, 50) * m["w_max"]
    assert np.allclose(P.omega_of_q(m, P.q_of_w(m, w)), w, rtol=1e-13)
    q = P.q_of_w(m, w)
    h = 1e-6 * m["q0"]
    fd = (P.omega_of_q(m, q + h) - P.omega_of_q(m, q - h)) / (2 * h)
    assert np.allclose(P.vg_of_w(m, w), fd, rtol=1e-7)
    # q0 = pi / a_D (the table's k0)
    assert m["q0"] == pytest.approx(math.pi / m["a_D"], rel=3e-3)


@pytest.mark.parametrize("m", [GAN, SIC])
def test_states_per_branch_equal_primitive_cells(m):
    N = m["q0"] ** 3 / (6 * math.pi ** 2)
    n = integrate.quad(lambda w: float(P.dos(m, w)), 0, m["w_max"], limit=400)[0]
    assert n == pytest.approx(N, rel=1e-9)


@pytest.mark.parametrize("m", [GAN, SIC])
def test_classical_heat_capacity(m):
    """T >> hbar omega_max / k_B: each mode holds k_B, so three branches give
    3 k_B N (the first correction is -<x^2>/12, x = hbar omega / k_B T)."""
    N = m["q0"] ** 3 / (6 * math.pi ** 2)
    T = 1e5
    c = 3 * integrate.quad(lambda w: float(P.heat_capacity(m, w, T)), 0, m["w_max"], limit=400)[0]
    assert c == pytest.approx(3 * P.KB * N, rel=1e-5)


def test_bulk_conductivities_table2_was_fitted_to():
    """The relaxation-time parameters reproduce measured bulk conductivities
    (phonon paragraph): about 230 W/m/K for GaN and several hundred for
    6H-SiC at room temperature, falling with temperature (Umklapp)."""
    kg, ks = P.kappa(GAN, 300.0), P.kappa(SIC, 300.0)
    assert 200.0 < kg < 260.0, kg
    assert 300.0 < ks < 500.0, ks
    assert P.kappa(GAN, 415.0) < 0.7 * kg


def test_fermi_level_limits():
    m = 0.21
    T = 300.0
    Nc = 2.0 * (m * P.M0 * P.KB * T / (2 * math.pi * P.HBAR ** 2)) ** 1.5
    n = 1e-4 * Nc                                   # nondegenerate: Boltzmann
    assert P.fermi_level(n, m, T) == pytest.approx(P.KB * T * math.log(n / Nc) / P.QE, abs=1e-4 * P.KB * T / P.QE)
    n = 1e27                                        # degenerate at 4 K: the T = 0 Fermi energy
    EF0 = P.HBAR ** 2 * (3 * math.pi ** 2 * n) ** (2 / 3) / (2 * m * P.M0) / P.QE
    assert P.fermi_level(n, m, 4.0) == pytest.approx(EF0, rel=1e-4)


def test_electron_scattering_limits_and_size():
    """Eq. (1): with the Fermi level far below the band the braces reduce to
    2 exp(-x) sinh(hbar omega / 2 k_B T) (few electrons), far above it to
    hbar omega / k_B T; and at 7e18 cm^-3 the extra scattering lowers the
    room-temperature conductivity of GaN by about the 13% the paper cites."""
    T, m, Da, rho, vs = 300.0, 0.21, 8.3, 6095.0, 3338.0
    w = np.array([3e11, 1e12, 5e12])
    kT = P.KB * T
    half = 0.5 * m * P.M0 * vs * vs
    pref = (Da * P.QE) ** 2 * (m * P.M0) ** 3 * vs / (4 * math.pi * P.HBAR ** 4 * rho) * kT / half
    EF = -0.5                                       # eV: nondegenerate
    x = (half - EF * P.QE) / kT + P.HBAR ** 2 * w * w / (8 * m * P.M0 * vs * vs * kT)
    want = pref * 2 * np.exp(-x) * np.sinh(P.HBAR * w / (2 * kT))
    assert np.allclose(P.inv_tau_electron(w, T, EF, m, Da, rho, vs), want, rtol=1e-9)
    EF = 2.0                                        # eV: deep in the band
    assert np.allclose(P.inv_tau_electron(w, T, EF, m, Da, rho, vs), pref * P.HBAR * w / kT, rtol=1e-9)
    assert np.all(P.inv_tau_electron(np.linspace(1e11, GAN["w_max"], 200), T, 0.03, m, Da, rho, vs) >= 0.0)
    EF7 = P.fermi_level(7e24, m, T)
    k0 = P.kappa(GAN, T)
    ke = P.kappa(GAN, T, lambda ww: P.inv_tau_electron(ww, T, EF7, m, Da, rho, vs))
    assert 0.80 < ke / k0 < 0.90, ke / k0


def test_dmm_transmissivity_closed_form_and_symmetry():
    w = np.linspace(0.001, 0.999, 101) * GAN["w_max"]       # GaN's band lies inside SiC's
    t12, t21 = P.transmissivity(GAN, SIC, w), P.transmissivity(SIC, GAN, w)
    assert np.allclose(t12 + t21, 1.0, rtol=0, atol=1e-14)
    q1, q2 = P.q_of_w(GAN, w), P.q_of_w(SIC, w)
    assert np.allclose(t12, q2 ** 2 / (q1 ** 2 + q2 ** 2), rtol=1e-12)
    assert np.allclose(P.transmissivity(GAN, GAN, w), 0.5, rtol=1e-14)
    above = np.linspace(1.01, 1.9, 10) * GAN["w_max"]       # SiC modes with no GaN partner
    assert np.all(P.transmissivity(SIC, GAN, above) == 0.0)


def test_interface_conductance_detailed_balance_and_classical_limit():
    """Eq. (3) gives the same conductance from either side (the transmitted
    fluxes balance at equal temperature); between two identical media in the
    classical limit it is (3/8) k_B (2 q0 / pi)^2 omega_max (pi^2/4 - 2) / (2 pi^2)."""
    for T in (300.0, 415.0):
        a, b = P.interface_conductance(GAN, SIC, T), P.interface_conductance(SIC, GAN, T)
        assert a == pytest.approx(b, rel=1e-9)
    T = 1e5
    want = 3 / 8 * P.KB * (2 * GAN["q0"] / math.pi) ** 2 * GAN["w_max"] * (math.pi ** 2 / 4 - 2) / (2 * math.pi ** 2)
    assert P.interface_conductance(GAN, GAN, T) == pytest.approx(want, rel=1e-5)
    # GaN/SiC at room temperature: a thermal boundary resistance of order 1e-8 m^2 K / W
    assert 5e-9 < 1.0 / P.interface_conductance(GAN, SIC, 300.0) < 1e-7


def test_mean_free_path_accumulation_matches_the_paper():
    """The thermal-resistance passage states that in bulk GaN at 415 K about
    60% of the lattice conductivity comes from phonons with mean free paths
    between 100 nm and 2 um.  Table II's dispersion, heat capacity and
    relaxation times give that share (0.587)."""
    m, T = GAN, 415.0
    w = np.linspace(1e-6, 1.0 - 1e-9, 200001) * m["w_max"]
    v = P.vg_of_w(m, w)
    tau = 1.0 / P.inv_tau_bulk(m, w, T)
    mfp = v * tau
    c = P.heat_capacity(m, w, T) * v * v * tau
    share = c[(mfp >= 100e-9) & (mfp < 2e-6)].sum() / c.sum()
    assert 0.55 < share < 0.65, share
