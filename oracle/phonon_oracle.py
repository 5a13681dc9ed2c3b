"""FP64 reference of the phonon side of the hybrid method: the sine-shaped
acoustic dispersion and the relaxation times of the phonon paragraph
(Table II), the phonon-free-electron scattering rate of Eq. (1), the
diffuse-mismatch transmissivity of Eq. (2) and the interface resistance of
Eq. (3).

TEST INFRASTRUCTURE ONLY: used by the tests; the GPU product path never
imports it.  Integrals use adaptive quadrature (scipy.integrate.quad), not
the bin sums of the library.

Model (phonon paragraph): three identical acoustic branches with
omega(q) = omega_max sin(pi q / 2 q0) for 0 <= q <= q0.  Per branch and unit
volume the density of states is D(omega) = q^2 / (2 pi^2 v_g) and the mode
heat capacity C(omega) = hbar omega d f_BE/dT D(omega).  Relaxation:
1/tau = A omega^4 + B1 omega^2 T exp(-B2 / T), plus Eq. (1) for scattering by
free electrons where the wire is doped.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

HBAR = 1.054571817e-34
KB = 1.380649e-23
QE = 1.602176634e-19
M0 = 9.1093837015e-31


def table2(material: str) -> dict:
    """Table II: q0 (the table's k0, 1/m), omega_max (rad/s), a_D (m), A (s^3),
    B1 (s/K), B2 (K); for GaN also the mass density of Table I (kg/m^3),
    which Eq. (1) uses."""
    if material == "GaN":
        return dict(q0=10.94e9, w_max=3.50e13, a_D=2.87e-10, A=5.26e-45, B1=1.10e-19, B2=200.0, rho=6095.0)
    if material == "6H-SiC":
        return dict(q0=8.94e9, w_max=7.12e13, a_D=3.51e-10, A=1.00e-45, B1=0.596e-19, B2=235.0, rho=None)
    raise ValueError(material)


def q_of_w(m: dict, w):
    return (2.0 * m["q0"] / math.pi) * np.arcsin(np.clip(np.asarray(w, float) / m["w_max"], 0.0, 1.0))


def omega_of_q(m: dict, q):
    return m["w_max"] * np.sin(math.pi * np.asarray(q, float) / (2.0 * m["q0"]))


def vg_of_w(m: dict, w):
    """Group velocity d omega / d q at frequency omega (m/s)."""
    w = np.asarray(w, float)
    return (math.pi / (2.0 * m["q0"])) * np.sqrt(np.maximum(m["w_max"] ** 2 - w * w, 0.0))


def dos(m: dict, w):
    """Density of states per branch per unit volume and angular frequency."""
    q = q_of_w(m, w)
    with np.errstate(divide="ignore", invalid="ignore"):
        return q * q / (2.0 * math.pi ** 2 * vg_of_w(m, w))


def dfdT(w, T):
    """d f_BE / dT of the Bose-Einstein occupation."""
    x = HBAR * np.asarray(w, float) / (KB * T)
    ex = np.exp(-x)
    return x / T * ex / (1.0 - ex) ** 2


def heat_capacity(m: dict, w, T):
    """C(omega) per branch: hbar omega df/dT D(omega), J/(m^3 K) per rad/s."""
    return HBAR * np.asarray(w, float) * dfdT(w, T) * dos(m, w)


def inv_tau_bulk(m: dict, w, T):
    w = np.asarray(w, float)
    return m["A"] * w ** 4 + m["B1"] * w * w * T * math.exp(-m["B2"] / T)


def fermi_level(n_m3: float, m_dos: float, T: float) -> float:
    """E_F (eV, from the band edge) of a parabolic band of mass m_dos (m0)
    holding n_m3 electrons per m^3 at T: n = N_c F_1/2(eta), with
    F_1/2(eta) = (2/sqrt(pi)) int_0^inf sqrt(e) / (1 + exp(e - eta)) de."""
    Nc = 2.0 * (m_dos * M0 * KB * T / (2.0 * math.pi * HBAR ** 2)) ** 1.5

    def F(eta):
        f = lambda e: math.sqrt(e) / (1.0 + math.exp(min(e - eta, 700.0)))
        top = max(eta, 0.0) + 60.0
        return 2.0 / math.sqrt(math.pi) * integrate.quad(f, 0.0, top, points=[max(eta, 0.0)] if eta > 0 else None,
                                                           limit=200, epsabs=0.0, epsrel=1e-13)[0]

    # bracket: below the Boltzmann estimate, above twice the T = 0 Fermi energy
    ef0 = HBAR ** 2 * (3.0 * math.pi ** 2 * n_m3) ** (2.0 / 3.0) / (2.0 * m_dos * M0) / (KB * T)
    lo = min(-60.0, math.log(n_m3 / Nc) - 10.0)
    hi = max(200.0, 2.0 * ef0 + 10.0)
    eta = optimize.brentq(lambda e: Nc * F(e) - n_m3, lo, hi, xtol=1e-14, rtol=1e-14)
    return eta * KB * T / QE


def inv_tau_electron(w, T: float, E_F_eV: float, m_dos: float, D_a_eV: float, rho: float, v_g: float):
    """Eq. (1): phonon scattering by free electrons (1/s)."""
    w = np.asarray(w, float)
    m = m_dos * M0
    Da = D_a_eV * QE
    kT = KB * T
    half_mv2 = 0.5 * m * v_g * v_g
    pref = Da * Da * m ** 3 * v_g / (4.0 * math.pi * HBAR ** 4 * rho) * kT / half_mv2
    x = (half_mv2 - E_F_eV * QE) / kT + HBAR ** 2 * w * w / (8.0 * m * v_g * v_g * kT)
    c = HBAR * w / (2.0 * kT)
    # the braces, 2c - ln((1 + e^(x + c)) / (1 + e^(x - c))), rewritten with
    # ln(1 + e^y) = y + ln(1 + e^-y) as ln(1 + e^(c - x)) - ln(1 + e^(-c - x)):
    # no cancellation where x >> c
    braces = np.logaddexp(0.0, c - x) - np.logaddexp(0.0, -c - x)
    return pref * braces


def kappa(m: dict, T: float, extra_inv_tau=None) -> float:
    """Bulk lattice conductivity (1/3) sum_p int C v^2 tau d omega over the
    three identical branches (W/m/K)."""
    def f(w):
        it = inv_tau_bulk(m, w, T) + (0.0 if extra_inv_tau is None else float(extra_inv_tau(w)))
        return float(heat_capacity(m, w, T) * vg_of_w(m, w) ** 2 / it)
    return integrate.quad(f, 0.0, m["w_max"], limit=400, epsrel=1e-12)[0]


def transmissivity(m1: dict, m2: dict, w):
    """Eq. (2) with three identical branches on each side: the sums over
    branches cancel, and v D = q^2 / (2 pi^2)."""
    w = np.asarray(w, float)
    with np.errstate(invalid="ignore"):   # v D at or above a band top is masked out
        a = np.where(w < m1["w_max"], vg_of_w(m1, w) * dos(m1, w), 0.0)
        b = np.where(w < m2["w_max"], vg_of_w(m2, w) * dos(m2, w), 0.0)
    return np.where(a + b > 0.0, b / np.where(a + b > 0.0, a + b, 1.0), 0.0)


def interface_conductance(m1: dict, m2: dict, T: float) -> float:
    """Eq. (3): 1/R_K = sum_p int_0^{w_max,1} v_1 c_1 tau_12 d omega / 4
    (W/m^2/K), three identical branches of material 1."""
    def f(w):
        return float(vg_of_w(m1, w) * heat_capacity(m1, w, T) * transmissivity(m1, m2, w))
    wm = min(m1["w_max"], m2["w_max"])
    pts = [wm] if wm < m1["w_max"] else None
    return 3.0 * integrate.quad(f, 0.0, m1["w_max"], points=pts, limit=400, epsrel=1e-12)[0] / 4.0


def bin_tables(m: dict, T: float, n_bins: int, electrons: dict | None = None):
    """Frequency bins of equal width over (0, omega_max), values at the bin
    midpoints: omega (rad/s), group velocity (m/s), heat capacity of the bin
    for the three branches (J/(m^3 K): 3 C(omega) d omega) and relaxation
    rate (1/s: Table II's impurity and Umklapp terms, plus Eq. (1) when
    `electrons` gives n_m3, m_dos, D_a_eV, rho, v_g)."""
    dw = m["w_max"] / n_bins
    w = (np.arange(n_bins) + 0.5) * dw
    it = inv_tau_bulk(m, w, T)
    if electrons:
        EF = fermi_level(electrons["n_m3"], electrons["m_dos"], T)
        it = it + inv_tau_electron(w, T, EF, electrons["m_dos"], electrons["D_a_eV"], electrons["rho"],
                                   electrons["v_g"])
    return w, vg_of_w(m, w), 3.0 * heat_capacity(m, w, T) * dw, it
