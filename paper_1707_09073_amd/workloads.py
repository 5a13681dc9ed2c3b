"""Seeded synthetic inputs shaped like the paper's device and bulk runs.

This module holds input recipes only -- material parameters, geometry,
bias points, seeds and lattice-temperature maps -- and none of the Monte
Carlo arithmetic.  Both the GPU library binding and the CPU reference
consume the plain dictionaries it returns.

Sources: Table I of arXiv:1707.09073 (masses, valley offsets, nonparabolicity,
dielectric constants, density, deformation potentials); the electron MC
paragraph (three valleys Gamma1, U, Gamma3; half nanowire of 120 nm cut in
two; 3x6x100 subcells); the phonon paragraph (LO phonon at 91.2 meV;
branch-averaged sound velocity 3338 m/s).  Every value the paper leaves open
is a named field with the reading stated beside it.
"""
from __future__ import annotations

import copy
import math

import numpy as np

BASE_SEED = 1707_09073


def table1_material() -> dict:
    """Table I (valley triples in the text's order Gamma1, U, Gamma3)."""
    return dict(
        m_eff=[0.21, 0.25, 0.40],      # m0
        alpha=[0.19, 0.10, 0.0],       # 1/eV
        E_c=[0.0, 1.95, 2.1],          # eV
        Z=[1, 6, 1],                   # valley degeneracy: reading (paper silent)
        eps_s=8.9, eps_inf=5.35,       # eps0
        rho=6095.0,                    # kg/m^3  (6.095 g/cm^3)
        D_ac_eV=8.3,                   # eV
        D_iv_eVm=1.0e11,               # eV/m    (1e9 eV/cm), all valley pairs
        hw_lo_eV=0.0912,               # LO phonon energy (phonon paragraph)
        hw_iv_eV=0.0912,               # intervalley phonon: reading, same as LO
        u_ac=3338.0,                   # m/s, the only sound velocity the paper states
    )


def _base(mode: str) -> dict:
    return dict(
        mode=mode, precision="fp64", material=table1_material(),
        seed=BASE_SEED, instance=0,
        n_particles=10_000, capacity=10_000,
        dt_fs=1.0, substeps=1, n_bins=3000, dE_eV=1e-3,
        T0_K=300.0, T_init_K=300.0, N_D_m3=1e23,
        F_bulk=[0.0, 0.0, 0.0],
        L_nm=[1000.0, 60.0, 120.0], n_cells=[100, 3, 6],
        gate_x_nm=[250.0, 750.0], Vgs=0.0, Vds=0.0, phi_offset=0.0,
        T_cells=None,
    )


def bulk_config(n_particles: int = 10_000, field_V_per_nm: float = 1e-3, doping_cm3: float = 1e17,
                T: float = 300.0, substeps: int = 1, seed: int | None = None, precision: str = "fp64") -> dict:
    """Bulk wurtzite GaN, uniform field along c (z): 10 kV/cm = 1e-3 V/nm."""
    c = _base("bulk")
    c.update(n_particles=n_particles, capacity=n_particles, substeps=substeps,
             N_D_m3=doping_cm3 * 1e6, T0_K=T, T_init_K=T, precision=precision,
             F_bulk=[0.0, 0.0, field_V_per_nm],
             seed=BASE_SEED + 1 if seed is None else seed)
    return c


def device_config(n_particles: int = 200_000, Vgs: float = 0.0, Vds: float = 5.0, doping_cm3: float = 1e18,
                  precision: str = "fp32", substeps: int = 10, capacity_factor: float = 1.3,
                  seed: int | None = None, n_cells=(100, 3, 6), L_nm=(1000.0, 60.0, 120.0)) -> dict:
    """Half-nanowire FinFET: 60 nm x 120 nm cross-section (the 120 nm wire cut
    in half along the symmetry plane), 1 um channel, 3x6x100 subcells, gate
    over the middle half of the channel, Poisson refresh every 10 fs."""
    c = _base("device")
    nx = int(n_cells[0])
    c.update(n_particles=n_particles, capacity=int(math.ceil(n_particles * capacity_factor)),
             substeps=substeps, N_D_m3=doping_cm3 * 1e6, precision=precision,
             Vgs=Vgs, Vds=Vds, n_cells=list(n_cells), L_nm=list(L_nm),
             gate_x_nm=[0.25 * L_nm[0], 0.75 * L_nm[0]],
             seed=BASE_SEED + 2 if seed is None else seed)
    assert nx > 0
    return c


# Table II: GaN's and 6H-SiC's acoustic branches (q0 is the table's k0) and
# relaxation constants; and the free electrons of the doped wire for Eq. (1) (the
# electron density of 1e18 cm^-3 doping, Gamma1 mass, acoustic deformation
# potential and mass density of Table I, and the averaged group velocity).
GAN_PHONONS = dict(q0=10.94e9, w_max=3.50e13, A=5.26e-45, B1=1.10e-19, B2=200.0)
SIC_PHONONS = dict(q0=8.94e9, w_max=7.12e13, A=1.00e-45, B1=0.596e-19, B2=235.0)
WIRE_ELECTRONS = dict(n_m3=1e24, m_dos=0.21, D_a_eV=8.3, rho=6095.0, v_g=3338.0)

# Phonon faces of the half-nanowire box (x = 0, x = L, y = 0, y = L, z = 0,
# z = L): the source and drain contacts and the junction with the film below
# are isothermal sinks, the cut along the wire's symmetry plane is specular,
# the free sidewall and the top are diffuse.
WIRE_FACES = ["isothermal", "isothermal", "specular", "diffuse", "isothermal", "diffuse"]
# The same box when the chip around it is solved by Fourier's law: the wire's
# heat passes to the film only, so the contact ends are adiabatic (diffuse)
# and the foot, held at the film's temperature below it, is the one sink.
WIRE_FACES_ON_CHIP = ["diffuse", "diffuse", "specular", "diffuse", "isothermal", "diffuse"]


def wire_heat_map(cfg: dict, power_W: float = 1e-3, x0_nm: float | None = None, sigma_nm: float = 60.0,
                  seed: int = BASE_SEED + 7, noise: float = 0.3) -> np.ndarray:
    """Synthetic net heat map (W/m^3 per subcell, index (ix*ny + iy)*nz + iz)
    of the shape the electron windows produce: a Gaussian along x centred
    just past the drain-side gate edge, uniform across the cut, with
    multiplicative noise of relative size `noise` (so a few subcells turn
    into sinks), scaled to `power_W` in total."""
    nx, ny, nz = cfg["n_cells"]
    L = cfg["L_nm"]
    x0 = cfg["gate_x_nm"][1] + 50.0 if x0_nm is None else x0_nm
    xc = (np.arange(nx) + 0.5) * L[0] / nx
    prof = np.exp(-0.5 * ((xc - x0) / sigma_nm) ** 2)
    rng = np.random.default_rng(seed)
    q = prof[:, None] * (1.0 + noise * rng.standard_normal((nx, ny * nz)))
    vc = (L[0] / nx) * (L[1] / ny) * (L[2] / nz) * 1e-27
    return (q * power_W / (q.sum() * vc)).reshape(-1)


def _graded(first: float, total: float, ratio: float) -> np.ndarray:
    """Widths growing geometrically from `first` until they span `total`
    (the last one trimmed to fit)."""
    w, acc = [], 0.0
    while acc < total * (1 - 1e-12):
        d = min(first * ratio ** len(w), total - acc)
        if d < 0.3 * first * ratio ** max(len(w) - 1, 0) and w:
            w[-1] += d
            break
        w.append(d)
        acc += d
    return np.array(w)


def chip_geometry(device: dict | None = None, n_wires: int = 31, pitch_nm: float = 240.0, margin_x_um: float = 7.0,
                  margin_y_um: float = 4.0, film_um: float = 2.0, substrate_um: float = 30.0,
                  growth: float = 1.25) -> dict:
    """Half of the nanowire-array chip for the Fourier analysis (Fig. 1 of the
    paper is absent; its dimensions here are readings): n_wires GaN wires of
    twice the electron domain's cut width (y) and its height (z), one pitch
    apart, over the electron domain's channel (x); a GaN film of film_um on
    a SiC substrate of substrate_um whose bottom is the heat sink; graded
    margins of margin_x_um and margin_y_um around the array.  The cut runs
    through the middle wire's centre plane (a symmetry plane: adiabatic), so
    that wire's half is the electron domain itself.

    Wire cells have the electron subcells' widths, so every wire takes the
    electron heat map cell for cell (mirrored about its own centre plane).
    Returns n, edges (x, y, z in m), material per cell (0 void, 1 SiC,
    2 GaN film, 3 GaN wire), src_index per cell (the electron subcell, or
    -1), k_interface (first film cell), the wire and chip extents, and the
    cell index of the middle wire's subcells."""
    dev = device or device_config(n_particles=1000)
    (Lx, Ly, Lz), (nxw, nyw, nzw) = dev["L_nm"], dev["n_cells"]
    dxw, dyw, dzw = Lx / nxw, Ly / nyw, Lz / nzw
    half = int(n_wires) // 2                               # full wires beside the middle one
    # x: the channel at the subcell width, graded margins on both sides
    mx = _graded(dxw, margin_x_um * 1e3, growth)
    wx = np.concatenate([mx[::-1], np.full(nxw, dxw), mx])
    i0 = len(mx)
    # y: from the middle wire's centre plane through the last wire, then a margin
    span_y = half * pitch_nm + Ly
    ny_arr = int(round(span_y / dyw))
    assert abs(ny_arr * dyw - span_y) < 1e-6 * span_y and abs(pitch_nm / dyw - round(pitch_nm / dyw)) < 1e-9
    wy = np.concatenate([np.full(ny_arr, dyw), _graded(dyw, margin_y_um * 1e3, growth)])
    # z: substrate (graded toward the sink), film (graded toward the interface), the wire layer
    film = _graded(dzw, film_um * 1e3, growth)[::-1]
    sub = _graded(film[0] * growth, substrate_um * 1e3, growth)[::-1]
    wz = np.concatenate([sub, film, np.full(nzw, dzw)])
    k_if, k_w = len(sub), len(sub) + len(film)
    nx, ny, nz = len(wx), len(wy), len(wz)
    ex = np.concatenate([[0.0], np.cumsum(wx)]) - mx.sum()       # x = 0 at the source end of the channel
    ey = np.concatenate([[0.0], np.cumsum(wy)])
    ez = np.concatenate([[0.0], np.cumsum(wz)]) - (sub.sum() + film.sum())   # z = 0 at the wires' foot
    mat = np.zeros((nx, ny, nz), np.uint8)
    mat[:, :, :k_if] = 1
    mat[:, :, k_if:k_w] = 2
    src = np.full((nx, ny, nz), -1, np.int32)
    step = int(round(pitch_nm / dyw))
    for w in range(half + 1):
        for jj in range(-nyw, nyw):
            j = w * step + jj
            if j < 0:
                continue                                   # the middle wire's other half lies across the cut
            iy = jj if jj >= 0 else -jj - 1                # distance from the wire's centre plane, in subcells
            for kk in range(nzw):
                for ii in range(nxw):
                    mat[i0 + ii, j, k_w + kk] = 3
                    src[i0 + ii, j, k_w + kk] = (ii * nyw + iy) * nzw + kk
    middle = np.array([((i0 + ii) * ny + iy) * nz + k_w + kk
                       for ii in range(nxw) for iy in range(nyw) for kk in range(nzw)])
    # per electron subcell: the film cell below its column, under the middle wire
    base = np.array([((i0 + ii) * ny + iy) * nz + k_w - 1
                     for ii in range(nxw) for iy in range(nyw) for kk in range(nzw)], np.int32)
    return dict(n=[nx, ny, nz], edges=[ex * 1e-9, ey * 1e-9, ez * 1e-9], material=mat.ravel(), src_index=src.ravel(),
                base_index=base, k_interface=k_if, k_wire=k_w, i_wire=i0, middle_cells=middle, wires=half + 1,
                half_wires=2 * half + 1)


def hotspot_T_map(cfg: dict, dT: float = 150.0, x0_nm: float | None = None, sigma_nm: float = 100.0) -> np.ndarray:
    """Lattice temperature per subcell: T0 plus a Gaussian hot spot along x,
    uniform in y and z (peak at the drain end unless x0 is given)."""
    nx, ny, nz = cfg["n_cells"]
    Lx = cfg["L_nm"][0]
    x0 = Lx if x0_nm is None else x0_nm
    xc = (np.arange(nx) + 0.5) * Lx / nx
    Tx = cfg["T0_K"] + dT * np.exp(-((xc - x0) ** 2) / (2.0 * sigma_nm ** 2))
    return np.repeat(Tx, ny * nz).astype(np.float64)   # cell index (ix*ny + iy)*nz + iz


def large_device_config(n_particles: int = 10_000_000, seed: int | None = None) -> dict:
    """10 million superparticles on the half-nanowire device with a drain-end
    hot spot (300 K + 150 K Gaussian, sigma 100 nm), FP32 state."""
    c = device_config(n_particles=n_particles, precision="fp32", seed=BASE_SEED + 4 if seed is None else seed)
    c["T_cells"] = hotspot_T_map(c)
    return c


def bias_sweep(n_instances: int = 64, seed: int = BASE_SEED + 3, n_min: int = 20_000, n_max: int = 500_000,
               scale: float = 1.0) -> list[dict]:
    """Seeded bias points: Vgs ~ U[-3,0] V, Vds ~ U[1,10] V, doping log-uniform
    in [1e17, 1e19] cm^-3, ensemble sizes uniform in [n_min, n_max]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_instances):
        vgs = float(rng.uniform(-3.0, 0.0))
        vds = float(rng.uniform(1.0, 10.0))
        dop = float(10.0 ** rng.uniform(17.0, 19.0))
        n = int(rng.integers(n_min, n_max + 1))
        n = max(1800, int(n * scale))
        c = device_config(n_particles=n, Vgs=vgs, Vds=vds, doping_cm3=dop, seed=BASE_SEED + 3)
        c["instance"] = i
        out.append(c)
    return out


def surrogate_inputs(n: int, seed: int) -> list[dict]:
    """Training / validation bias points with random hot-spot T maps:
    amplitude ~ U[0,150] K, centre ~ U[500,1000] nm, sigma ~ U[50,200] nm."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        c = device_config(n_particles=200_000,
                          Vgs=float(rng.uniform(-3.0, 0.0)), Vds=float(rng.uniform(1.0, 10.0)),
                          doping_cm3=float(10.0 ** rng.uniform(17.0, 19.0)), seed=int(seed) * 7919 + i)
        c["T_cells"] = hotspot_T_map(c, dT=float(rng.uniform(0.0, 150.0)), x0_nm=float(rng.uniform(500.0, 1000.0)),
                                     sigma_nm=float(rng.uniform(50.0, 200.0)))
        out.append(c)
    return out


def scaled(cfg: dict, **kw) -> dict:
    c = copy.deepcopy(cfg)
    c.update(kw)
    return c
