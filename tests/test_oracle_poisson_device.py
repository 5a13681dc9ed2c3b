"""Pins of the reference's electrostatics (finite-volume Poisson on the
subcell grid) and device-level sanity of the ensemble with contacts."""
import math

import numpy as np
import pytest

from paper_1707_09073_amd import workloads as W

QE, EPS0 = 1.602176634e-19, 8.8541878128e-12


def _dev(nx=100, Vds=5.0, Vgs=0.0, gate=True, n=1800, L=(1000.0, 60.0, 120.0)):
    c = W.device_config(n_particles=n, precision="fp64", Vds=Vds, Vgs=Vgs, n_cells=(nx, 3, 6), L_nm=L)
    if not gate:
        c["gate_x_nm"] = [-1.0, -1.0]
    return c


def test_linear_potential_without_charge_or_gate(oracle_mod):
    cfg = _dev(gate=False, Vds=5.0)
    o = oracle_mod.Oracle(cfg)
    phi, F = o.poisson_solve(np.zeros(o.ncell))
    nx = cfg["n_cells"][0]
    xc = (np.arange(nx) + 0.5) * cfg["L_nm"][0] / nx
    want = np.repeat(5.0 * xc / cfg["L_nm"][0], 18)
    assert np.allclose(phi, want, rtol=0, atol=1e-12)
    assert np.allclose(F[:, 0], -5.0 / cfg["L_nm"][0], rtol=1e-11)
    assert np.allclose(F[:, 1:], 0.0, atol=1e-14)


def test_zero_terminals_zero_charge_gives_zero(oracle_mod):
    cfg = _dev(Vds=0.0, Vgs=0.0)
    o = oracle_mod.Oracle(cfg)
    phi, F = o.poisson_solve(np.zeros(o.ncell))
    assert np.abs(phi).max() < 1e-14 and np.abs(F).max() < 1e-14


def test_gate_symmetry_and_maximum_principle(oracle_mod):
    cfg = _dev(Vds=0.0, Vgs=-1.5)
    o = oracle_mod.Oracle(cfg)
    phi, F = o.poisson_solve(np.zeros(o.ncell))
    P = phi.reshape(100, 3, 6)
    assert np.allclose(P, P[::-1], atol=1e-12)            # S and D both grounded, gate centred
    assert phi.min() >= -1.5 - 1e-12 and phi.max() <= 1e-12
    # the gated top/outer cells are pulled towards the gate
    assert P[50, 2, 5] < P[50, 0, 0] < 0.0
    Fx = F[:, 0].reshape(100, 3, 6)
    assert np.allclose(Fx, -Fx[::-1], atol=1e-12)


def _manufactured_error(oracle_mod, nx):
    L = 1000.0
    cfg = _dev(nx=nx, gate=False, Vds=2.0, n=nx * 18, L=(L, 60.0, 120.0))
    o = oracle_mod.Oracle(cfg)
    A = 0.7
    eps = cfg["material"]["eps_s"] * EPS0 * 1e-9         # F/nm
    dx = L / nx
    x0 = np.arange(nx) * dx
    # charge per cell = integral of eps A (pi/L)^2 sin(pi x/L) over the cell (exact)
    q = eps * A * (math.pi / L) * (np.cos(math.pi * x0 / L) - np.cos(math.pi * (x0 + dx) / L)) * 20.0 * 20.0
    phi, _ = o.poisson_solve(np.repeat(q, 18))
    xc = x0 + dx / 2
    exact = 2.0 * xc / L + A * np.sin(math.pi * xc / L)
    return np.abs(phi.reshape(nx, 18)[:, 0] - exact).max()


def test_manufactured_solution_second_order(oracle_mod):
    e = [_manufactured_error(oracle_mod, nx) for nx in (25, 50, 100, 200)]
    rates = [e[i] / e[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in rates), (e, rates)
    assert e[2] < 1e-4


def test_initial_state_is_neutral_and_injection_fills_contacts(oracle_mod):
    cfg = _dev(n=18000, nx=20, L=(200.0, 60.0, 120.0), Vds=1.0)
    o = oracle_mod.Oracle(cfg)
    w = o.weight
    assert w == pytest.approx(1e-3 * 200 * 60 * 120 / 18000, rel=1e-14)
    target = round(1e-3 * 10 * 20 * 20 / w)
    _, _, n = o.fields()
    n = n.reshape(20, 18)
    assert np.all(n[0] >= target) and np.all(n[-1] >= target)
    o.run(30)
    _, _, n = o.fields()
    n = n.reshape(20, 18)
    assert np.all(n[0] >= target) and np.all(n[-1] >= target)
    c = o.counts()
    assert c["exits"].sum() > 0 and c["injections"].sum() > 0
    P = o.particles()
    ids = P["id"][P["alive"] == 1]
    assert len(np.unique(ids)) == len(ids)                 # identities stay unique
    assert o.next_id == 18000 + c["injections"].sum()


def test_zero_bias_no_current_no_net_heat(oracle_mod):
    """V_ds = V_gs = 0 (everything grounded): the drain current and the net
    phonon emission per cell vanish within 3 sigma (detailed balance)."""
    cfg = _dev(n=20000, nx=20, L=(200.0, 60.0, 120.0), Vds=0.0, Vgs=0.0)
    o = oracle_mod.Oracle(cfg)
    o.run(20)
    o.reset_window()
    o.run(100)                         # 1 ps
    c = o.counts()
    net_d = c["exits"][1] - c["injections"][1]
    assert abs(net_d) < 3 * math.sqrt(c["exits"][1] + c["injections"][1] + 1)
    heat, _ = o.maps()
    em, ab = heat[:, 0].astype(float).sum(), heat[:, 1].astype(float).sum()
    assert em > 1000 and abs(em - ab) < 3 * math.sqrt(em + ab)


def test_biased_device_drives_current_and_heats_near_drain(oracle_mod):
    cfg = _dev(n=30000, nx=50, L=(500.0, 60.0, 120.0), Vds=2.0, Vgs=0.0)
    o = oracle_mod.Oracle(cfg)
    o.run(50)
    o.reset_window()
    o.run(100)
    c = o.counts()
    net_d = c["exits"][1] - c["injections"][1]
    assert net_d > 5 * math.sqrt(c["exits"][1] + c["injections"][1])   # electrons flow to the drain
    heat, _ = o.maps()
    net = (heat[:, 0].astype(float) - heat[:, 1]).reshape(50, 18).sum(1)
    assert net.sum() > 0
    assert net[25:].sum() > net[:25].sum()                               # dissipation grows towards the drain


def _gated_manufactured(oracle_mod, nx, ny, nz):
    """Gate over the whole channel, every terminal at 0 V: the Dirichlet faces
    are the source, the drain, the top and the outer side; y = 0 and z = 0
    are Neumann.  phi = A sin(pi x / L) cos(pi y / 2 Ly) cos(pi z / 2 Lz)
    meets all of them, and -eps lap(phi) = eps lam phi."""
    L, Ly, Lz = 200.0, 60.0, 120.0
    cfg = W.device_config(n_particles=nx * ny * nz, precision="fp64", Vds=0.0, Vgs=0.0, n_cells=(nx, ny, nz),
                          L_nm=(L, Ly, Lz))
    cfg["gate_x_nm"] = [0.0, L]
    o = oracle_mod.Oracle(cfg)
    A = 0.4
    eps = cfg["material"]["eps_s"] * EPS0 * 1e-9
    lam = math.pi ** 2 * (1 / L ** 2 + 1 / (4 * Ly ** 2) + 1 / (4 * Lz ** 2))
    dx, dy, dz = L / nx, Ly / ny, Lz / nz
    # exact cell integrals of the separable source
    ix = np.arange(nx) * dx
    Ix = (L / math.pi) * (np.cos(math.pi * ix / L) - np.cos(math.pi * (ix + dx) / L))
    iy = np.arange(ny) * dy
    Iy = (2 * Ly / math.pi) * (np.sin(math.pi * (iy + dy) / (2 * Ly)) - np.sin(math.pi * iy / (2 * Ly)))
    iz = np.arange(nz) * dz
    Iz = (2 * Lz / math.pi) * (np.sin(math.pi * (iz + dz) / (2 * Lz)) - np.sin(math.pi * iz / (2 * Lz)))
    q = eps * lam * A * (Ix[:, None, None] * Iy[None, :, None] * Iz[None, None, :]).ravel()
    phi, F = o.poisson_solve(q)
    xc, yc, zc = ix + dx / 2, iy + dy / 2, iz + dz / 2
    X, Y, Z = np.meshgrid(xc, yc, zc, indexing="ij")
    exact = A * np.sin(math.pi * X / L) * np.cos(math.pi * Y / (2 * Ly)) * np.cos(math.pi * Z / (2 * Lz))
    dphidy = -A * (math.pi / (2 * Ly)) * np.sin(math.pi * X / L) * np.sin(math.pi * Y / (2 * Ly)) * \
        np.cos(math.pi * Z / (2 * Lz))
    dphidz = -A * (math.pi / (2 * Lz)) * np.sin(math.pi * X / L) * np.cos(math.pi * Y / (2 * Ly)) * \
        np.sin(math.pi * Z / (2 * Lz))
    Fr = F.reshape(nx, ny, nz, 3)
    err_phi = np.abs(phi.reshape(nx, ny, nz) - exact).max() / A
    # field in the cells along the gated faces (outer side, top), where a
    # Dirichlet neighbour sits half a cell away
    err_fy = np.abs(Fr[:, -1, :, 1] + dphidy[:, -1, :]).max() / np.abs(dphidy).max()
    err_fz = np.abs(Fr[:, :, -1, 2] + dphidz[:, :, -1]).max() / np.abs(dphidz).max()
    return err_phi, err_fy, err_fz


def test_gated_faces_manufactured_solution(oracle_mod):
    """Second-order potential and a converging field at the gated faces: a
    wrong gate-face coefficient in the matrix or the right-hand side, or a
    wrong half-cell distance in the field, stops the convergence."""
    e = [_gated_manufactured(oracle_mod, 10 * s, 3 * s, 6 * s) for s in (1, 2, 4)]
    phi = [x[0] for x in e]
    assert all(3.5 < phi[i] / phi[i + 1] < 4.5 for i in range(2)), phi
    assert phi[-1] < 2e-3
    for j in (1, 2):
        f = [x[j] for x in e]
        assert all(f[i] / f[i + 1] > 1.8 for i in range(2)), f
        assert f[-1] < 0.05, f


def test_gated_superposition_and_bounds(oracle_mod):
    """No charge, gate over the whole channel: the potential of (V_ds, V_gs)
    is the sum of those of (V_ds, 0) and (0, V_gs), and lies between the
    lowest and highest terminal potential."""
    cfg = W.device_config(n_particles=1800, precision="fp64", Vds=0.7, Vgs=-0.4, n_cells=(20, 3, 6),
                          L_nm=(200.0, 60.0, 120.0))
    cfg["gate_x_nm"] = [0.0, 200.0]
    a = oracle_mod.Oracle(dict(cfg, Vgs=0.0)).poisson_solve(np.zeros(360))[0]
    b = oracle_mod.Oracle(dict(cfg, Vds=0.0)).poisson_solve(np.zeros(360))[0]
    ab = oracle_mod.Oracle(cfg).poisson_solve(np.zeros(360))[0]
    assert np.allclose(ab, a + b, rtol=0, atol=1e-13)
    assert np.all(ab <= 0.7 + 1e-13) and np.all(ab >= -0.4 - 1e-13)
