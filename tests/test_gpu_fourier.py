"""GPU parity of the Fourier's-law spreading (coupling paragraph) against the
direct sparse solve of the same finite-volume system, the size-limited
conductivities against their bin sums and quadrature, and the chip-scale
problem of the nanowire array."""
import sys

import numpy as np
import pytest

from oracle import fourier_oracle as F
from oracle import phonon_oracle as P
from paper_1707_09073_amd import workloads as W

pytestmark = pytest.mark.gpu

GAN, SIC = P.table2("GaN"), P.table2("6H-SiC")


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


def _edges(widths):
    return np.concatenate([[0.0], np.cumsum(widths)])


def _problem(seed, n, held, k_if, R_K):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    edges = [_edges(rng.uniform(10e-9, 300e-9, m)) for m in n]
    kap = rng.uniform(20.0, 400.0, n)
    kap[1:3, 2:5, nz // 2:] = 0.0
    q = rng.uniform(0.0, 1e-6, n)
    cfg = dict(n=list(n), dirichlet=held, k_interface=k_if, R_K_m2KW=R_K, T_sink_K=300.0, rtol=1e-13,
               max_iterations=20000)
    return cfg, edges, kap.ravel(), q.ravel()


@pytest.mark.parametrize("n,held,k_if", [((9, 8, 7), [1, 0, 0, 0, 1, 0], 3), ((33, 17, 5), [0, 0, 0, 1, 0, 0], 2),
                                         ((5, 41, 23), [1, 1, 1, 1, 1, 1], -1), ((1, 1, 64), [0, 0, 0, 0, 1, 0], 40)])
def test_solver_matches_direct_solve(G, n, held, k_if):
    cfg, edges, kap, q = _problem(sum(n), n, held, k_if, 2.5e-9)
    _say("fourier solve", n, "held", held)
    r = G.fo_solve(cfg, edges, kap, q)
    T = r["T"].cpu().numpy()
    ref = F.solve(cfg, edges, kap, q)
    rise = ref - 300.0
    assert np.abs((T - 300.0) - rise).max() <= 1e-9 * np.abs(rise).max()
    assert r["rel_residual"] <= 1e-13 and r["iterations"] > 0
    # the same bits on a second solve (dot products in a fixed order)
    assert np.array_equal(G.fo_solve(cfg, edges, kap, q)["T"].cpu().numpy(), T)


@pytest.mark.parametrize("n,held,k_if", [((33, 17, 5), [0, 0, 0, 1, 0, 0], 2), ((5, 41, 23), [1, 1, 1, 1, 1, 1], -1)])
def test_warm_start_reaches_the_direct_solution_in_fewer_iterations(G, n, held, k_if):
    """A solve started from a nearby temperature (the solution of the same
    problem with the heat 1e-5 lower, as between iterations of a converging
    coupled loop) meets the same stopping rule and the same direct solution
    as a cold solve, in fewer iterations (checks every 25); started from the
    direct answer it needs fewer still."""
    cfg, edges, kap, q = _problem(sum(n) + 1, n, held, k_if, 2.5e-9)
    _say("fourier warm start", n, "held", held)
    cold = G.fo_solve(cfg, edges, kap, q)
    near = G.fo_solve(cfg, edges, kap, (1.0 - 1e-5) * q)["T"]
    warm = G.fo_solve(cfg, edges, kap, q, T0=near)
    ref = F.solve(cfg, edges, kap, q)
    rise = ref - 300.0
    for r in (cold, warm):
        T = r["T"].cpu().numpy()
        assert np.abs((T - 300.0) - rise).max() <= 1e-9 * np.abs(rise).max()
        assert r["rel_residual"] <= 1e-13
    assert 0 < warm["iterations"] < cold["iterations"], (warm["iterations"], cold["iterations"])
    exact = G.fo_solve(cfg, edges, kap, q, T0=ref)
    assert exact["iterations"] <= warm["iterations"] and exact["rel_residual"] <= 1e-13
    assert np.abs((exact["T"].cpu().numpy() - 300.0) - rise).max() <= 1e-9 * np.abs(rise).max()


def test_layered_flux_is_exact(G):
    """Heat in the top cell only: the rise at the centres below is the flux
    times the series resistance from the sink, with the R_K jump."""
    rng = np.random.default_rng(5)
    wz = rng.uniform(20e-9, 200e-9, 30)
    kz = np.where(np.arange(30) < 12, 400.0, 130.0)
    kap = np.broadcast_to(kz, (2, 3, 30)).copy()
    q = np.zeros((2, 3, 30))
    q[:, :, -1] = 1e-6
    R_K = 4e-9
    cfg = dict(n=[2, 3, 30], dirichlet=[0, 0, 0, 0, 1, 0], k_interface=12, R_K_m2KW=R_K, T_sink_K=300.0, rtol=1e-14)
    T = G.fo_solve(cfg, [_edges(np.full(2, 50e-9)), _edges(np.full(3, 50e-9)), _edges(wz)], kap.ravel(),
                   q.ravel())["T"].cpu().numpy().reshape(2, 3, 30)
    flux = 1e-6 / (50e-9) ** 2
    r = wz[0] / (2 * kz[0])
    want = [flux * r]
    for i in range(1, 30):
        r += wz[i - 1] / (2 * kz[i - 1]) + wz[i] / (2 * kz[i]) + (R_K if i == 12 else 0.0)
        want.append(flux * r)
    assert np.allclose(T[0, 0, :-1] - 300.0, want[:-1], rtol=1e-10)


def test_rejected_configurations(G):
    cfg, edges, kap, q = _problem(1, (4, 4, 4), [0] * 6, -1, 0.0)
    with pytest.raises(G.MCError):
        G.fo_solve(cfg, edges, kap, q)                    # no held face
    cfg["dirichlet"] = [1, 0, 0, 0, 0, 0]
    for bad in (dict(k_interface=0), dict(k_interface=4), dict(rtol=0.0), dict(max_iterations=0)):
        with pytest.raises(G.MCError):
            G.fo_solve(dict(cfg, **bad), edges, kap, q)
    r = G.fo_solve(dict(cfg, max_iterations=3, rtol=1e-15), edges, kap, q, check=False)
    assert r["status"] == G.MC_E_RANGE and r["iterations"] == 3


@pytest.mark.parametrize("m,T,d", [(GAN, 300.0, 120e-9), (GAN, 415.0, 2e-6), (SIC, 300.0, 0.0)])
def test_size_limited_conductivity(G, m, T, d):
    import torch
    tab, _ = G.ph_tables(m, T, 4096)
    k = float(G.ph_conductivity(tab, d).cpu()[0])
    torch.cuda.synchronize()
    _, v, Cb, it = P.bin_tables(m, T, 4096)
    rate = it + (v / d if d > 0 else 0.0)
    assert k == pytest.approx((Cb * v * v / (3.0 * rate)).sum(), rel=1e-12)
    assert k == pytest.approx(F.size_limited_kappa(m, T, d), rel=1e-4)


def _chip_inputs(G, geom, heat_W, T):
    """Conductivities from the bins (wire and film size-limited, SiC bulk)
    and 1/R_K of Eq. (3) from GaN's side, then the per-cell fields."""
    tg, _ = G.ph_tables(GAN, T, 2048)
    ts, _ = G.ph_tables(SIC, T, 2048)
    k_wire = float(G.ph_conductivity(tg, 120e-9).cpu()[0])
    k_film = float(G.ph_conductivity(tg, 2e-6).cpu()[0])
    k_sic = float(G.ph_conductivity(ts, 0.0).cpu()[0])
    _, sums = G.ph_interface(GAN, SIC, tg)
    R_K = 1.0 / float(sums.cpu()[0])
    kt = [0.0, k_sic, k_film, k_wire]
    kap, q = G.fo_chip_fields(geom["material"], kt, geom["src_index"], heat_W)
    return kt, R_K, kap, q


def test_chip_fields_and_a_small_chip(G):
    """A small array (5 wires over a 200 nm channel, thin film and
    substrate): the fields equal their definition, and the temperature
    equals the direct solve."""
    dev = W.device_config(n_particles=1000, n_cells=(20, 3, 6), L_nm=(200.0, 60.0, 120.0))
    geom = W.chip_geometry(dev, n_wires=5, margin_x_um=0.4, margin_y_um=0.3, film_um=0.3, substrate_um=1.0)
    heat = np.random.default_rng(3).uniform(0.0, 1e-7, 360)
    kt, R_K, kap, q = _chip_inputs(G, geom, heat, 300.0)
    kap_h, q_h = kap.cpu().numpy(), q.cpu().numpy()
    assert np.array_equal(kap_h, np.asarray(kt)[geom["material"]])
    si = geom["src_index"]
    assert np.array_equal(q_h, np.where(si >= 0, heat[np.maximum(si, 0)], 0.0))
    assert q_h.sum() == pytest.approx(5 * heat.sum(), rel=1e-12)          # five half-wires in the half chip
    cfg = dict(n=geom["n"], dirichlet=[0, 0, 0, 0, 1, 0], k_interface=geom["k_interface"], R_K_m2KW=R_K,
               T_sink_K=300.0, rtol=1e-13, max_iterations=50000)
    _say("small chip", geom["n"], "cells", int(np.prod(geom["n"])))
    r = G.fo_solve(cfg, geom["edges"], kap, q)
    T = r["T"].cpu().numpy()
    ref = F.solve(cfg, geom["edges"], kap_h, q_h)
    assert np.abs(T - ref).max() <= 1e-9 * (ref - 300.0).max()
    assert F.boundary_flux(cfg, geom["edges"], kap_h, T) == pytest.approx(q_h.sum(), rel=1e-9)


def test_full_chip(G):
    """The half chip of 31 wires (1.03e6 cells) under a 1 mW synthetic heat
    map per half-wire: converged, every watt leaves through the sink, the
    middle wire runs hotter than the edge wire (more of the edge wire's heat
    spreads into the film beside the array), the hot spot lies on the drain
    side of the gate."""
    dev = W.device_config(n_particles=1000)
    geom = W.chip_geometry(dev)
    L, nc = dev["L_nm"], dev["n_cells"]
    vc = (L[0] / nc[0]) * (L[1] / nc[1]) * (L[2] / nc[2]) * 1e-27
    heat = W.wire_heat_map(dev, power_W=1e-3) * vc
    kt, R_K, kap, q = _chip_inputs(G, geom, heat, 300.0)
    cfg = dict(n=geom["n"], dirichlet=[0, 0, 0, 0, 1, 0], k_interface=geom["k_interface"], R_K_m2KW=R_K,
               T_sink_K=300.0, rtol=1e-11, max_iterations=100000)
    _say("full chip", geom["n"], "cells", int(np.prod(geom["n"])), "R_K", R_K, "kappa", kt)
    r = G.fo_solve(cfg, geom["edges"], kap, q)
    _say("iterations", r["iterations"], "residual", r["rel_residual"])
    T = r["T"].cpu().numpy()
    kap_h = kap.cpu().numpy()
    assert F.boundary_flux(cfg, geom["edges"], kap_h, T) == pytest.approx(31e-3, rel=1e-8)
    nx, ny, nz = geom["n"]
    T3 = T.reshape(nx, ny, nz)
    kw, i0 = geom["k_wire"], geom["i_wire"]
    wires = T3[i0:i0 + 100, :, kw:]
    step = 12
    mid = wires[:, 0:3].max() - 300.0
    edge = wires[:, 15 * step - 3:15 * step + 3].max() - 300.0
    _say("middle wire rise", mid, "K, edge wire", edge, "K")
    assert mid > edge > 0
    hot = np.unravel_index(np.argmax(T3), T3.shape)
    assert hot[1] < 3 and kw <= hot[2] and 50 <= hot[0] - i0 < 100
