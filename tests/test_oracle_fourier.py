"""Pins of the reference Fourier's-law spreading (coupling paragraph): the
finite-volume system against exact piecewise-linear profiles along each
axis (with the interface resistance jump), energy conservation through the
sinks, Green's reciprocity of the assembled operator, mirror symmetry; and
the size-limited conductivities against their bulk and ballistic limits."""
import math

import numpy as np
import pytest

from oracle import fourier_oracle as F
from oracle import phonon_oracle as P

GAN = P.table2("GaN")


def _edges(widths):
    return np.concatenate([[0.0], np.cumsum(widths)])


@pytest.mark.parametrize("ax", [0, 1, 2])
def test_flux_through_layers_is_exact(ax):
    """Heat generated in the last cell along `ax` only, the first face held:
    every face below carries the same flux F, so the rise at the cell centres
    is exactly F times the series resistance from the sink, with the jump
    F R_K at the interface plane (z only), on a non-uniform grid."""
    rng = np.random.default_rng(ax)
    n_ax, n_t = 17, 3
    w_ax = rng.uniform(20e-9, 200e-9, n_ax)
    w_t = np.full(n_t, 50e-9)
    k_iface = 7
    kap_ax = np.where(np.arange(n_ax) < k_iface, 150.0, 40.0)
    n = [n_t, n_t, n_t]
    n[ax] = n_ax
    widths = [w_t, w_t, w_t]
    widths[ax] = w_ax
    shape = tuple(n)
    kap = np.broadcast_to(np.expand_dims(kap_ax, [a for a in range(3) if a != ax]), shape).copy()
    area = 50e-9 * 50e-9
    q = np.zeros(shape)
    sl = [slice(None)] * 3
    sl[ax] = -1
    q[tuple(sl)] = 1e-6                                  # W per cell of the last layer
    dirichlet = [0] * 6
    dirichlet[2 * ax] = 1
    R_K = 3e-9 if ax == 2 else 0.0
    cfg = dict(n=n, dirichlet=dirichlet, k_interface=k_iface if ax == 2 else -1, R_K_m2KW=R_K, T_sink_K=300.0)
    T = F.solve(cfg, [_edges(w) for w in widths], kap.ravel(), q.ravel()).reshape(shape)
    prof = np.moveaxis(T, ax, 0)[:, 0, 0] - 300.0
    flux = 1e-6 / area                                   # W/m^2 through every face below the last cell
    want = np.zeros(n_ax)
    r = w_ax[0] / (2 * kap_ax[0])
    want[0] = flux * r
    for i in range(1, n_ax):
        r += w_ax[i - 1] / (2 * kap_ax[i - 1]) + w_ax[i] / (2 * kap_ax[i]) + (R_K if i == k_iface else 0.0)
        want[i] = flux * r
    assert np.allclose(prof[:-1], want[:-1], rtol=1e-11)
    assert np.allclose(np.moveaxis(T, ax, 0) - 300.0, prof[:, None, None], rtol=1e-11)


def _random_problem(seed, nx=9, ny=8, nz=7):
    rng = np.random.default_rng(seed)
    edges = [_edges(rng.uniform(10e-9, 300e-9, m)) for m in (nx, ny, nz)]
    kap = rng.uniform(20.0, 400.0, (nx, ny, nz))
    kap[2:4, 3:6, 5:] = 0.0                              # a void
    q = rng.uniform(0.0, 1e-6, (nx, ny, nz))
    cfg = dict(n=[nx, ny, nz], dirichlet=[1, 0, 0, 0, 1, 0], k_interface=3, R_K_m2KW=2e-9, T_sink_K=290.0)
    return cfg, edges, kap.ravel(), q.ravel()


def test_heat_leaves_through_the_sinks():
    cfg, edges, kap, q = _random_problem(1)
    T = F.solve(cfg, edges, kap, q)
    live = kap > 0
    assert F.boundary_flux(cfg, edges, kap, T) == pytest.approx(q[live].sum(), rel=1e-10)
    assert np.all(T[~live] == 290.0) and np.all(T[live] > 290.0)


def test_reciprocity_and_mirror_symmetry():
    cfg, edges, kap, _ = _random_problem(2)
    nc = kap.size
    i, j = 17, 401
    ei, ej = np.zeros(nc), np.zeros(nc)
    ei[i], ej[j] = 1e-6, 1e-6
    Ti, Tj = F.solve(cfg, edges, kap, ei), F.solve(cfg, edges, kap, ej)
    assert Ti[j] - 290.0 == pytest.approx(Tj[i] - 290.0, rel=1e-10)
    # a problem symmetric under x -> L - x
    rng = np.random.default_rng(3)
    wx = rng.uniform(20e-9, 100e-9, 5)
    wx = np.concatenate([wx, wx[::-1]])
    kap = rng.uniform(20.0, 400.0, (10, 4, 5))
    kap = 0.5 * (kap + kap[::-1])
    q = rng.uniform(0.0, 1e-6, (10, 4, 5))
    q = 0.5 * (q + q[::-1])
    cfg = dict(n=[10, 4, 5], dirichlet=[1, 1, 0, 0, 1, 0], k_interface=2, R_K_m2KW=1e-9, T_sink_K=300.0)
    T = F.solve(cfg, [_edges(wx), _edges(np.full(4, 30e-9)), _edges(np.full(5, 40e-9))], kap.ravel(),
                q.ravel()).reshape(10, 4, 5)
    assert np.allclose(T, T[::-1], rtol=1e-12)


def test_size_limited_conductivity_limits():
    """Matthiessen's rule with 1/tau + v/d: a size far above every mean free
    path leaves the bulk value; a size far below them gives the ballistic
    (1/3) sum C v d; in between, the 2 um film and the 120 nm wire of the
    device keep about 55% and 16% of GaN's 228 W/m/K at 300 K."""
    bulk = P.kappa(GAN, 300.0)
    assert F.size_limited_kappa(GAN, 300.0, 1.0) == pytest.approx(bulk, rel=1e-3)
    d = 1e-12
    cv = 3.0 * __import__("scipy").integrate.quad(
        lambda w: float(P.heat_capacity(GAN, w, 300.0) * P.vg_of_w(GAN, w)), 0.0, GAN["w_max"], limit=400)[0]
    assert F.size_limited_kappa(GAN, 300.0, d) == pytest.approx(cv * d / 3.0, rel=1e-3)
    film, wire = F.size_limited_kappa(GAN, 300.0, 2e-6), F.size_limited_kappa(GAN, 300.0, 120e-9)
    assert 0.5 < film / bulk < 0.6 and 0.13 < wire / bulk < 0.19
