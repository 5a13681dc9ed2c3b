"""GPU parity of the phonon side against the FP64 reference: the bin tables
(sine dispersion, heat capacity, relaxation with and without the electrons
of Eq. (1)), the Fermi level, the transmissivity of Eq. (2), the sums of
Eq. (3) and of the bulk conductivity, and the packet Monte Carlo packet for
packet (same tables, same Philox streams)."""
import sys

import numpy as np
import pytest

from oracle import phonon_oracle as P

pytestmark = pytest.mark.gpu

GAN, SIC = P.table2("GaN"), P.table2("6H-SiC")
ELEC = dict(n_m3=4e24, m_dos=0.21, D_a_eV=8.3, rho=6095.0, v_g=3338.0)


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


@pytest.mark.parametrize("n_m3,T", [(1e20, 300.0), (4e24, 300.0), (4e24, 450.0), (1e27, 30.0)])
def test_fermi_level(G, n_m3, T):
    import torch
    d = G.ph_fermi_level(n_m3, 0.21, T)
    torch.cuda.synchronize()
    want = P.fermi_level(n_m3, 0.21, T)
    assert float(d.cpu()[0]) == pytest.approx(want, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("name,m,elec,nb", [("GaN", GAN, ELEC, 4096), ("GaN", GAN, None, 333), ("SiC", SIC, None, 1000)])
def test_bin_tables(G, name, m, elec, nb):
    import torch
    _say("phonon tables", name, nb, "bins", "with electrons" if elec else "")
    for T in (300.0, 415.0):
        tab, ef = G.ph_tables(m, T, nb, elec)
        torch.cuda.synchronize()
        g = tab.cpu().numpy()
        w, v, Cb, it = P.bin_tables(m, T, nb, electrons=elec)
        for k, ref in enumerate((w, v, Cb, it)):
            assert np.allclose(g[k], ref, rtol=1e-11, atol=0), (k, np.abs(g[k] / ref - 1).max())
        if elec:
            assert float(ef.cpu()[0]) == pytest.approx(P.fermi_level(elec["n_m3"], elec["m_dos"], T), rel=1e-9)


def test_interface_transmissivity_and_resistance(G):
    import torch
    nb = 4096
    for T in (300.0, 415.0):
        tab, _ = G.ph_tables(GAN, T, nb)
        tau, sums = G.ph_interface(GAN, SIC, tab)
        torch.cuda.synchronize()
        w = tab.cpu().numpy()[0]
        assert np.allclose(tau.cpu().numpy(), P.transmissivity(GAN, SIC, w), rtol=1e-12, atol=1e-15)
        inv_rk, kap = sums.cpu().numpy()
        # midpoint sums over 4096 bins against adaptive quadrature
        assert inv_rk == pytest.approx(P.interface_conductance(GAN, SIC, T), rel=1e-5)
        assert kap == pytest.approx(P.kappa(GAN, T), rel=1e-4)
    # from the wider band: SiC modes above GaN's top see no partner
    tab, _ = G.ph_tables(SIC, 300.0, nb)
    tau, sums = G.ph_interface(SIC, GAN, tab)
    torch.cuda.synchronize()
    w = tab.cpu().numpy()[0]
    t = tau.cpu().numpy()
    assert np.all(t[w >= GAN["w_max"]] == 0.0)
    # the same bin sum on the host, to rounding; against the quadrature, the
    # bin holding GaN's band top (where tau_21 jumps to zero) limits the
    # midpoint sum to first order: one bin's share, about 1e-3
    _, v, Cb, _ = P.bin_tables(SIC, 300.0, nb)
    host = (v * Cb * P.transmissivity(SIC, GAN, w)).sum() / 4
    assert float(sums.cpu()[0]) == pytest.approx(host, rel=1e-10)
    assert float(sums.cpu()[0]) == pytest.approx(P.interface_conductance(SIC, GAN, 300.0), rel=2e-3)


def _mc_case(G, oracle_mod, cfg, q, tables, n_packets):
    import torch
    v, it, Cb = tables[1], tables[3], tables[2]
    ref = oracle_mod.phonon_mc(cfg, q, v, it, Cb, n_packets)
    mc = G.PhononMC(dict(cfg, n_bins=len(v), n_packets=n_packets))
    tab = torch.tensor(np.stack(tables), dtype=torch.float64, device="cuda")
    r = mc.ph_mc_run(tab, torch.tensor(q, dtype=torch.float64))
    t = r["t_fs"].cpu().numpy()
    for key in ("scatterings", "wall_specular", "wall_diffuse", "dropped", "segments"):
        assert r[key] == ref[key], (key, r[key], ref[key])
    assert np.array_equal(r["absorbed"], ref["absorbed"])
    scale = np.abs(ref["t_fs"]).max()
    assert np.abs(t - ref["t_fs"]).max() <= 1e-9 * scale, np.abs(t - ref["t_fs"]).max() / scale
    dT = r["dT"].cpu().numpy()
    assert np.abs(dT - ref["dT"]).max() <= 1e-9 * np.abs(ref["dT"]).max()
    return r, ref


def test_packet_monte_carlo_wire_domain(G, oracle_mod):
    """The half wire (100 x 3 x 6 subcells): specular symmetry plane,
    diffuse free surfaces, isothermal contacts and film; heat generated near
    the drain-side gate edge.  Every count equal, per-subcell times and
    temperatures to 1e-9."""
    tables = P.bin_tables(GAN, 300.0, 1024, electrons=ELEC)
    cfg = dict(L_nm=[1000.0, 60.0, 120.0], n_cells=[100, 3, 6],
               faces=["isothermal", "isothermal", "specular", "diffuse", "isothermal", "diffuse"], seed=17,
               instance=3, max_events=1 << 22)
    q = np.zeros(1800)
    q.reshape(100, 18)[70:80] = 1e-6 / 180
    q.reshape(100, 18)[20:25, :9] = 2e-7 / 45
    _say("phonon packets: wire domain, 100003 packets")
    r, ref = _mc_case(G, oracle_mod, cfg, q, tables, 100003)
    assert ref["scatterings"] > 100000 and ref["wall_diffuse"] > 0


def test_packet_monte_carlo_ragged_and_guarded(G, oracle_mod):
    """A ragged 37 x 2 x 5 grid with a bin count that is no power of two,
    packet for packet; and a box with no isothermal face, where every packet
    reaches the event guard and is dropped (counted, nothing hangs)."""
    import torch
    tables = P.bin_tables(SIC, 415.0, 333)
    cfg = dict(L_nm=[370.0, 40.0, 100.0], n_cells=[37, 2, 5],
               faces=["isothermal", "specular", "diffuse", "diffuse", "specular", "isothermal"], seed=5,
               instance=0, max_events=1 << 20)
    q = np.random.default_rng(2).uniform(0.0, 1e-7, 370)
    _mc_case(G, oracle_mod, cfg, q, tables, 7777)

    # The closed box: 500 events per packet.  Over that many reflections a
    # packet's path is chaotic: the device's FP64 log, sin and cos differ
    # from the host's in the last bit now and then, and a shift of one ulp
    # in a flight length decides, a hundred events later, whether a flight
    # ends at a wall or at a scattering (one-ulp changes to the reference's
    # own transcendentals move a few percent of the packets too).  Exact
    # here: every packet dropped, none absorbed, and scatterings plus
    # reflections equal to the guard for every packet; per-packet counts
    # identical for the large majority, totals and subcell times within
    # sampling noise of that minority.
    n, guard = 1000, 500
    closed = dict(cfg, faces=["specular", "diffuse", "specular", "diffuse", "specular", "diffuse"],
                  max_events=guard)
    v, it, Cb = tables[1], tables[3], tables[2]
    ref = oracle_mod.phonon_mc(closed, q, v, it, Cb, n)
    mc = G.PhononMC(dict(closed, n_bins=len(v), n_packets=n))
    tab = torch.tensor(np.stack(tables), dtype=torch.float64, device="cuda")
    r = mc.ph_mc_run(tab, torch.tensor(q, dtype=torch.float64), packet_scatterings=True)
    assert r["dropped"] == n and ref["dropped"] == n
    assert not r["absorbed"].any() and not np.asarray(ref["absorbed"]).any()
    for d in (r, ref):
        assert d["scatterings"] + d["wall_specular"] + d["wall_diffuse"] == n * guard
    same = r["packet_scatterings"] == ref["packet_scatterings"]
    assert same.mean() >= 0.9, same.mean()
    # (one-ulp perturbations of the reference's log, sin and cos move 6 % of
    # the packets, the totals by 1e-4 and no subcell time by more than 1.2 %)
    assert r["scatterings"] == pytest.approx(ref["scatterings"], rel=0.005)
    t, tr = r["t_fs"].cpu().numpy(), ref["t_fs"]
    assert t.sum() == pytest.approx(tr.sum(), rel=0.005)
    assert np.abs(t - tr).max() <= 0.05 * tr.max()
