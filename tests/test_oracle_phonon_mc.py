"""Pins of the reference phonon Monte Carlo (steady-state energy packets in
the wire domain): the diffusive limit against Fourier's law with the
kinetic conductivity of the same frequency bins, the ballistic limit
against brute-force chord lengths, and energy conservation through the
isothermal faces."""
import math

import numpy as np
import pytest

from oracle import phonon_oracle as P

GAN = P.table2("GaN")


def _bar(n_cells, L, faces, seed=3):
    return dict(L_nm=[L[0], L[1], L[2]], n_cells=list(n_cells), faces=faces, seed=seed, instance=0,
                max_events=1 << 24)


def test_diffusive_limit_is_fouriers_law(oracle_mod):
    """A 400 nm bar with specular sides and isothermal ends, uniform heat
    generation Q, relaxation times that vary with frequency (mean free paths
    from 12 nm at low frequency to 6 nm at the top of the band): the
    temperature rise approaches Q x (L - x) / (2 kappa) with
    kappa = sum_b C_b v_b^2 tau_b / 3.  Only a re-emission that leaves the
    time-weighted bin occupation proportional to C_b gives this kappa."""
    w, v, Cb, _ = P.bin_tables(GAN, 300.0, 256)
    mfp = 6e-9 + 6e-9 * (1.0 - w / GAN["w_max"])
    it = v / mfp
    L, nx = 400.0, 40
    cfg = _bar((nx, 1, 1), (L, 20.0, 20.0), ["isothermal", "isothermal"] + ["specular"] * 4)
    Q = 1e15                                             # W/m^3
    Vc = (L / nx) * 20.0 * 20.0 * 1e-27
    q = np.full(nx, Q * Vc)
    r = oracle_mod.phonon_mc(cfg, q, v, it, Cb, 40000)
    assert r["dropped"] == 0 and r["absorbed"].sum() == 40000
    kappa = (Cb * v * v / it).sum() / 3.0
    xc = (np.arange(nx) + 0.5) * L / nx * 1e-9
    # inside, the profile is Fourier's parabola -Q (x - L/2)^2 / (2 kappa)
    # lifted by the temperature slip at the absorbing ends (about a mean
    # free path times the wall flux over kappa): fit both
    mid = slice(4, 36)
    X = np.stack([np.ones(nx), (xc - L * 0.5e-9) ** 2], axis=1)[mid]
    (a, b), *_ = np.linalg.lstsq(X, r["dT"][mid], rcond=None)
    assert -Q / (2 * b) == pytest.approx(kappa, rel=0.03)
    slip = a - Q * (L * 0.5e-9) ** 2 / (2 * kappa)
    q_wall, mfp_mean = Q * L * 0.5e-9, 9e-9
    assert 0.2 * q_wall * mfp_mean / kappa < slip < 2.0 * q_wall * mfp_mean / kappa


def test_ballistic_limit_matches_chord_lengths(oracle_mod):
    """No scattering, a 200 x 100 x 50 nm box with isothermal faces, uniform
    generation: a packet lives for its distance to the boundary along its
    flight divided by its speed.  The time per packet equals the mean of that
    distance (brute force over uniform points and directions) times the mean
    of 1/v over the emitted bins."""
    w, v, Cb, _ = P.bin_tables(GAN, 300.0, 64)
    it = np.full(64, 1e-30)                              # no scattering; emission weights proportional to C_b
    L = np.array([200.0, 100.0, 50.0])
    cfg = _bar((4, 2, 1), L, ["isothermal"] * 6)
    q = np.full(8, 1.0)
    n = 200000
    r = oracle_mod.phonon_mc(cfg, q, v, it, Cb, n)
    assert r["scatterings"] == 0 and r["absorbed"].sum() == n
    rng = np.random.default_rng(11)
    m = 2_000_000
    x = rng.uniform(0.0, 1.0, (m, 3)) * L
    mu = rng.uniform(-1.0, 1.0, m)
    ph = rng.uniform(0.0, 2 * math.pi, m)
    s = np.sqrt(1 - mu * mu)
    d = np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)
    with np.errstate(divide="ignore"):
        t = np.where(d > 0, (L - x) / d, np.where(d < 0, -x / d, np.inf))
    dist = t.min(axis=1)
    p = Cb / Cb.sum()
    inv_v = (p / (v * 1e-6)).sum()                       # fs per nm
    want = dist.mean() * inv_v
    got = r["t_fs"].sum() / n
    # sampling error of both estimates (distance and speed are independent)
    sig = math.hypot(dist.std() / math.sqrt(m) * inv_v,
                     math.sqrt((dist ** 2).mean() * (p / (v * 1e-6) ** 2).sum() - want ** 2) / math.sqrt(n))
    assert abs(got - want) < 4 * sig, (got, want, sig)


def test_specular_and_diffuse_walls_conserve_packets(oracle_mod):
    """The wire's own faces: specular symmetry plane, diffuse free surfaces,
    isothermal contacts and film: every packet ends at an isothermal face,
    none at a specular or diffuse one, and the temperature rises most where
    the heat is generated."""
    w, v, Cb, it = P.bin_tables(GAN, 300.0, 512)
    cfg = _bar((100, 3, 6), (1000.0, 60.0, 120.0),
               ["isothermal", "isothermal", "specular", "diffuse", "isothermal", "diffuse"])
    q = np.zeros(1800)
    q.reshape(100, 18)[70:80] = 1e-6 / 180
    r = oracle_mod.phonon_mc(cfg, q, v, it, Cb, 20000)
    assert r["absorbed"].sum() == 20000 and r["dropped"] == 0
    assert r["absorbed"][2] == r["absorbed"][3] == r["absorbed"][5] == 0
    assert r["wall_specular"] > 0 and r["wall_diffuse"] > 0
    prof = r["dT"].reshape(100, 18).mean(1)
    assert 70 <= int(np.argmax(prof)) < 80


def test_sinks_carry_negative_packets(oracle_mod):
    """A subcell where the electrons absorb more phonon energy than they emit
    is a heat sink: its packets carry negative energy.  Reversing every
    source reverses every temperature rise exactly (same packets, same
    paths); in a box that is mirror-symmetric in x, a source in the left half
    and the mirrored sink in the right half give an antisymmetric profile,
    and its size is set by the sum of |q| (a total of q, zero here, would
    give no rise at all)."""
    w, v, Cb, _ = P.bin_tables(GAN, 300.0, 64)
    it = np.full(64, 1e-30)                              # ballistic: no scattering
    L = np.array([200.0, 100.0, 50.0])
    cfg = _bar((4, 2, 1), L, ["isothermal"] * 6)
    q = np.array([1.0, 1.0, 0.5, 0.5, -0.5, -0.5, -1.0, -1.0])   # index (ix*2 + iy)
    a = oracle_mod.phonon_mc(cfg, q, v, it, Cb, 30000, threads=1)    # one thread: one summation order
    b = oracle_mod.phonon_mc(cfg, -q, v, it, Cb, 30000, threads=1)
    assert np.array_equal(a["dT"], -b["dT"]) and np.array_equal(a["packet_scatterings"], b["packet_scatterings"])
    assert a["absorbed"].sum() == 30000
    R, A = [], []
    for seed in range(10):
        r = oracle_mod.phonon_mc(dict(cfg, seed=100 + seed), q, v, it, Cb, 20000)["dT"].reshape(4, 2)
        R.append((r + r[::-1]).sum())                    # zero by the mirror symmetry
        A.append(r[:2].sum() - r[2:].sum())
    R, A = np.array(R), np.array(A)
    se = lambda x: x.std(ddof=1) / math.sqrt(len(x))
    assert abs(R.mean()) < 4 * se(R), (R.mean(), se(R))
    assert A.mean() > 20 * se(A)
    # the same packets from |q|, all positive: the rise of the left half is
    # the same packets' time, so it equals the signed run's there up to the
    # right half's negative packets that cross over
    pos = oracle_mod.phonon_mc(dict(cfg, seed=100), np.abs(q), v, it, Cb, 20000)["dT"].reshape(4, 2)
    mix = oracle_mod.phonon_mc(dict(cfg, seed=100), q, v, it, Cb, 20000)["dT"].reshape(4, 2)
    half = 0.5 * (pos + mix)                             # the positive packets alone
    assert np.all(half >= -1e-12 * np.abs(pos).max()) and np.all(pos - half >= -1e-12 * np.abs(pos).max())
    assert mix[0].sum() > 0.5 * pos[0].sum()
