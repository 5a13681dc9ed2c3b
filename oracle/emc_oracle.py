"""ctypes wrapper of the FP64 CPU reference (emc_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg; the GPU product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "emc_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "phonon_mc_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

NV, NM, NF = 3, 10, 7
MECH_NAMES = ["ac", "ii", "pop_ab", "pop_em", "iv_ab_G1", "iv_em_G1", "iv_ab_U", "iv_em_U", "iv_ab_G3", "iv_em_G3"]


class OrConfig(C.Structure):
    _fields_ = [
        ("m_eff", C.c_double * 3), ("alpha", C.c_double * 3), ("E_c", C.c_double * 3),
        ("Z", C.c_int * 3),
        ("eps_s", C.c_double), ("eps_inf", C.c_double), ("rho", C.c_double), ("D_ac_eV", C.c_double),
        ("D_iv_eVm", C.c_double), ("hw_lo_eV", C.c_double), ("hw_iv_eV", C.c_double), ("u_ac", C.c_double),
        ("mode", C.c_int), ("pad0", C.c_int),
        ("seed", C.c_uint64), ("instance", C.c_uint32),
        ("n_particles", C.c_int), ("capacity", C.c_int),
        ("dt_fs", C.c_double), ("substeps", C.c_int), ("n_bins", C.c_int), ("dE_eV", C.c_double),
        ("T0_K", C.c_double), ("T_init_K", C.c_double), ("N_D_m3", C.c_double),
        ("F_bulk", C.c_double * 3), ("L_nm", C.c_double * 3), ("n_cells", C.c_int * 3), ("pad1", C.c_int),
        ("gate_x_nm", C.c_double * 2), ("Vgs", C.c_double), ("Vds", C.c_double), ("phi_offset", C.c_double),
    ]


class OrObs(C.Structure):
    _fields_ = [
        ("intervals", C.c_int), ("pad", C.c_int), ("t_window_s", C.c_double),
        ("I_D", C.c_double), ("I_S", C.c_double), ("P_heat_W", C.c_double), ("P_emit_W", C.c_double),
        ("E_out_J", C.c_double * 2), ("E_in_J", C.c_double * 2), ("dE_ens_J", C.c_double), ("W_field_J", C.c_double), ("E_abs_J", C.c_double),
        ("v_drift_ms", C.c_double * 3), ("mean_E_eV", C.c_double), ("valley_frac", C.c_double * 3),
        ("half_mean", C.c_double * 4), ("half_se", C.c_double * 4), ("steady", C.c_int),
    ]


class OrPhConfig(C.Structure):
    _fields_ = [("L_nm", C.c_double * 3), ("n_cells", C.c_int * 3), ("face", C.c_int * 6), ("n_bins", C.c_int),
                ("seed", C.c_uint64), ("instance", C.c_uint32), ("max_events", C.c_int)]


class OrPhCounts(C.Structure):
    _fields_ = [("scatterings", C.c_uint64), ("wall_specular", C.c_uint64), ("wall_diffuse", C.c_uint64),
                ("absorbed", C.c_uint64 * 6), ("dropped", C.c_uint64), ("segments", C.c_uint64),
                ("path_nm", C.c_double)]


FACE = {"specular": 0, "diffuse": 1, "isothermal": 2}


def phonon_mc(cfg: dict, q_cell, v_ms, inv_tau, C_bin, n_packets: int, threads: int = 0) -> dict:
    """Steady-state phonon packets of the wire domain (see phonon_mc_oracle.c):
    cfg has L_nm, n_cells, faces (six of 'specular', 'diffuse', 'isothermal'
    for x0 x1 y0 y1 z0 z1), seed, instance, max_events; q_cell the power per
    subcell (W, either sign: a sink's packets carry negative energy); per
    frequency bin the group velocity (m/s), relaxation rate
    (1/s) and heat capacity (J/(m^3 K)).  Returns the time packets spent per
    subcell (fs), the temperature rise per subcell (K) and the counts."""
    c = OrPhConfig()
    c.L_nm[:] = [float(x) for x in cfg["L_nm"]]
    c.n_cells[:] = [int(x) for x in cfg["n_cells"]]
    c.face[:] = [FACE[f] for f in cfg["faces"]]
    v = np.ascontiguousarray(np.asarray(v_ms, np.float64) * 1e-6)            # nm/fs
    tau = np.ascontiguousarray(1e15 / np.asarray(inv_tau, np.float64))         # fs
    Cb = np.asarray(C_bin, np.float64)
    c.n_bins = int(v.size)
    c.seed = int(cfg["seed"]) & 0xFFFFFFFFFFFFFFFF
    c.instance = int(cfg.get("instance", 0))
    c.max_events = int(cfg.get("max_events", 1 << 20))
    emit = Cb * np.asarray(inv_tau, np.float64)
    cum = np.ascontiguousarray(np.cumsum(emit))   # in bin order
    q = np.ascontiguousarray(q_cell, np.float64)
    nc = int(np.prod(cfg["n_cells"]))
    t = np.zeros(nc)
    cnt = OrPhCounts()
    pk = np.zeros(int(n_packets), np.uint32)
    lib().or_ph_run(C.byref(c), _p(q, C.c_double), _p(v, C.c_double), _p(tau, C.c_double), _p(cum, C.c_double),
                    int(n_packets), int(threads), _p(t, C.c_double), C.byref(cnt), _p(pk, C.c_uint32))
    P = float(np.abs(q).sum())
    Vc = np.prod(np.asarray(cfg["L_nm"], float) / np.asarray(cfg["n_cells"], float)) * 1e-27
    dT = P * t * 1e-15 / n_packets / (Cb.sum() * Vc)
    return dict(t_fs=t, dT=dT, scatterings=int(cnt.scatterings), wall_specular=int(cnt.wall_specular),
                wall_diffuse=int(cnt.wall_diffuse), absorbed=np.array(cnt.absorbed[:], np.int64),
                dropped=int(cnt.dropped), segments=int(cnt.segments), path_nm=cnt.path_nm, packet_scatterings=pk)


def build(force: bool = False) -> str:
    """Compile the reference with gcc (plain -O2: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp, u32p, u64p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                C.POINTER(C.c_int32))
        L.or_philox.argtypes = [u32p, u32p, u32p]
        L.or_kane_energy.argtypes = [C.c_double, C.c_double]
        L.or_kane_energy.restype = C.c_double
        L.or_rate.argtypes = [C.POINTER(OrConfig), C.c_int, C.c_int, C.c_double, C.c_double]
        L.or_rate.restype = C.c_double
        L.or_dos.argtypes = [C.POINTER(OrConfig), C.c_int, C.c_double]
        L.or_dos.restype = C.c_double
        L.or_onb.argtypes = [dp, dp, dp]
        L.or_create.argtypes = [C.POINTER(OrConfig), dp]
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_run.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.or_run.restype = C.c_int
        L.or_poisson_update.argtypes = [C.c_void_p]
        L.or_reset_window.argtypes = [C.c_void_p]
        L.or_set_temperature.argtypes = [C.c_void_p, dp]
        L.or_set_tables.argtypes = [C.c_void_p, dp, dp]
        L.or_ncell.argtypes = [C.c_void_p]
        L.or_ncell.restype = C.c_int
        L.or_weight.argtypes = [C.c_void_p]
        L.or_weight.restype = C.c_double
        for f in ("or_intervals_done", "or_window_intervals", "or_next_id"):
            getattr(L, f).argtypes = [C.c_void_p]
            getattr(L, f).restype = C.c_uint32
        L.or_gamma.argtypes = [C.c_void_p, dp]
        L.or_tables.argtypes = [C.c_void_p, dp, dp]
        L.or_factors.argtypes = [C.c_void_p, dp]
        L.or_get_particles.argtypes = [C.c_void_p, dp, dp, i32p, i32p, u32p]
        L.or_set_particles.argtypes = [C.c_void_p, dp, dp, i32p, i32p, u32p]
        L.or_set_progress.argtypes = [C.c_void_p, C.c_int, C.c_uint32]
        L.or_get_fields.argtypes = [C.c_void_p, dp, dp, u32p]
        L.or_get_counts.argtypes = [C.c_void_p, u64p]
        L.or_get_maps.argtypes = [C.c_void_p, u64p, u64p]
        L.or_history.argtypes = [C.c_void_p, dp, C.c_int]
        L.or_history.restype = C.c_int
        L.or_poisson_solve.argtypes = [C.c_void_p, dp, dp, dp]
        L.or_sample_selection.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_uint32, C.c_int, u64p]
        L.or_scatter_once.argtypes = [C.c_void_p, dp, i32p, C.c_int, u32p]
        L.or_scatter_once.restype = C.c_int
        L.or_steady_test.argtypes = [dp, C.c_int, dp]
        L.or_steady_test.restype = C.c_int
        L.or_power_maps.argtypes = [C.c_void_p, dp, dp, dp]
        L.or_observables.argtypes = [C.c_void_p, C.POINTER(OrObs)]
        L.or_ensemble_energy.argtypes = [C.c_void_p]
        L.or_ensemble_energy.restype = C.c_double
        L.or_ph_run.argtypes = [C.POINTER(OrPhConfig), dp, dp, dp, dp, C.c_long, C.c_int, dp, C.POINTER(OrPhCounts),
                                u32p]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def make_config(cfg: dict) -> OrConfig:
    m = cfg["material"]
    c = OrConfig()
    for name in ("m_eff", "alpha", "E_c"):
        getattr(c, name)[:] = [float(x) for x in m[name]]
    c.Z[:] = [int(x) for x in m["Z"]]
    for name in ("eps_s", "eps_inf", "rho", "D_ac_eV", "D_iv_eVm", "hw_lo_eV", "hw_iv_eV", "u_ac"):
        setattr(c, name, float(m[name]))
    c.mode = 1 if cfg["mode"] == "device" else 0
    c.seed = int(cfg["seed"]) & 0xFFFFFFFFFFFFFFFF
    c.instance = int(cfg.get("instance", 0))
    c.n_particles = int(cfg["n_particles"])
    c.capacity = int(cfg["capacity"])
    c.dt_fs = float(cfg["dt_fs"])
    c.substeps = int(cfg["substeps"])
    c.n_bins = int(cfg["n_bins"])
    c.dE_eV = float(cfg["dE_eV"])
    c.T0_K = float(cfg["T0_K"])
    c.T_init_K = float(cfg.get("T_init_K", cfg["T0_K"]))
    c.N_D_m3 = float(cfg["N_D_m3"])
    c.F_bulk[:] = [float(x) for x in cfg["F_bulk"]]
    c.L_nm[:] = [float(x) for x in cfg["L_nm"]]
    c.n_cells[:] = [int(x) for x in cfg["n_cells"]]
    c.gate_x_nm[:] = [float(x) for x in cfg["gate_x_nm"]]
    c.Vgs, c.Vds, c.phi_offset = float(cfg["Vgs"]), float(cfg["Vds"]), float(cfg["phi_offset"])
    return c


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def kane_energy(gamma: float, alpha: float) -> float:
    return lib().or_kane_energy(float(gamma), float(alpha))


def rate(cfg: dict, valley: int, mech: int, E_eV: float, T: float) -> float:
    """Analytic rate (1/s) of mechanism `mech` in `valley` at kinetic energy E."""
    c = make_config(cfg)
    return lib().or_rate(C.byref(c), int(valley), int(mech), float(E_eV), float(T))


def dos(cfg: dict, valley: int, E_eV: float) -> float:
    c = make_config(cfg)
    return lib().or_dos(C.byref(c), int(valley), float(E_eV))


def steady_test(series) -> tuple[int, np.ndarray]:
    """Steady-state test of a per-interval series: (flag, [mean1, mean2,
    se1, se2]) for the two halves of its last 2*(m//2) values."""
    a = np.ascontiguousarray(series, dtype=np.float64)
    out = np.zeros(4)
    f = lib().or_steady_test(_p(a, C.c_double), int(a.size), _p(out, C.c_double))
    return f, out


def onb(n):
    n = np.ascontiguousarray(n, dtype=np.float64)
    e1, e2 = np.zeros(3), np.zeros(3)
    lib().or_onb(_p(n, C.c_double), _p(e1, C.c_double), _p(e2, C.c_double))
    return e1, e2


class Oracle:
    """One ensemble (one instance) of the reference Monte Carlo."""

    def __init__(self, cfg: dict, T_cells=None):
        self.cfg = cfg
        self._c = make_config(cfg)
        T = T_cells if T_cells is not None else cfg.get("T_cells")
        self._T = None if T is None else np.ascontiguousarray(T, dtype=np.float64)
        self._h = lib().or_create(C.byref(self._c), None if self._T is None else _p(self._T, C.c_double))
        self.ncell = lib().or_ncell(self._h)
        self.cap = int(cfg["capacity"])
        self.nb = int(cfg["n_bins"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    def run(self, n_intervals: int, threads: int = 0) -> int:
        return lib().or_run(self._h, int(n_intervals), int(threads))

    def poisson_update(self):
        lib().or_poisson_update(self._h)

    def reset_window(self):
        lib().or_reset_window(self._h)

    def set_temperature(self, T):
        self._T = np.ascontiguousarray(T, dtype=np.float64)
        lib().or_set_temperature(self._h, _p(self._T, C.c_double))

    def set_tables(self, shape, k4):
        s = np.ascontiguousarray(shape, dtype=np.float64)
        k = np.ascontiguousarray(k4, dtype=np.float64)
        lib().or_set_tables(self._h, _p(s, C.c_double), _p(k, C.c_double))

    @property
    def weight(self) -> float:
        return lib().or_weight(self._h)

    @property
    def intervals_done(self) -> int:
        return lib().or_intervals_done(self._h)

    @property
    def window_intervals(self) -> int:
        return lib().or_window_intervals(self._h)

    @property
    def next_id(self) -> int:
        return lib().or_next_id(self._h)

    def gamma(self) -> np.ndarray:
        g = np.zeros(NV)
        lib().or_gamma(self._h, _p(g, C.c_double))
        return g

    def tables(self):
        s = np.zeros((NV, self.nb, NM))
        k = np.zeros((NV, self.nb))
        lib().or_tables(self._h, _p(s, C.c_double), _p(k, C.c_double))
        return s, k

    def factors(self) -> np.ndarray:
        f = np.zeros((self.ncell, NF))
        lib().or_factors(self._h, _p(f, C.c_double))
        return f

    def particles(self) -> dict:
        k = np.zeros((self.cap, 3)); r = np.zeros((self.cap, 3))
        v = np.zeros(self.cap, np.int32); a = np.zeros(self.cap, np.int32); i = np.zeros(self.cap, np.uint32)
        lib().or_get_particles(self._h, _p(k, C.c_double), _p(r, C.c_double), _p(v, C.c_int32),
                               _p(a, C.c_int32), _p(i, C.c_uint32))
        return dict(k=k, r=r, valley=v, alive=a, id=i)

    def set_particles(self, k, r, valley, alive, ident):
        k = np.ascontiguousarray(k, dtype=np.float64); r = np.ascontiguousarray(r, dtype=np.float64)
        v = np.ascontiguousarray(valley, dtype=np.int32); a = np.ascontiguousarray(alive, dtype=np.int32)
        i = np.ascontiguousarray(ident, dtype=np.uint32)
        lib().or_set_particles(self._h, _p(k, C.c_double), _p(r, C.c_double), _p(v, C.c_int32),
                               _p(a, C.c_int32), _p(i, C.c_uint32))

    def set_progress(self, n_done: int, next_id: int):
        """Continue from interval `n_done` with identities from `next_id`."""
        lib().or_set_progress(self._h, int(n_done), int(next_id))

    def fields(self):
        phi = np.zeros(self.ncell); F = np.zeros((self.ncell, 3)); n = np.zeros(self.ncell, np.uint32)
        lib().or_get_fields(self._h, _p(phi, C.c_double), _p(F, C.c_double), _p(n, C.c_uint32))
        return phi, F, n

    def counts(self) -> dict:
        o = np.zeros(38, np.uint64)
        lib().or_get_counts(self._h, _p(o, C.c_uint64))
        return dict(selections=int(o[0]), self_events=int(o[1]), overflow=int(o[2]),
                    real=o[3:33].reshape(NV, NM).astype(np.int64),
                    exits=o[33:35].astype(np.int64), injections=o[35:37].astype(np.int64),
                    reflect_guard=int(o[37]))

    def maps(self):
        heat = np.zeros((self.ncell, 4), np.uint64)
        dens = np.zeros(self.ncell, np.uint64)
        lib().or_get_maps(self._h, _p(heat, C.c_uint64), _p(dens, C.c_uint64))
        return heat, dens

    def history(self, max_rows: int = 1 << 16) -> np.ndarray:
        rows = np.zeros((max_rows, 8))
        n = lib().or_history(self._h, _p(rows, C.c_double), int(max_rows))
        return rows[:n].copy()

    def power_maps(self):
        """Window maps: net and emission-only phonon power density (W/m^3),
        electron density (1/m^3)."""
        qn, qe, n = np.zeros(self.ncell), np.zeros(self.ncell), np.zeros(self.ncell)
        lib().or_power_maps(self._h, _p(qn, C.c_double), _p(qe, C.c_double), _p(n, C.c_double))
        return qn, qe, n

    def observables(self) -> dict:
        o = OrObs()
        lib().or_observables(self._h, C.byref(o))
        return dict(intervals=o.intervals, t_window_s=o.t_window_s, I_D=o.I_D, I_S=o.I_S,
                    P_heat_W=o.P_heat_W, P_emit_W=o.P_emit_W, E_out_J=np.array(o.E_out_J[:]),
                    E_in_J=np.array(o.E_in_J[:]), dE_ens_J=o.dE_ens_J, W_field_J=o.W_field_J, E_abs_J=o.E_abs_J, v_drift_ms=np.array(o.v_drift_ms[:]),
                    mean_E_eV=o.mean_E_eV, valley_frac=np.array(o.valley_frac[:]),
                    half_mean=np.array(o.half_mean[:]).reshape(2, 2), half_se=np.array(o.half_se[:]).reshape(2, 2),
                    steady=o.steady)

    def ensemble_energy_eV(self) -> float:
        return lib().or_ensemble_energy(self._h)

    def poisson_solve(self, charge_C):
        q = np.ascontiguousarray(charge_C, dtype=np.float64)
        phi = np.zeros(self.ncell); F = np.zeros((self.ncell, 3))
        lib().or_poisson_solve(self._h, _p(q, C.c_double), _p(phi, C.c_double), _p(F, C.c_double))
        return phi, F

    def sample_selection(self, valley: int, E_eV: float, cell: int, pid: int, n: int) -> np.ndarray:
        counts = np.zeros(NM + 1, np.uint64)
        lib().or_sample_selection(self._h, int(valley), float(E_eV), int(cell), int(pid), int(n),
                                  _p(counts, C.c_uint64))
        return counts.astype(np.int64)

    def scatter_once(self, k, valley: int, cell: int, words):
        kk = np.ascontiguousarray(k, dtype=np.float64).copy()
        v = np.array([valley], np.int32)
        w = np.ascontiguousarray(words, dtype=np.uint32)
        m = lib().or_scatter_once(self._h, _p(kk, C.c_double), _p(v, C.c_int32), int(cell), _p(w, C.c_uint32))
        return m, kk, int(v[0])
