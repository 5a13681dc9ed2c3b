"""Thin ctypes binding of libgfmc.so (C ABI in include/gfmc.h).

Argument marshalling only: every step of the Monte Carlo runs in the HIP
kernels of the library.  PyTorch supplies the device workspace and the stream.
The binding raises if the library is not built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfmc.so")

MC_OK, MC_E_ARG, MC_E_HIP, MC_E_CAPACITY, MC_E_RANGE, MC_E_STATE, MC_E_NAN = 0, -1, -2, -3, -4, -5, -6
MC_PREC_FP64, MC_PREC_FP32_STATE = 0, 1
MC_BULK, MC_DEVICE = 0, 1


class McMaterial(C.Structure):
    _fields_ = [("m_eff", C.c_double * 3), ("alpha", C.c_double * 3), ("E_c", C.c_double * 3),
                ("Z", C.c_int32 * 3), ("eps_s", C.c_double), ("eps_inf", C.c_double), ("rho", C.c_double),
                ("D_ac_eV", C.c_double), ("D_iv_eVm", C.c_double), ("hw_lo_eV", C.c_double),
                ("hw_iv_eV", C.c_double), ("u_ac", C.c_double)]


class McConfig(C.Structure):
    _fields_ = [("mode", C.c_int), ("prec", C.c_int), ("mat", McMaterial), ("seed", C.c_uint64),
                ("instance", C.c_uint32), ("n_particles", C.c_int32), ("capacity", C.c_int32),
                ("dt_fs", C.c_double), ("substeps", C.c_int32), ("n_bins", C.c_int32), ("dE_eV", C.c_double),
                ("T0_K", C.c_double), ("T_init_K", C.c_double), ("N_D_m3", C.c_double),
                ("F_bulk", C.c_double * 3), ("L_nm", C.c_double * 3), ("n_cells", C.c_int32 * 3),
                ("gate_x_nm", C.c_double * 2), ("Vgs", C.c_double), ("Vds", C.c_double),
                ("phi_offset", C.c_double)]


class McTallyOut(C.Structure):
    _fields_ = [("intervals", C.c_uint32), ("intervals_total", C.c_uint32), ("t_window_fs", C.c_double),
                ("n_alive", C.c_uint64), ("selections", C.c_uint64), ("self_events", C.c_uint64),
                ("overflow", C.c_uint64), ("real", (C.c_uint64 * 10) * 3), ("exits", C.c_uint64 * 2),
                ("injections", C.c_uint64 * 2), ("segments", C.c_uint64), ("reflect_guard", C.c_uint64),
                ("weight", C.c_double), ("drain_current_A", C.c_double), ("flags", C.c_int32)]


class McObservablesOut(C.Structure):
    _fields_ = [("intervals", C.c_uint32), ("t_window_fs", C.c_double), ("drain_current_A", C.c_double),
                ("source_current_A", C.c_double), ("heat_W", C.c_double), ("emit_W", C.c_double),
                ("drift_velocity_ms", C.c_double * 3), ("mean_energy_eV", C.c_double),
                ("valley_fraction", C.c_double * 3), ("half_mean", C.c_double * 4), ("half_se", C.c_double * 4),
                ("steady", C.c_int32)]


class McParticlesView(C.Structure):
    _fields_ = [("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("z", C.c_void_p), ("meta", C.c_void_p), ("capacity", C.c_int32),
                ("elem_bytes", C.c_int32)]


EXPORTS = ["mc_status_string", "mc_last_error", "mc_workspace_bytes", "mc_init", "mc_destroy",
           "mc_set_lattice_temperature", "mc_set_tables", "mc_step", "poisson_update", "mc_tally", "mc_maps",
           "mc_history", "mc_observables", "mc_particles", "mc_read_particles", "mc_write_particles", "mc_read_fields",
           "mc_read_tables", "mc_get_config", "mc_get_lattice_temperature", "mc_set_launch", "mc_get_launch", "mc_get_ncell",
           "mc_get_instances", "mc_get_stream", "mc_occupancy", "mc_set_variant", "mc_use_graph", "mc_profile", "mc_profile_read",
           "mc_checkpoint", "mc_restore"]

_lib = None


def lib():
    """Load libgfmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1707_09073_amd/build.py (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, dp, u64p, u32p, i32p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64), \
            C.POINTER(C.c_uint32), C.POINTER(C.c_int32)
        L.mc_status_string.argtypes = [C.c_int]; L.mc_status_string.restype = C.c_char_p
        L.mc_last_error.argtypes = [vp]; L.mc_last_error.restype = C.c_char_p
        L.mc_workspace_bytes.argtypes = [C.POINTER(McConfig), C.c_int]; L.mc_workspace_bytes.restype = C.c_size_t
        L.mc_init.argtypes = [C.POINTER(vp), C.POINTER(McConfig), C.c_int, vp, C.c_size_t, vp]
        L.mc_destroy.argtypes = [vp]
        L.mc_set_lattice_temperature.argtypes = [vp, C.c_int, dp]
        L.mc_set_tables.argtypes = [vp, dp, dp]
        L.mc_step.argtypes = [vp, C.c_int]
        L.poisson_update.argtypes = [vp]
        L.mc_tally.argtypes = [vp, C.c_int, C.POINTER(McTallyOut), C.c_int]
        L.mc_maps.argtypes = [vp, C.c_int, u64p, u64p, dp, dp, dp]
        L.mc_observables.argtypes = [vp, C.c_int, C.POINTER(McObservablesOut)]
        L.mc_history.argtypes = [vp, C.c_int, dp, C.c_int, C.POINTER(C.c_int)]
        L.mc_particles.argtypes = [vp, C.c_int, C.POINTER(McParticlesView)]
        L.mc_read_particles.argtypes = [vp, C.c_int, dp, dp, i32p, i32p, u32p]
        L.mc_write_particles.argtypes = [vp, C.c_int, dp, dp, i32p, i32p, u32p]
        L.mc_read_fields.argtypes = [vp, C.c_int, dp, dp, u32p]
        L.mc_read_tables.argtypes = [vp, C.c_int, dp, dp, dp, dp]
        L.mc_get_config.argtypes = [vp, C.c_int, C.POINTER(McConfig)]
        L.mc_get_lattice_temperature.argtypes = [vp, C.c_int, dp]
        L.mc_set_launch.argtypes = [vp, C.c_int, C.c_int]
        L.mc_get_launch.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.mc_get_ncell.argtypes = [vp, C.POINTER(C.c_int)]
        L.mc_get_instances.argtypes = [vp, C.POINTER(C.c_int)]
        L.mc_get_stream.argtypes = [vp, C.POINTER(vp)]
        L.mc_occupancy.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.mc_use_graph.argtypes = [vp, C.c_int]
        L.mc_set_variant.argtypes = [vp, C.c_int]
        L.mc_profile.argtypes = [vp, C.c_int]
        L.mc_profile_read.argtypes = [vp, dp, C.POINTER(C.c_int), dp, C.POINTER(C.c_int), C.c_int]
        L.mc_checkpoint.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.mc_restore.argtypes = [vp, vp, C.c_size_t]
        for name in EXPORTS:
            if name not in ("mc_status_string", "mc_last_error", "mc_workspace_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class MCError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {lib().mc_status_string(code).decode()} ({code}) {detail}".strip())


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def make_config(cfg: dict) -> McConfig:
    """Marshal an input-recipe dictionary into the C struct."""
    m = cfg["material"]
    c = McConfig()
    c.mode = MC_DEVICE if cfg["mode"] == "device" else MC_BULK
    c.prec = MC_PREC_FP32_STATE if cfg.get("precision", "fp64") == "fp32" else MC_PREC_FP64
    for name in ("m_eff", "alpha", "E_c"):
        getattr(c.mat, name)[:] = [float(x) for x in m[name]]
    c.mat.Z[:] = [int(x) for x in m["Z"]]
    for name in ("eps_s", "eps_inf", "rho", "D_ac_eV", "D_iv_eVm", "hw_lo_eV", "hw_iv_eV", "u_ac"):
        setattr(c.mat, name, float(m[name]))
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


def mc_workspace_bytes(cfgs: list[dict]) -> int:
    arr = (McConfig * len(cfgs))(*[make_config(c) for c in cfgs])
    return int(lib().mc_workspace_bytes(arr, len(cfgs)))


class Ensemble:
    """A library context over one or more instances; owns its torch workspace."""

    def __init__(self, cfgs, device="cuda", stream=None):
        import torch
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        self.n = len(self.cfgs)
        self._carr = (McConfig * self.n)(*[make_config(c) for c in self.cfgs])
        nbytes = int(lib().mc_workspace_bytes(self._carr, self.n))
        if nbytes == 0:
            raise MCError(MC_E_ARG, "mc_workspace_bytes", "invalid configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        # a stream of our own (default priority): the legacy null stream cannot be graph-captured
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._ctx = C.c_void_p()
        rc = lib().mc_init(C.byref(self._ctx), self._carr, self.n, C.c_void_p(self.workspace.data_ptr()),
                           nbytes, C.c_void_p(self.stream.cuda_stream))
        if rc != MC_OK:
            detail = lib().mc_last_error(self._ctx).decode() if self._ctx.value else ""
            raise MCError(rc, "mc_init", detail)
        self.ncell = 1 if self.cfgs[0]["mode"] != "device" else int(np.prod(self.cfgs[0]["n_cells"]))
        self.nb = int(self.cfgs[0]["n_bins"])
        for i, c in enumerate(self.cfgs):
            if c.get("T_cells") is not None:
                self.mc_set_lattice_temperature(i, c["T_cells"])

    def _chk(self, rc, where):
        if rc != MC_OK:
            raise MCError(rc, where, lib().mc_last_error(self._ctx).decode())
        return rc

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().mc_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- the C ABI, same names ---
    def mc_set_lattice_temperature(self, inst, T):
        T = np.ascontiguousarray(T, dtype=np.float64)
        assert T.size == self.ncell
        self._chk(lib().mc_set_lattice_temperature(self._ctx, int(inst), _p(T, C.c_double)),
                  "mc_set_lattice_temperature")

    def mc_set_tables(self, shape, k4):
        s = np.ascontiguousarray(shape, dtype=np.float64)
        k = np.ascontiguousarray(k4, dtype=np.float64)
        assert s.size == 3 * self.nb * 10 and k.size == 3 * self.nb
        self._chk(lib().mc_set_tables(self._ctx, _p(s, C.c_double), _p(k, C.c_double)), "mc_set_tables")

    def mc_step(self, n_substeps: int):
        self._chk(lib().mc_step(self._ctx, int(n_substeps)), "mc_step")

    def poisson_update(self):
        self._chk(lib().poisson_update(self._ctx), "poisson_update")

    def mc_tally(self, inst: int = 0, reset_window: bool = False, check: bool = True) -> dict:
        t = McTallyOut()
        rc = lib().mc_tally(self._ctx, int(inst), C.byref(t), int(bool(reset_window)))
        if check:
            self._chk(rc, "mc_tally")
        return dict(intervals=t.intervals, intervals_total=t.intervals_total, t_window_fs=t.t_window_fs,
                    n_alive=t.n_alive, selections=t.selections, self_events=t.self_events, overflow=t.overflow,
                    real=np.array([[t.real[v][m] for m in range(10)] for v in range(3)], dtype=np.int64),
                    exits=np.array(list(t.exits), np.int64), injections=np.array(list(t.injections), np.int64),
                    segments=t.segments, reflect_guard=t.reflect_guard, weight=t.weight,
                    drain_current_A=t.drain_current_A, flags=t.flags, status=rc)

    def mc_maps(self, inst: int = 0):
        n = self.ncell
        heat4 = np.zeros((n, 4), np.uint64); dens = np.zeros(n, np.uint64)
        q = np.zeros(n); d = np.zeros(n); e = np.zeros(n)
        self._chk(lib().mc_maps(self._ctx, int(inst), _p(heat4, C.c_uint64), _p(dens, C.c_uint64),
                                _p(q, C.c_double), _p(d, C.c_double), _p(e, C.c_double)), "mc_maps")
        return dict(heat4=heat4, dens_sum=dens, heat_Wm3=q, density_m3=d, emit_Wm3=e)

    def mc_observables(self, inst: int = 0, check: bool = True) -> dict:
        o = McObservablesOut()
        rc = lib().mc_observables(self._ctx, int(inst), C.byref(o))
        if check:
            self._chk(rc, "mc_observables")
        return dict(intervals=o.intervals, t_window_fs=o.t_window_fs, drain_current_A=o.drain_current_A,
                    source_current_A=o.source_current_A, heat_W=o.heat_W, emit_W=o.emit_W,
                    drift_velocity_ms=np.array(o.drift_velocity_ms[:]), mean_energy_eV=o.mean_energy_eV,
                    valley_fraction=np.array(o.valley_fraction[:]),
                    half_mean=np.array(o.half_mean[:]).reshape(2, 2), half_se=np.array(o.half_se[:]).reshape(2, 2),
                    steady=o.steady, status=rc)

    def mc_history(self, inst: int = 0, max_rows: int = 8192) -> np.ndarray:
        rows = np.zeros((max_rows, 8)); n = C.c_int(0)
        self._chk(lib().mc_history(self._ctx, int(inst), _p(rows, C.c_double), int(max_rows), C.byref(n)),
                  "mc_history")
        return rows[:n.value].copy()

    def mc_particles(self, inst: int = 0) -> McParticlesView:
        v = McParticlesView()
        self._chk(lib().mc_particles(self._ctx, int(inst), C.byref(v)), "mc_particles")
        return v

    def mc_read_particles(self, inst: int = 0) -> dict:
        cap = int(self.cfgs[inst]["capacity"])
        k = np.zeros((cap, 3)); r = np.zeros((cap, 3))
        v = np.zeros(cap, np.int32); a = np.zeros(cap, np.int32); i = np.zeros(cap, np.uint32)
        self._chk(lib().mc_read_particles(self._ctx, int(inst), _p(k, C.c_double), _p(r, C.c_double),
                                          _p(v, C.c_int32), _p(a, C.c_int32), _p(i, C.c_uint32)),
                  "mc_read_particles")
        return dict(k=k, r=r, valley=v, alive=a, id=i)

    def mc_write_particles(self, inst, k, r, valley, alive, ident):
        k = np.ascontiguousarray(k, np.float64); r = np.ascontiguousarray(r, np.float64)
        v = np.ascontiguousarray(valley, np.int32); a = np.ascontiguousarray(alive, np.int32)
        i = np.ascontiguousarray(ident, np.uint32)
        self._chk(lib().mc_write_particles(self._ctx, int(inst), _p(k, C.c_double), _p(r, C.c_double),
                                           _p(v, C.c_int32), _p(a, C.c_int32), _p(i, C.c_uint32)),
                  "mc_write_particles")

    def mc_read_fields(self, inst: int = 0):
        n = self.ncell
        phi = np.zeros(n); F = np.zeros((n, 3)); cnt = np.zeros(n, np.uint32)
        self._chk(lib().mc_read_fields(self._ctx, int(inst), _p(phi, C.c_double), _p(F, C.c_double),
                                       _p(cnt, C.c_uint32)), "mc_read_fields")
        return phi, F, cnt

    def mc_read_tables(self, inst: int = 0):
        s = np.zeros((3, self.nb, 10)); k = np.zeros((3, self.nb)); f = np.zeros((self.ncell, 7)); g = np.zeros(3)
        self._chk(lib().mc_read_tables(self._ctx, int(inst), _p(s, C.c_double), _p(k, C.c_double),
                                       _p(f, C.c_double), _p(g, C.c_double)), "mc_read_tables")
        return s, k, f, g

    def mc_get_config(self, inst: int = 0) -> McConfig:
        c = McConfig()
        self._chk(lib().mc_get_config(self._ctx, int(inst), C.byref(c)), "mc_get_config")
        return c

    def mc_get_lattice_temperature(self, inst: int = 0) -> np.ndarray:
        T = np.zeros(self.ncell)
        self._chk(lib().mc_get_lattice_temperature(self._ctx, int(inst), _p(T, C.c_double)),
                  "mc_get_lattice_temperature")
        return T

    def mc_set_launch(self, block: int, tile: int):
        self._chk(lib().mc_set_launch(self._ctx, int(block), int(tile)), "mc_set_launch")

    def mc_get_launch(self):
        b, t, n = C.c_int(), C.c_int(), C.c_int()
        self._chk(lib().mc_get_launch(self._ctx, C.byref(b), C.byref(t), C.byref(n)), "mc_get_launch")
        return b.value, t.value, n.value

    def mc_get_ncell(self) -> int:
        n = C.c_int()
        self._chk(lib().mc_get_ncell(self._ctx, C.byref(n)), "mc_get_ncell")
        return n.value

    def mc_occupancy(self, block: int):
        """(resident workgroups per compute unit, compute units) of the particle kernel."""
        w, n = C.c_int(), C.c_int()
        self._chk(lib().mc_occupancy(self._ctx, int(block), C.byref(w), C.byref(n)), "mc_occupancy")
        return w.value, n.value

    def mc_set_variant(self, variant: int):
        """Particle kernel: 0 lane refill per tile, 1 one electron per lane,
        2 persistent (resident workgroups, each working every nw-th slot chunk
        of its instance), 3 persistent with each wavefront's next 128 slots
        staged in LDS."""
        self._chk(lib().mc_set_variant(self._ctx, int(variant)), "mc_set_variant")

    def mc_use_graph(self, enable: bool):
        self._chk(lib().mc_use_graph(self._ctx, int(bool(enable))), "mc_use_graph")

    def mc_profile(self, enable: bool):
        self._chk(lib().mc_profile(self._ctx, int(bool(enable))), "mc_profile")

    def mc_profile_read(self, reset: bool = True) -> dict:
        fm, rm = C.c_double(), C.c_double()
        nf, nr = C.c_int(), C.c_int()
        self._chk(lib().mc_profile_read(self._ctx, C.byref(fm), C.byref(nf), C.byref(rm), C.byref(nr),
                                        int(bool(reset))), "mc_profile_read")
        return dict(flight_ms=fm.value, n_flight=nf.value, refresh_ms=rm.value, n_refresh=nr.value)

    def mc_checkpoint(self) -> bytes:
        n = C.c_size_t(0)
        self._chk(lib().mc_checkpoint(self._ctx, None, C.byref(n)), "mc_checkpoint")
        buf = C.create_string_buffer(n.value)
        self._chk(lib().mc_checkpoint(self._ctx, buf, C.byref(n)), "mc_checkpoint")
        return buf.raw[:n.value]

    def mc_restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._chk(lib().mc_restore(self._ctx, buf, len(blob)), "mc_restore")


# ---------------------------------------------------------------------------
# MLP surrogate (sg_* entry points)
# ---------------------------------------------------------------------------
class SgConfig(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_out", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("ensemble", C.c_int32), ("max_batch", C.c_int32), ("seed", C.c_uint64),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("weight_decay", C.c_float)]


class SgQuery(C.Structure):
    _fields_ = [("h_x", C.c_void_p), ("h_box_lo", C.c_void_p), ("h_box_hi", C.c_void_p), ("calib", C.c_float),
                ("tol", C.c_float), ("warm_substeps", C.c_int32), ("window_substeps", C.c_int32)]


SG_EXPORTS = ["sg_workspace_bytes", "sg_init", "sg_destroy", "sg_last_error", "sg_layer_dims",
              "sg_set_normalization", "sg_forward", "sg_backward", "sg_adam", "sg_train_step", "sg_predict", "sg_predict_static",
              "sg_get_params", "sg_set_params", "sg_get_grads", "sg_predict_or_mc"]
EXPORTS = EXPORTS + SG_EXPORTS

_sg_ready = False


def _sg_lib():
    global _sg_ready
    L = lib()
    if not _sg_ready:
        vp, fp = C.c_void_p, C.POINTER(C.c_float)
        L.sg_workspace_bytes.argtypes = [C.POINTER(SgConfig)]; L.sg_workspace_bytes.restype = C.c_size_t
        L.sg_init.argtypes = [C.POINTER(vp), C.POINTER(SgConfig), vp, C.c_size_t, vp]
        L.sg_destroy.argtypes = [vp]
        L.sg_last_error.argtypes = [vp]; L.sg_last_error.restype = C.c_char_p
        L.sg_layer_dims.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.sg_set_normalization.argtypes = [vp, fp, fp, fp, fp]
        L.sg_forward.argtypes = [vp, C.c_int, vp, C.c_int, vp]
        L.sg_backward.argtypes = [vp, C.c_int, vp, vp, C.c_int, fp]
        L.sg_adam.argtypes = [vp, C.c_int, C.c_float]
        L.sg_train_step.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.c_float, fp]
        L.sg_predict.argtypes = [vp, vp, C.c_int, vp, vp]
        L.sg_predict_static.argtypes = [vp, vp, C.c_int, vp, vp]
        L.sg_get_params.argtypes = [vp, C.c_int, C.c_int, fp, fp]
        L.sg_set_params.argtypes = [vp, C.c_int, C.c_int, fp, fp]
        L.sg_get_grads.argtypes = [vp, C.c_int, C.c_int, fp, fp]
        L.sg_predict_or_mc.argtypes = [vp, vp, C.c_int, C.POINTER(SgQuery), C.POINTER(C.c_double), fp,
                                       C.POINTER(C.c_int)]
        for n in SG_EXPORTS:
            if n not in ("sg_workspace_bytes", "sg_last_error"):
                getattr(L, n).restype = C.c_int
        _sg_ready = True
    return L


class SurrogateNet:
    """A library surrogate context (ensemble of MLPs); owns its torch workspace.
    Inputs and outputs are torch FP32 CUDA tensors (row-major)."""

    def __init__(self, n_in, n_out, width=1024, depth=4, ensemble=4, max_batch=256, seed=1707_09073,
                 beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, device="cuda", stream=None):
        import torch
        L = _sg_lib()
        self.cfg = SgConfig(n_in, n_out, width, depth, ensemble, max_batch, seed, beta1, beta2, eps, weight_decay)
        nbytes = int(L.sg_workspace_bytes(C.byref(self.cfg)))
        if nbytes == 0:
            raise MCError(MC_E_ARG, "sg_workspace_bytes", "invalid surrogate configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._ctx = C.c_void_p()
        rc = L.sg_init(C.byref(self._ctx), C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()), nbytes,
                       C.c_void_p(self.stream.cuda_stream))
        if rc != MC_OK:
            raise MCError(rc, "sg_init")
        self.n_in, self.n_out, self.depth, self.ensemble, self.max_batch = n_in, n_out, depth, ensemble, max_batch

    def _chk(self, rc, where):
        if rc != MC_OK:
            raise MCError(rc, where, _sg_lib().sg_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _sg_lib().sg_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _in(self):
        """Order this context's stream after torch's current stream (inputs written by torch)."""
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _out(self):
        """Order torch's current stream after this context's stream (outputs read by torch)."""
        import torch
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    @staticmethod
    def _ptr(t, rows, cols):
        import torch
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() >= rows * cols
        return C.c_void_p(t.data_ptr())

    def sg_layer_dims(self, layer):
        K, N = C.c_int(), C.c_int()
        self._chk(_sg_lib().sg_layer_dims(self._ctx, int(layer), C.byref(K), C.byref(N)), "sg_layer_dims")
        return K.value, N.value

    def sg_set_normalization(self, x_mean, x_std, y_mean, y_std):
        a = [np.ascontiguousarray(v, np.float32) for v in (x_mean, x_std, y_mean, y_std)]
        self._norm = a
        self._chk(_sg_lib().sg_set_normalization(self._ctx, *[_p(v, C.c_float) for v in a]),
                  "sg_set_normalization")

    def sg_forward(self, member, x, out):
        b = x.shape[0]
        self._in()
        self._chk(_sg_lib().sg_forward(self._ctx, int(member), self._ptr(x, b, self.n_in), b,
                                       self._ptr(out, b, self.n_out)), "sg_forward")
        self._out()

    def sg_backward(self, member, x, y) -> float:
        b = x.shape[0]
        loss = C.c_float()
        self._in()
        self._chk(_sg_lib().sg_backward(self._ctx, int(member), self._ptr(x, b, self.n_in),
                                        self._ptr(y, b, self.n_out), b, C.byref(loss)), "sg_backward")
        self._out()
        return loss.value

    def sg_adam(self, member, lr):
        self._chk(_sg_lib().sg_adam(self._ctx, int(member), float(lr)), "sg_adam")

    def sg_train_step(self, member, x, y, lr, want_loss=True):
        b = x.shape[0]
        loss = C.c_float()
        self._in()
        self._chk(_sg_lib().sg_train_step(self._ctx, int(member), self._ptr(x, b, self.n_in),
                                          self._ptr(y, b, self.n_out), b, float(lr),
                                          C.byref(loss) if want_loss else None), "sg_train_step")
        # the caller's x and y may be freed (and their memory handed out
        # again on torch's stream) as soon as this returns
        self._out()
        return loss.value if want_loss else None

    def sg_predict_or_mc(self, x, calib: float, tol: float, ens=None, instance: int = 0, warm_substeps: int = 0,
                         window_substeps: int = 1, box=None):
        """One query (host FP32 features): the maps [2 ncell] (heat W/m^3, then
        density m^-3), the predicted relative error, and whether the Monte
        Carlo context `ens` (set up for the same bias point) answered."""
        x = np.ascontiguousarray(x, np.float32)
        assert x.size == self.n_in
        lo = hi = None
        if box is not None:
            lo = np.ascontiguousarray(box[0], np.float32)
            hi = np.ascontiguousarray(box[1], np.float32)
            assert lo.size == self.n_in and hi.size == self.n_in
        q = SgQuery(x.ctypes.data, None if lo is None else lo.ctypes.data, None if hi is None else hi.ctypes.data,
                    float(calib), float(tol), int(warm_substeps), int(window_substeps))
        maps = np.zeros(self.n_out - 2)
        perr, used = C.c_float(), C.c_int()
        self._in()
        self._chk(_sg_lib().sg_predict_or_mc(self._ctx, None if ens is None else ens._ctx, int(instance), C.byref(q),
                                             maps.ctypes.data_as(C.POINTER(C.c_double)), C.byref(perr),
                                             C.byref(used)), "sg_predict_or_mc")
        return maps, perr.value, bool(used.value)

    def sg_predict(self, x, mean_out, std_out=None):
        b = x.shape[0]
        self._in()
        self._chk(_sg_lib().sg_predict(self._ctx, self._ptr(x, b, self.n_in), b, self._ptr(mean_out, b, self.n_out),
                                       None if std_out is None else self._ptr(std_out, b, self.n_out)), "sg_predict")
        self._out()

    def sg_predict_static(self, x, mean_out, std_out=None):
        """sg_predict for batch <= 8 with the library's static scratch (no
        device allocation inside the call)."""
        b = x.shape[0]
        self._in()
        self._chk(_sg_lib().sg_predict_static(self._ctx, self._ptr(x, b, self.n_in), b,
                                              self._ptr(mean_out, b, self.n_out),
                                              None if std_out is None else self._ptr(std_out, b, self.n_out)),
                  "sg_predict_static")
        self._out()

    def sg_get_params(self, member, layer):
        K, N = self.sg_layer_dims(layer)
        W = np.zeros((K, N), np.float32); b = np.zeros(N, np.float32)
        self._chk(_sg_lib().sg_get_params(self._ctx, int(member), int(layer), _p(W, C.c_float), _p(b, C.c_float)),
                  "sg_get_params")
        return W, b

    def sg_set_params(self, member, layer, W, b):
        W = np.ascontiguousarray(W, np.float32); b = np.ascontiguousarray(b, np.float32)
        self._chk(_sg_lib().sg_set_params(self._ctx, int(member), int(layer), _p(W, C.c_float), _p(b, C.c_float)),
                  "sg_set_params")

    def sg_get_grads(self, member, layer):
        K, N = self.sg_layer_dims(layer)
        dW = np.zeros((K, N), np.float32); db = np.zeros(N, np.float32)
        self._chk(_sg_lib().sg_get_grads(self._ctx, int(member), int(layer), _p(dW, C.c_float), _p(db, C.c_float)),
                  "sg_get_grads")
        return dW, db


# ---------------------------------------------------------------------------
# Phonon side (ph_* entry points, include/gfph.h)
# ---------------------------------------------------------------------------
PH_OK, PH_E_ARG, PH_E_HIP = 0, -1, -2
PH_FACE = {"specular": 0, "diffuse": 1, "isothermal": 2}


class PhMaterial(C.Structure):
    _fields_ = [("q0", C.c_double), ("w_max", C.c_double), ("A", C.c_double), ("B1", C.c_double), ("B2", C.c_double)]


class PhElectrons(C.Structure):
    _fields_ = [("n_m3", C.c_double), ("m_dos", C.c_double), ("D_a_eV", C.c_double), ("rho", C.c_double),
                ("v_g", C.c_double)]


class PhMcConfig(C.Structure):
    _fields_ = [("L_nm", C.c_double * 3), ("n_cells", C.c_int32 * 3), ("face", C.c_int32 * 6), ("n_bins", C.c_int32),
                ("seed", C.c_uint64), ("instance", C.c_uint32), ("max_events", C.c_int32), ("n_packets", C.c_int64)]


PH_EXPORTS = ["ph_fermi_level", "ph_tables", "ph_interface", "ph_conductivity", "ph_mc_workspace_bytes", "ph_mc_run"]
EXPORTS = EXPORTS + PH_EXPORTS
_ph_ready = False


def _ph_lib():
    global _ph_ready
    L = lib()
    if not _ph_ready:
        vp, dp = C.c_void_p, C.c_void_p
        L.ph_fermi_level.argtypes = [C.c_double, C.c_double, C.c_double, dp, vp]
        L.ph_tables.argtypes = [C.POINTER(PhMaterial), C.POINTER(PhElectrons), C.c_double, C.c_int, dp, dp, vp]
        L.ph_interface.argtypes = [C.POINTER(PhMaterial), C.POINTER(PhMaterial), dp, C.c_int, dp, dp, vp]
        L.ph_conductivity.argtypes = [dp, C.c_int, C.c_double, dp, vp]
        L.ph_mc_workspace_bytes.argtypes = [C.POINTER(PhMcConfig)]
        L.ph_mc_workspace_bytes.restype = C.c_size_t
        L.ph_mc_run.argtypes = [C.POINTER(PhMcConfig), dp, dp, dp, dp, dp, C.POINTER(C.c_uint64), vp, C.c_size_t, vp]
        for n in ("ph_fermi_level", "ph_tables", "ph_interface", "ph_conductivity", "ph_mc_run"):
            getattr(L, n).restype = C.c_int
        _ph_ready = True
    return L


def _ph_chk(rc, where):
    if rc != PH_OK:
        raise MCError(rc, where, "phonon call failed")


def ph_material(m: dict) -> PhMaterial:
    return PhMaterial(float(m["q0"]), float(m["w_max"]), float(m["A"]), float(m["B1"]), float(m["B2"]))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def ph_fermi_level(n_m3: float, m_dos: float, T_K: float, stream=None):
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    _ph_chk(_ph_lib().ph_fermi_level(float(n_m3), float(m_dos), float(T_K), _dptr(out), _stream_ptr(stream)),
            "ph_fermi_level")
    return out


def ph_tables(material: dict, T_K: float, n_bins: int, electrons: dict | None = None, stream=None):
    """Bin tables [4, n_bins] (device FP64: omega, v_g, C_bin, 1/tau) and the
    Fermi level tensor (None without electrons)."""
    import torch
    tab = torch.empty((4, int(n_bins)), dtype=torch.float64, device="cuda")
    ef = None
    e = None
    if electrons:
        e = PhElectrons(float(electrons["n_m3"]), float(electrons["m_dos"]), float(electrons["D_a_eV"]),
                        float(electrons["rho"]), float(electrons["v_g"]))
        ef = torch.zeros(1, dtype=torch.float64, device="cuda")
    m = ph_material(material)
    _ph_chk(_ph_lib().ph_tables(C.byref(m), None if e is None else C.byref(e), float(T_K), int(n_bins), _dptr(tab),
                                _dptr(ef), _stream_ptr(stream)), "ph_tables")
    return tab, ef


def ph_interface(m1: dict, m2: dict, tables1, stream=None):
    """(tau_12 per bin of material 1, [1/R_K, bulk kappa of material 1]) as device tensors."""
    import torch
    nb = int(tables1.shape[1])
    tau = torch.empty(nb, dtype=torch.float64, device="cuda")
    sums = torch.empty(2, dtype=torch.float64, device="cuda")
    a, b = ph_material(m1), ph_material(m2)
    _ph_chk(_ph_lib().ph_interface(C.byref(a), C.byref(b), _dptr(tables1), nb, _dptr(tau), _dptr(sums),
                                   _stream_ptr(stream)), "ph_interface")
    return tau, sums


def ph_conductivity(tables, d_m: float, stream=None):
    """Conductivity (W/m/K, a device tensor of one element) from bin tables
    with the mean free paths limited by a structure size d_m (<= 0: bulk)."""
    import torch
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    _ph_chk(_ph_lib().ph_conductivity(_dptr(tables), int(tables.shape[1]), float(d_m), _dptr(out),
                                      _stream_ptr(stream)), "ph_conductivity")
    return out


class PhononMC:
    """Workspace and configuration of ph_mc_run."""

    def __init__(self, cfg: dict):
        import torch
        c = PhMcConfig()
        c.L_nm[:] = [float(x) for x in cfg["L_nm"]]
        c.n_cells[:] = [int(x) for x in cfg["n_cells"]]
        c.face[:] = [PH_FACE[f] for f in cfg["faces"]]
        c.n_bins = int(cfg["n_bins"])
        c.seed = int(cfg["seed"]) & 0xFFFFFFFFFFFFFFFF
        c.instance = int(cfg.get("instance", 0))
        c.max_events = int(cfg.get("max_events", 1 << 20))
        c.n_packets = int(cfg["n_packets"])
        self.cfg = c
        self.ncell = int(np.prod(cfg["n_cells"]))
        n = int(_ph_lib().ph_mc_workspace_bytes(C.byref(c)))
        if n == 0:
            raise MCError(PH_E_ARG, "ph_mc_workspace_bytes", "invalid configuration")
        self.workspace = torch.empty(n, dtype=torch.uint8, device="cuda")

    def ph_mc_run(self, tables, q_cell, stream=None, packet_scatterings: bool = False) -> dict:
        """Per-subcell packet time (fs) and temperature rise (K) as device
        tensors, and the event counts (synchronises); optionally each
        packet's scatterings."""
        import torch
        t = torch.empty(self.ncell, dtype=torch.float64, device="cuda")
        dT = torch.empty(self.ncell, dtype=torch.float64, device="cuda")
        q = q_cell.to(dtype=torch.float64, device="cuda").contiguous()
        pk = torch.zeros(int(self.cfg.n_packets), dtype=torch.int32, device="cuda") if packet_scatterings else None
        cnt = np.zeros(11, np.uint64)
        _ph_chk(_ph_lib().ph_mc_run(C.byref(self.cfg), _dptr(tables), _dptr(q), _dptr(t), _dptr(dT), _dptr(pk),
                                    cnt.ctypes.data_as(C.POINTER(C.c_uint64)), C.c_void_p(self.workspace.data_ptr()),
                                    self.workspace.numel(), _stream_ptr(stream)), "ph_mc_run")
        return dict(t_fs=t, dT=dT, scatterings=int(cnt[0]), wall_specular=int(cnt[1]), wall_diffuse=int(cnt[2]),
                    absorbed=cnt[3:9].astype(np.int64), dropped=int(cnt[9]), segments=int(cnt[10]),
                    packet_scatterings=None if pk is None else pk.cpu().numpy().view(np.uint32))


# --- Fourier's-law spreading (include/gffo.h) ---

class FoConfig(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dirichlet", C.c_int32 * 6), ("k_interface", C.c_int32),
                ("R_K_m2KW", C.c_double), ("T_sink_K", C.c_double), ("max_iterations", C.c_int32),
                ("rtol", C.c_double), ("warm_start", C.c_int32)]


FO_EXPORTS = ["fo_workspace_bytes", "fo_solve", "fo_chip_fields"]
EXPORTS = EXPORTS + FO_EXPORTS
_fo_ready = False


def _fo_lib():
    global _fo_ready
    L = lib()
    if not _fo_ready:
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.fo_workspace_bytes.argtypes = [C.POINTER(FoConfig)]
        L.fo_workspace_bytes.restype = C.c_size_t
        L.fo_solve.argtypes = [C.POINTER(FoConfig), vp, vp, vp, vp, C.POINTER(C.c_int), dp, vp, C.c_size_t, vp]
        L.fo_solve.restype = C.c_int
        L.fo_chip_fields.argtypes = [vp, dp, C.c_int, vp, vp, C.c_int, C.c_double, C.c_longlong, vp, vp, vp]
        L.fo_chip_fields.restype = C.c_int
        _fo_ready = True
    return L


def fo_config(cfg: dict) -> FoConfig:
    c = FoConfig()
    c.n[:] = [int(v) for v in cfg["n"]]
    c.dirichlet[:] = [int(v) for v in cfg["dirichlet"]]
    c.k_interface = int(cfg.get("k_interface", -1))
    c.R_K_m2KW = float(cfg.get("R_K_m2KW", 0.0))
    c.T_sink_K = float(cfg["T_sink_K"])
    c.max_iterations = int(cfg.get("max_iterations", 20000))
    c.rtol = float(cfg.get("rtol", 1e-12))
    c.warm_start = int(cfg.get("warm_start", 0))
    return c


def fo_solve(cfg: dict, edges, kappa, q, stream=None, check: bool = True, T0=None) -> dict:
    """Temperature per cell (device tensor, K) of a conduction problem; edges
    is the x, y, z edge coordinates (m) concatenated or a list of three.
    With T0 (per cell, K) the iteration starts from that temperature (a
    warm start) instead of T_sink."""
    import torch
    c = fo_config(cfg)
    if T0 is not None:
        c.warm_start = 1
    L = _fo_lib()
    n = int(L.fo_workspace_bytes(C.byref(c)))
    if n == 0:
        raise MCError(MC_E_ARG, "fo_workspace_bytes", "invalid configuration")
    if isinstance(edges, (list, tuple)):
        edges = np.concatenate([np.asarray(e, np.float64) for e in edges])
    e = torch.as_tensor(np.asarray(edges, np.float64) if not hasattr(edges, "data_ptr") else edges,
                        dtype=torch.float64).to("cuda").contiguous()
    k = torch.as_tensor(kappa, dtype=torch.float64).to("cuda").contiguous()
    qq = torch.as_tensor(q, dtype=torch.float64).to("cuda").contiguous()
    if T0 is not None:
        T = torch.as_tensor(T0, dtype=torch.float64).to("cuda").clone().contiguous()
        if T.numel() != k.numel():
            raise MCError(MC_E_ARG, "fo_solve", "T0 must have one value per cell")
    else:
        T = torch.empty_like(k)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    it, rel = C.c_int(0), C.c_double(0.0)
    st = _stream_ptr(stream)
    torch.cuda.current_stream().synchronize()
    rc = L.fo_solve(C.byref(c), _dptr(e), _dptr(k), _dptr(qq), _dptr(T), C.byref(it), C.byref(rel), _dptr(ws), n, st)
    if check and rc != MC_OK:
        raise MCError(rc, "fo_solve", f"after {it.value} iterations, relative residual {rel.value:.3e}")
    return dict(T=T, iterations=it.value, rel_residual=rel.value, status=rc)


def fo_chip_fields(material, kappa_by_material, src_index, src, scale: float = 1.0, stream=None):
    """Per-cell conductivity and heat of a chip problem (device tensors)."""
    import torch
    m = torch.as_tensor(material, dtype=torch.uint8).to("cuda").contiguous()
    si = torch.as_tensor(src_index, dtype=torch.int32).to("cuda").contiguous()
    sv = torch.as_tensor(src, dtype=torch.float64).to("cuda").contiguous()
    kt = np.ascontiguousarray(kappa_by_material, dtype=np.float64)
    nc = m.numel()
    kap = torch.empty(nc, dtype=torch.float64, device="cuda")
    q = torch.empty(nc, dtype=torch.float64, device="cuda")
    torch.cuda.current_stream().synchronize()
    rc = _fo_lib().fo_chip_fields(_dptr(m), _p(kt, C.c_double), int(kt.size), _dptr(si), _dptr(sv), int(sv.numel()),
                                  float(scale), nc, _dptr(kap), _dptr(q), _stream_ptr(stream))
    if rc != MC_OK:
        raise MCError(rc, "fo_chip_fields")
    return kap, q


# --- electro-thermal iteration (include/gfhy.h) ---

class HyConfig(C.Structure):
    _fields_ = [("mat", PhMaterial), ("elec", PhElectrons), ("n_bins", C.c_int32), ("face", C.c_int32 * 6),
                ("max_events", C.c_int32), ("n_packets", C.c_int64), ("seed", C.c_uint64), ("T_sink_K", C.c_double),
                ("T_lin_K", C.c_double), ("warmup_intervals", C.c_int32), ("window_intervals", C.c_int32),
                ("max_iterations", C.c_int32), ("relax", C.c_double), ("tol_K", C.c_double)]


class HyRecord(C.Structure):
    _fields_ = [("iteration", C.c_int32), ("instance", C.c_int32), ("source", C.c_int32), ("steady", C.c_int32),
                ("drain_current_A", C.c_double), ("heat_W", C.c_double), ("emit_W", C.c_double),
                ("T_lin_K", C.c_double), ("dT_max_K", C.c_double), ("dT_mean_K", C.c_double),
                ("hot_cell", C.c_int32), ("pad", C.c_int32), ("change_K", C.c_double), ("R_th_KW", C.c_double),
                ("packets_absorbed", C.c_uint64), ("packets_dropped", C.c_uint64),
                ("dT_junction_max_K", C.c_double), ("dT_fourier_max_K", C.c_double), ("R_th_device_KW", C.c_double),
                ("R_th_fourier_KW", C.c_double), ("fo_iterations", C.c_int32), ("pad2", C.c_int32)]


HY_EXPORTS = ["hy_workspace_bytes", "hy_run"]
EXPORTS = EXPORTS + HY_EXPORTS
_hy_ready = False


def _hy_lib():
    global _hy_ready
    L = lib()
    if not _hy_ready:
        vp = C.c_void_p
        L.hy_workspace_bytes.argtypes = [vp, C.POINTER(HyConfig), vp]
        L.hy_workspace_bytes.restype = C.c_size_t
        L.hy_run.argtypes = [vp, C.POINTER(HyConfig), vp, C.POINTER(C.c_double), vp, C.c_size_t, C.POINTER(HyRecord),
                             C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.hy_run.restype = C.c_int
        _hy_ready = True
    return L


def hy_config(h: dict) -> HyConfig:
    """hy_config from a dict: mat (Table II dict), electrons (dict or None),
    n_bins, faces (six names), max_events, n_packets, seed, T_sink_K,
    T_lin_K, warmup_intervals, window_intervals, max_iterations, relax, tol_K."""
    c = HyConfig()
    c.mat = ph_material(h["mat"])
    e = h.get("electrons")
    if e:
        c.elec = PhElectrons(float(e["n_m3"]), float(e["m_dos"]), float(e["D_a_eV"]), float(e["rho"]), float(e["v_g"]))
    c.n_bins = int(h["n_bins"])
    c.face[:] = [PH_FACE[f] for f in h["faces"]]
    c.max_events = int(h.get("max_events", 1 << 22))
    c.n_packets = int(h["n_packets"])
    c.seed = int(h["seed"]) & 0xFFFFFFFFFFFFFFFF
    c.T_sink_K = float(h["T_sink_K"])
    c.T_lin_K = float(h.get("T_lin_K", 0.0))
    c.warmup_intervals = int(h["warmup_intervals"])
    c.window_intervals = int(h["window_intervals"])
    c.max_iterations = int(h["max_iterations"])
    c.relax = float(h.get("relax", 1.0))
    c.tol_K = float(h.get("tol_K", 0.0))
    return c


class HyChip(C.Structure):
    _fields_ = [("fo", FoConfig), ("d_edges", C.c_void_p), ("d_material", C.c_void_p), ("d_src_index", C.c_void_p),
                ("d_base_index", C.c_void_p), ("kappa_by_material", C.c_double * 16), ("n_materials", C.c_int32),
                ("half_wires", C.c_int32)]


def hy_chip(chip: dict):
    """(HyChip, the device tensors it points to) from a dict: fo (an fo_solve
    configuration), edges, material, src_index, base_index (host arrays or
    tensors), kappa_by_material, half_wires."""
    import torch
    keep = dict(edges=torch.as_tensor(np.concatenate([np.asarray(e, np.float64) for e in chip["edges"]]),
                                      dtype=torch.float64).cuda(),
                material=torch.as_tensor(np.asarray(chip["material"], np.uint8)).cuda(),
                src=torch.as_tensor(np.asarray(chip["src_index"], np.int32)).cuda(),
                base=torch.as_tensor(np.asarray(chip["base_index"], np.int32)).cuda())
    c = HyChip()
    c.fo = fo_config(dict(chip["fo"], T_sink_K=chip["fo"].get("T_sink_K", 0.0)))
    c.d_edges, c.d_material = keep["edges"].data_ptr(), keep["material"].data_ptr()
    c.d_src_index, c.d_base_index = keep["src"].data_ptr(), keep["base"].data_ptr()
    kt = list(chip["kappa_by_material"])
    c.kappa_by_material[:len(kt)] = [float(v) for v in kt]
    c.n_materials = len(kt)
    c.half_wires = int(chip["half_wires"])
    torch.cuda.synchronize()
    return c, keep


def hy_workspace_bytes(ens: "Ensemble", h: dict, chip: dict | None = None) -> int:
    c = hy_config(h)
    ch = hy_chip(chip) if chip else None
    return int(_hy_lib().hy_workspace_bytes(ens._ctx, C.byref(c), None if ch is None else C.byref(ch[0])))


def hy_run(ens: "Ensemble", h: dict, heat0_Wm3=None, chip: dict | None = None) -> dict:
    """The coupled iteration on every instance of `ens` (device mode), with
    the Fourier stage when `chip` is given (see hy_chip).  Returns the
    records (list of dicts, one per instance and iteration), the iterations
    done and each instance's final lattice temperature."""
    import torch
    c = hy_config(h)
    L = _hy_lib()
    ch = hy_chip(chip) if chip else None
    chp = None if ch is None else C.byref(ch[0])
    n = int(L.hy_workspace_bytes(ens._ctx, C.byref(c), chp))
    if n == 0:
        raise MCError(MC_E_ARG, "hy_workspace_bytes", "invalid configuration for this context")
    ws = torch.empty(n, dtype=torch.uint8, device=ens.device)
    cap = ens.n * c.max_iterations
    recs = (HyRecord * cap)()
    nrec, nit = C.c_int(0), C.c_int(0)
    h0 = None
    if heat0_Wm3 is not None:
        h0 = np.ascontiguousarray(heat0_Wm3, dtype=np.float64).reshape(ens.n, ens.ncell)
    torch.cuda.synchronize()
    rc = L.hy_run(ens._ctx, C.byref(c), chp, None if h0 is None else _p(h0, C.c_double), C.c_void_p(ws.data_ptr()),
                  n, recs, cap, C.byref(nrec), C.byref(nit))
    out = [{k: getattr(recs[i], k) for k, _ in HyRecord._fields_ if k not in ("pad", "pad2")}
           for i in range(nrec.value)]
    ens._chk(rc, "hy_run")
    T = np.zeros((ens.n, ens.ncell))
    for i in range(ens.n):
        ens._chk(lib().mc_get_lattice_temperature(ens._ctx, i, _p(T[i], C.c_double)), "mc_get_lattice_temperature")
    return dict(records=out, iterations=nit.value, T_cells=T)
