"""Benchmark of the electron Monte Carlo hot path on one MI355X.

Workload: the half-nanowire FinFET device (60 x 120 nm cross-section, 1 um
channel, 3x6x100 subcells) with 10 million superparticles, FP32 particle
state with FP64 tallies and Poisson, 1e18 cm^-3 doping, Vgs = 0, Vds = 5 V,
lattice temperature 300 K plus a +150 K Gaussian hot spot at the drain end.
One step = one flight interval: 10 sub-steps of 1 fs of free flight and
scattering for every electron, then the subcell deposit, the contact refill
and the Poisson refresh.  The default run times 500 steps (5 ps).

Prints one JSON line.  The metric counts free-flight segments as a
sub-step-at-a-time Monte Carlo would fly them (one per electron per 1 fs
sub-step plus one per scattering selection, real or self) per second.  The
kernel fuses the ten sub-steps of an interval and draws each electron's
flight afresh only at the interval start, so the flights it actually flies
(one per electron per interval plus one per selection) are reported beside
the metric as flights_per_s, with real scattering events/s and
electron-fs/s.  The roofline is the algorithmic HBM stream of the particle
kernel: each live electron's state read and written once per interval.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "electron scatter+flight events/s per MI355X; surrogate vs MC heat-map time @2% err"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic FP64 operations of the phonon packet kernel, counted from the
# method's arithmetic (a division, square root, logarithm, sine or cosine
# counts as one): per straight flight piece, the distance to the subcell
# boundary along each axis (3 x 3), the time in the subcell and its signed
# tally (3), the move (6) and the remaining free path (1); per scattering,
# four uniforms (8), the bin draw (1), the isotropic direction (10) and the
# free path (4); per diffuse reflection, two uniforms and the cosine-law
# direction (13); per packet, its emission (38).
PH_FLOPS = {"segment": 19, "scattering": 23, "diffuse": 13, "packet": 38}
# VALU issue peak in lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz (one non-packed FP32 or integer operation per lane and cycle; the
# build disables packed FP32 math)
ALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# Per-segment figures of each particle-kernel variant from its rocprofv3
# counter passes (the profile named), valid for the kernel sources whose
# digest is given: VALU lane-instructions issued per free-flight segment
# (SQ_INSTS_VALU x 64 / segments) and HBM bytes per segment (FETCH_SIZE x
# 2.000 + WRITE_SIZE x 1.000, scales from a 1 GiB device copy).
KERNELS = {0: "k_flight_refill<float,true>", 1: "k_flight<float,true>", 2: "k_flight_persist<float,true>",
           3: "k_flight_persist_staged<float,true>"}
KERNEL_COUNTERS = {
    0: {"sources_digest": "35e64eb5d2ea9021", "valu_lane_ops_per_segment": 183.9, "hbm_bytes_per_segment": 11.48,
        "active_lane_fraction": 0.534, "profile": "profiles/k_flight_refill_device1e7_counters.md",
        "note": "counters at block 1024 / tile 8192 over intervals 6-10 (9.9e6 electrons, state beyond the "
                "Infinity Cache, non-temporal state loads); the active lanes include lanes without an electron, "
                "which run the segment on stale state and drop it, so the useful fraction is an upper bound"},
    2: {"sources_digest": "35e64eb5d2ea9021", "valu_lane_ops_per_segment": 157.7, "hbm_bytes_per_segment": 8.80,
        "active_lane_fraction": 0.458, "profile": "profiles/k_flight_persist_device1e7_counters.md",
        "note": "counters at block 1024 / tile 8192 over intervals 6-10 (9.9e6 electrons, state beyond the "
                "Infinity Cache, non-temporal state loads); one resident workgroup of 1024 lanes per CU, chunks of "
                "128 slots"},
    3: {"sources_digest": "35e64eb5d2ea9021", "valu_lane_ops_per_segment": 168.2, "hbm_bytes_per_segment": 6.62,
        "active_lane_fraction": 0.431, "profile": "profiles/k_flight_persist_staged_device1e7_counters.md",
        "note": "counters at block 1024 / tile 8192 over intervals 6-10 (9.9e6 electrons, state beyond the "
                "Infinity Cache); slots staged in LDS a piece of 128 ahead, one resident workgroup per CU, chunks "
                "of 128 slots"},
}


# The phonon packet kernel's counters (profiles/k_ph_packets_wire_trace.md),
# valid for the phonon.hip whose digest is given: VALU lane-instructions per
# flight segment and the share of active lanes.
PH_COUNTERS = {"sources_digest": "823147b268c32621", "valu_lane_ops_per_segment": 793.0, "active_lane_fraction": 0.354,
               "profile": "profiles/k_ph_packets_wire_trace.md"}


def _ph_issue(segs_launch: float, avg_ms: float):
    """VALU issue of the packet kernel from its counters (None once
    phonon.hip differs from the sources they were taken on): the kernel is
    bound by divergent VALU issue, not by its algorithmic operations."""
    if _kernel_digest(("phonon.hip",)) != PH_COUNTERS["sources_digest"]:
        return None
    ops = PH_COUNTERS["valu_lane_ops_per_segment"] * segs_launch
    rate = ops / (avg_ms * 1e-3)
    return dict(lane_instructions_per_launch=ops, achieved=rate / 1e12, peak=ALU_PEAK_LANE_OPS / 1e12,
                unit="T lane-instr/s", frac_issue=rate / ALU_PEAK_LANE_OPS,
                active_lane_fraction=PH_COUNTERS["active_lane_fraction"],
                frac_useful=rate * PH_COUNTERS["active_lane_fraction"] / ALU_PEAK_LANE_OPS,
                profile=PH_COUNTERS["profile"])


def _kernel_digest(files=("gfmc_kernels.h", "gfmc_device.h", "gfmc.hip")) -> str:
    """Digest of kernel sources (by default the particle kernels, the device
    arithmetic they use and the host code that sets their launch, chunks
    included; the refresh kernels live in a header of their own) with
    comments and blank lines removed, so that a comment edit does not
    invalidate the counters."""
    import hashlib
    import re
    h = []
    for f in files:
        with open(os.path.join(ROOT, "paper_1707_09073_amd", "csrc", f)) as fh:
            code = [re.sub(r"//.*$", "", line).rstrip() for line in fh]
        h.append(hashlib.sha256("\n".join(l for l in code if l.strip()).encode()).hexdigest())
    return hashlib.sha256("".join(h).encode()).hexdigest()[:16]


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n_intervals: int = 40) -> dict:
    """The FP64 CPU reference on the same workload, timed on the host cores
    for its first flight intervals after initialisation (about 10 s of work
    on 16 cores)."""
    from oracle import emc_oracle
    from paper_1707_09073_amd import workloads as W
    emc_oracle.build()
    cfg = W.large_device_config()
    cfg["precision"] = "fp64"
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    o = emc_oracle.Oracle(cfg)
    t_init = time.perf_counter() - t0
    o.reset_window()
    import numpy as np
    alive0 = int(np.count_nonzero(o.particles()["alive"]))
    t0 = time.perf_counter()
    o.run(n_intervals, threads)
    dt = time.perf_counter() - t0
    c = o.counts()
    # alive electrons x sub-steps + selections, as for the GPU (the live count
    # taken as the mean of its values before and after the sample)
    alive1 = int(np.count_nonzero(o.particles()["alive"]))
    segs = 0.5 * (alive0 + alive1) * cfg["substeps"] * n_intervals + c["selections"]
    return dict(value=segs / dt, unit="events/s", cores=threads, kind="oracle",
                sample=(f"same 1e7-superparticle device workload in FP64, first {n_intervals} flight intervals "
                        f"({n_intervals * cfg['substeps']} fs) after initialisation; {dt:.1f} s timed, "
                        f"init {t_init:.1f} s untimed; segments counted as on the GPU (alive x sub-steps "
                        f"with the live count averaged over the sample)"))


MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense BF16 MFMA, MI355X


def surrogate_mlp(args) -> dict:
    """The surrogate's dense layers at a large batch: one member of the
    1803 -> 1024 x 4 -> 3600 MLP (BF16 MFMA, FP32 accumulation), the forward
    pass and the training step (forward, backward, Adam) timed with HIP events
    on the surrogate's stream."""
    import numpy as np
    import torch
    from paper_1707_09073_amd import gfmc
    from paper_1707_09073_amd.surrogate import N_CELL, N_ENC
    N_IN = 3 + N_CELL
    B = args.sg_batch
    net = gfmc.SurrogateNet(N_IN, N_ENC, width=1024, depth=4, ensemble=1, max_batch=B)
    g = torch.Generator(device="cuda:0").manual_seed(7)
    x = torch.randn(B, N_IN, device="cuda:0", generator=g)
    y = torch.randn(B, N_ENC, device="cuda:0", generator=g)
    net.sg_set_normalization(np.zeros(N_IN), np.ones(N_IN), np.zeros(N_ENC), np.ones(N_ENC))
    out = torch.empty(B, N_ENC, device="cuda:0")
    dims = [net.sg_layer_dims(l) for l in range(5)]
    dims[0] = (N_IN, dims[0][1])  # algorithmic flops: the unpadded input width
    flops_fwd = 2.0 * B * sum(k * n for k, n in dims)
    # backward: dX and dW per layer (dX skipped for the first layer)
    flops_bwd = 2.0 * B * (2 * sum(k * n for k, n in dims) - dims[0][0] * dims[0][1])
    res = {}
    for name, fn, flops in (("forward", lambda: net.sg_forward(0, x, out), flops_fwd),
                            ("train_step", lambda: net.sg_train_step(0, x, y, 1e-4, want_loss=False),
                             flops_fwd + flops_bwd)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
        for _ in range(args.steps):
            fn()
        e1.record(net.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[name] = dict(ms=ms, tflops=flops / (ms * 1e-3) / 1e12)
    net.close()
    return dict(batch=B, dims=dims, flops_forward=flops_fwd, flops_backward=flops_bwd, **res)


def sweep64(args) -> dict:
    """Batched bias sweep: 64 device instances (uneven ensembles of 20k-500k
    electrons, FP32 state) in one context, one launch per kernel per interval
    replayed from a hipGraph, against the same 64 bias points run one after
    another as separate contexts."""
    import torch
    from paper_1707_09073_amd import gfmc, workloads as W
    cfgs = W.bias_sweep(64)
    K = cfgs[0]["substeps"]
    n_tot = sum(c["n_particles"] for c in cfgs)
    _log(f"sweep: 64 instances, {n_tot} electrons in total")
    ens = gfmc.Ensemble(cfgs, device="cuda:0")
    ens.mc_step(10 * K)
    if args.block and args.tile:
        ens.mc_set_launch(args.block, args.tile)
    elif not args.no_autotune:
        from paper_1707_09073_amd.autotune import autotune
        autotune(ens, log=_log)
    block, tile, n_tiles = ens.mc_get_launch()
    # per-kernel split from a few profiled intervals (eager launches)
    ens.mc_profile(True)
    ens.mc_profile_read(reset=True)
    ens.mc_step(10 * K)
    prof = ens.mc_profile_read(reset=True)
    ens.mc_profile(False)
    ens.mc_use_graph(True)
    ens.mc_step(args.warmup * K)
    for i in range(64):
        ens.mc_tally(i, reset_window=(i == 63))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.mc_step(args.steps * K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    segs = sum(ens.mc_tally(i)["segments"] for i in range(64))
    ens.close()
    del ens
    torch.cuda.synchronize()
    # the same bias points as 64 separate contexts, run back to back
    sep_steps = max(1, args.steps // 4)
    sep_wall, sep_segs = 0.0, 0
    for i, c in enumerate(cfgs):
        e = gfmc.Ensemble(c, device="cuda:0")
        e.mc_step(10 * K)
        e.mc_use_graph(True)
        e.mc_step(2 * K)
        e.mc_tally(reset_window=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.mc_step(sep_steps * K)
        torch.cuda.synchronize()
        sep_wall += time.perf_counter() - t0
        sep_segs += e.mc_tally()["segments"]
        e.close()
    return dict(value=segs / wall, ms_per_step=wall / args.steps * 1e3, n_tot=n_tot, block=block, tile=tile,
                n_tiles=n_tiles, separate_value=sep_segs / sep_wall, separate_steps=sep_steps,
                flight_ms=prof["flight_ms"] / max(1, prof["n_flight"]),
                refresh_ms=prof["refresh_ms"] / max(1, prof["n_refresh"]))


def phonon_packets(args) -> dict:
    """The phonon packet kernel alone on the half-wire domain: GaN tables at
    300 K with Eq. (1) (1024 bins), the synthetic net heat map of an electron
    window (1 mW around the drain-side gate edge), `--packets` packets per
    launch.  Per-launch device time from HIP events on the launch stream."""
    import torch
    from paper_1707_09073_amd import gfmc, workloads as W
    dev = W.device_config(n_particles=1000)
    tab, _ = gfmc.ph_tables(W.GAN_PHONONS, 300.0, 1024, W.WIRE_ELECTRONS)
    L, nc = dev["L_nm"], dev["n_cells"]
    vc_m3 = (L[0] / nc[0]) * (L[1] / nc[1]) * (L[2] / nc[2]) * 1e-27
    q = torch.tensor(W.wire_heat_map(dev) * vc_m3, dtype=torch.float64, device="cuda")   # W per subcell
    n = int(args.packets)
    mc = gfmc.PhononMC(dict(L_nm=dev["L_nm"], n_cells=dev["n_cells"], faces=W.WIRE_FACES, n_bins=1024,
                            seed=W.BASE_SEED + 11, instance=0, max_events=1 << 22, n_packets=n))
    st = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        mc.ph_mc_run(tab, q, stream=st)
    torch.cuda.synchronize()
    tot = dict(segments=0, scatterings=0, wall_diffuse=0, wall_specular=0, dropped=0)
    ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        r = mc.ph_mc_run(tab, q, stream=st)
        b.record(st)
        b.synchronize()
        ms += a.elapsed_time(b)
        for k in tot:
            tot[k] += r[k]
    wall = time.perf_counter() - t0
    dT = r["dT"].cpu().numpy()
    return dict(n=n, wall=wall, avg_ms=ms / args.steps, dT_max=float(dT.max()), **tot)


FO_BYTES_PER_CELL_ITERATION = 136   # SpMV 48 (diag, p, three conductances read, Ap written), update 56, direction 32


def fourier_chip(args) -> dict:
    """The Fourier's-law solve over the 31-wire half chip (1.03e6 cells):
    conductivities from the bins at 300 K, the interface resistance of
    Eq. (3), a 1 mW synthetic heat map per half-wire on every wire."""
    import numpy as np
    import torch
    from paper_1707_09073_amd import gfmc, workloads as W
    dev = W.device_config(n_particles=1000)
    geom = W.chip_geometry(dev)
    tg, _ = gfmc.ph_tables(W.GAN_PHONONS, 300.0, 2048)
    ts, _ = gfmc.ph_tables(W.SIC_PHONONS, 300.0, 2048)
    kt = [0.0, float(gfmc.ph_conductivity(ts, 0.0).cpu()[0]), float(gfmc.ph_conductivity(tg, 2e-6).cpu()[0]),
          float(gfmc.ph_conductivity(tg, 120e-9).cpu()[0])]
    _, sums = gfmc.ph_interface(W.GAN_PHONONS, W.SIC_PHONONS, tg)
    L, nc = dev["L_nm"], dev["n_cells"]
    vc = (L[0] / nc[0]) * (L[1] / nc[1]) * (L[2] / nc[2]) * 1e-27
    kap, q = gfmc.fo_chip_fields(geom["material"], kt, geom["src_index"], W.wire_heat_map(dev, power_W=1e-3) * vc)
    cfg = dict(n=geom["n"], dirichlet=[0, 0, 0, 0, 1, 0], k_interface=geom["k_interface"],
               R_K_m2KW=1.0 / float(sums.cpu()[0]), T_sink_K=300.0, rtol=1e-10, max_iterations=100000)
    for _ in range(max(1, args.warmup)):
        gfmc.fo_solve(cfg, geom["edges"], kap, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for _ in range(args.steps):
        r = gfmc.fo_solve(cfg, geom["edges"], kap, q)
        its += r["iterations"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T = r["T"].cpu().numpy()
    return dict(cells=int(np.prod(geom["n"])), wall=wall, iterations=its, dT_max=float(T.max()) - 300.0)


def hybrid_sweep(args) -> dict:
    """The electro-thermal iteration as a batched drain-voltage sweep: five
    device instances (Vds = 2, 4, 6, 8, 10 V, Vgs = 0, 2e6 electrons each,
    FP32 state) in one context from 300 K; per iteration 50 settling and 150
    window intervals, then 2^21 phonon packets per instance in the half-wire
    domain; three iterations.  Reports the thermal resistance against Vds."""
    import torch
    from paper_1707_09073_amd import gfmc, workloads as W
    vds = [2.0, 4.0, 6.0, 8.0, 10.0]
    per = max(10_000, args.particles // len(vds))
    cfgs = []
    for i, v in enumerate(vds):
        c = W.device_config(n_particles=per, precision="fp32", Vds=v, Vgs=0.0, seed=W.BASE_SEED + 40 + i)
        c["instance"] = i
        cfgs.append(c)
    hy = dict(mat=W.GAN_PHONONS, electrons=W.WIRE_ELECTRONS, n_bins=1024,
              faces=W.WIRE_FACES, n_packets=1 << 21, seed=W.BASE_SEED + 12, T_sink_K=300.0, T_lin_K=0.0,
              warmup_intervals=50, window_intervals=150, max_iterations=3, relax=1.0, tol_K=0.0)
    chip = None
    if args.chip:
        # the 31-wire half chip: conductivities from the bins at T_sink (the
        # wire and film with their mean free paths limited by 120 nm and
        # 2 um), 1/R_K of Eq. (3) from GaN's side; the wire's contact ends
        # adiabatic, its foot on the film
        geom = W.chip_geometry(cfgs[0])
        tg, _ = gfmc.ph_tables(W.GAN_PHONONS, 300.0, 2048)
        ts, _ = gfmc.ph_tables(W.SIC_PHONONS, 300.0, 2048)
        kt = [0.0, float(gfmc.ph_conductivity(ts, 0.0).cpu()[0]), float(gfmc.ph_conductivity(tg, 2e-6).cpu()[0]),
              float(gfmc.ph_conductivity(tg, 120e-9).cpu()[0])]
        _, sums = gfmc.ph_interface(W.GAN_PHONONS, W.SIC_PHONONS, tg)
        chip = dict(fo=dict(n=geom["n"], dirichlet=[0, 0, 0, 0, 1, 0], k_interface=geom["k_interface"],
                            R_K_m2KW=1.0 / float(sums.cpu()[0]), rtol=1e-10, max_iterations=100000),
                    edges=geom["edges"], material=geom["material"], src_index=geom["src_index"],
                    base_index=geom["base_index"], kappa_by_material=kt, half_wires=2 * geom["half_wires"])
        hy["faces"] = W.WIRE_FACES_ON_CHIP
    ens = gfmc.Ensemble(cfgs, device="cuda:0")
    ens.mc_use_graph(True)
    ens.mc_step(10 * cfgs[0]["substeps"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = gfmc.hy_run(ens, hy, chip=chip)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    last = [x for x in r["records"] if x["iteration"] == r["iterations"] - 1]
    out = dict(wall=wall, iterations=r["iterations"], electrons=per * len(vds), vds=vds,
               R_th_KW=[x["R_th_KW"] for x in last], dT_max_K=[x["dT_max_K"] for x in last],
               emit_W=[x["emit_W"] for x in last], drain_current_A=[x["drain_current_A"] for x in last],
               hot_x_nm=[(x["hot_cell"] // 18 + 0.5) * 10.0 for x in last], records=r["records"])
    if chip:
        out.update(R_th_device_KW=[x["R_th_device_KW"] for x in last],
                   R_th_fourier_KW=[x["R_th_fourier_KW"] for x in last],
                   dT_junction_max_K=[x["dT_junction_max_K"] for x in last],
                   dT_fourier_max_K=[x["dT_fourier_max_K"] for x in last],
                   fo_iterations=[x["fo_iterations"] for x in last])
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed flight intervals (10 fs each)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--particles", type=int, default=10_000_000)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32",
                    help="particle state precision (tallies and the Poisson solve are FP64 either way)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--graph", action="store_true", help="replay intervals from a hipGraph (no per-kernel timing)")
    ap.add_argument("--variant", type=int, default=0,
                    help="particle kernel: 0 lane refill per tile, 1 one electron per lane, 2 persistent, "
                         "3 persistent with staged slots")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default (or given) launch shape")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sg-batch", type=int, default=4096, help="batch of the surrogate workload")
    ap.add_argument("--workload", choices=["device1e7", "sweep64", "surrogate", "phonon", "hybrid", "fourier"],
                    default="device1e7",
                    help="device1e7: one 10M-electron device (the headline); sweep64: 64-instance batched sweep; "
                         "phonon: the phonon packet kernel; hybrid: the electro-thermal iteration over five drain "
                         "voltages; fourier: the chip-scale conduction solve")
    ap.add_argument("--packets", type=int, default=1 << 23, help="packets per launch of the phonon workload")
    ap.add_argument("--chip", action="store_true",
                    help="hybrid workload: add the Fourier's-law stage over the 31-wire chip")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the hot path here is the per-GPU share and is not sharded "
              "(see the design notes for how it would shard).", file=sys.stderr)
        return 2

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 5}))
        return 0
    from paper_1707_09073_amd import gfmc, workloads as W
    if not os.path.exists(gfmc.LIB_PATH):
        from paper_1707_09073_amd import build as B
        B.build(force=True)
    torch.cuda.set_device(0)
    if args.workload == "surrogate":
        r = surrogate_mlp(args)
        fw = r["forward"]
        print(json.dumps({
            "metric": "surrogate MLP throughput (BF16 MFMA, FP32 accumulation)", "value": fw["tflops"],
            "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": fw["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "surrogate MLP 1803 -> 1024 x 4 -> 3600, one member, forward at batch "
                                   f"{r['batch']}", "batch": r["batch"]},
            "train_step": r["train_step"],
            "roofline": {"bound": "mfma", "achieved": fw["tflops"], "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": fw["tflops"] / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                         "flops_per_forward": r["flops_forward"]}}), flush=True)
        return 0
    if args.workload == "phonon":
        r = phonon_packets(args)
        segs_launch = r["segments"] / args.steps
        flops = (PH_FLOPS["segment"] * r["segments"] + PH_FLOPS["scattering"] * r["scatterings"] +
                 PH_FLOPS["diffuse"] * r["wall_diffuse"] + PH_FLOPS["packet"] * r["n"] * args.steps) / args.steps
        achieved = flops / (r["avg_ms"] * 1e-3) / 1e12
        print(json.dumps({
            "metric": "phonon packet flight segments/s", "value": r["segments"] / (r["avg_ms"] * 1e-3 * args.steps),
            "unit": "segments/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["avg_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "phonon packets in the half-wire domain (1000 x 60 x 120 nm, 100 x 3 x 6 "
                                   "subcells, contacts and film isothermal, symmetry cut specular, sidewall and top "
                                   "diffuse), GaN tables at 300 K with Eq. (1), 1024 bins, 1 mW synthetic heat map",
                       "packets": r["n"]},
            "segments_per_launch": segs_launch, "scatterings_per_launch": r["scatterings"] / args.steps,
            "diffuse_per_launch": r["wall_diffuse"] / args.steps, "dropped": r["dropped"], "dT_max_K": r["dT_max"],
            "packets_per_s": r["n"] / (r["avg_ms"] * 1e-3),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "k_ph_packets",
                         "algorithmic_flops_per_launch": flops, "flops_per_unit": PH_FLOPS,
                         "avg_launch_ms": r["avg_ms"],
                         "note": "launch time includes the one-thread set-up and the temperature kernels; "
                                 "divisions and transcendentals count one operation each",
                         "valu_issue": _ph_issue(segs_launch, r["avg_ms"])}}), flush=True)
        return 0
    if args.workload == "fourier":
        r = fourier_chip(args)
        ci = r["cells"] * r["iterations"]
        achieved = ci * FO_BYTES_PER_CELL_ITERATION / r["wall"] / 1e9
        print(json.dumps({
            "metric": "chip conduction: conjugate-gradient cell-iterations/s", "value": ci / r["wall"],
            "unit": "cell-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["wall"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Fourier's-law solve of the 31-wire GaN-on-SiC half chip (146 x 201 x 35 cells), "
                                   "size-limited conductivities, Eq. (3) interface resistance, 1 mW per half-wire",
                       "cells": r["cells"]},
            "iterations_per_solve": r["iterations"] / args.steps, "dT_max_K": r["dT_max"],
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "bytes_per_cell_iteration": FO_BYTES_PER_CELL_ITERATION,
                         "note": "whole solves timed on the host clock (three launches per iteration and a host "
                                 "check every 25 iterations included)"}}), flush=True)
        return 0
    if args.workload == "hybrid":
        r = hybrid_sweep(args)
        print(json.dumps({
            "metric": "electro-thermal iterations/s (electron windows + phonon packets, five drain voltages)",
            "value": r["iterations"] / r["wall"], "unit": "iterations/s", "n_gpus": 1, "steps": r["iterations"],
            "warmup": 10, "ms_per_step": r["wall"] / r["iterations"] * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "hybrid iteration: 5 half-nanowire instances (Vds 2-10 V, Vgs 0, 1e18 cm^-3) "
                                   "in one context, 50 + 150 intervals and 2^21 phonon packets per instance and "
                                   "iteration, 3 iterations from 300 K" +
                                   (", with the Fourier stage over the 31-wire half chip" if args.chip else ""),
                       "electrons": r["electrons"]},
            "vds_V": r["vds"], "R_th_KW": r["R_th_KW"], "dT_max_K": r["dT_max_K"], "emit_W": r["emit_W"],
            "drain_current_A": r["drain_current_A"], "hot_x_nm": r["hot_x_nm"],
            **({k: r[k] for k in ("R_th_device_KW", "R_th_fourier_KW", "dT_junction_max_K", "dT_fourier_max_K",
                                  "fo_iterations")} if args.chip else {})}), flush=True)
        return 0
    if args.workload == "sweep64":
        r = sweep64(args)
        print(json.dumps({
            "metric": METRIC, "value": r["value"], "unit": "events/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batched bias sweep: 64 half-nanowire device instances, Vgs U[-3,0] V, "
                                   "Vds U[1,10] V, doping log-uniform 1e17-1e19 cm^-3, 20k-500k electrons each, "
                                   "one hipGraph replay per interval", "electrons": r["n_tot"],
                       "block": r["block"], "tile": r["tile"], "tiles": r["n_tiles"]},
            "separate_contexts_events_per_s": r["separate_value"], "separate_steps": r["separate_steps"],
            "batched_over_separate": r["value"] / r["separate_value"],
            "flight_avg_ms": r["flight_ms"], "refresh_avg_ms": r["refresh_ms"]}), flush=True)
        return 0
    cfg = W.large_device_config(n_particles=args.particles)
    cfg["precision"] = args.precision
    f32 = args.precision == "fp32"
    K = cfg["substeps"]
    _log(f"init: {args.particles} superparticles, capacity {cfg['capacity']}")
    ens = gfmc.Ensemble(cfg, device="cuda:0")
    ens.mc_set_variant(args.variant)
    if args.block and args.tile:
        ens.mc_set_launch(args.block, args.tile)
    _log(f"warmup {args.warmup} intervals")
    ens.mc_step(args.warmup * K)
    if not (args.block and args.tile) and not args.no_autotune:
        # tuned on the state the timed window starts from (the live
        # population and its layout in the slots change over the first
        # picoseconds); every trial restarts from a checkpoint of it
        from paper_1707_09073_amd.autotune import autotune
        _log("autotuning launch shape")
        tuned = autotune(ens, log=_log)
        args.variant = tuned["variant"]
    block, tile, n_tiles = ens.mc_get_launch()
    ens.mc_use_graph(args.graph)
    _log(f"launch: block {block}, tile {tile}, {n_tiles} tiles, variant {args.variant}")
    ens.mc_tally(reset_window=True)
    ens.mc_profile(not args.graph)
    torch.cuda.synchronize()
    _log(f"timing {args.steps} intervals")
    t0 = time.perf_counter()
    ens.mc_step(args.steps * K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tal = ens.mc_tally()
    prof = ens.mc_profile_read() if not args.graph else None
    segments = tal["segments"]
    real = int(tal["real"].sum())
    proc = (segments - tal["selections"]) // K           # electrons processed per interval, summed
    value = segments / wall
    _log(f"wall {wall:.3f} s, segments {segments}, selections {tal['selections']}, real {real}")

    roofline = None
    if prof and prof["n_flight"]:
        # the particle kernel (one launch per interval), timed by HIP events on
        # the library's stream.  Algorithmic bytes: the fused interval must read
        # and write each live electron's state once per launch (six coordinates
        # and the meta word: 28 B each way in FP32 state, 52 B in FP64)
        flight_s = prof["flight_ms"] / prof["n_flight"] * 1e-3
        per_launch = proc / prof["n_flight"]
        state_b = (28 if f32 else 52) * 2
        achieved = per_launch * state_b / flight_s / 1e9
        kc = KERNEL_COUNTERS.get(args.variant) if f32 else None
        fresh = bool(kc) and _kernel_digest() == kc["sources_digest"]
        segs_launch = segments / prof["n_flight"]
        roofline = dict(
            bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
            traffic=kc["hbm_bytes_per_segment"] * segs_launch if fresh else None,
            kernel=KERNELS[args.variant] if f32 else KERNELS[args.variant].replace("<float", "<double"),
            algorithmic_bytes_per_launch=per_launch * state_b, bytes_per_electron_interval=state_b,
            electrons_per_launch=per_launch, avg_launch_ms=flight_s * 1e3,
            refresh_avg_ms=prof["refresh_ms"] / max(1, prof["n_refresh"]),
            flight_share=prof["flight_ms"] / (prof["flight_ms"] + prof["refresh_ms"]),
            counters_current=fresh,
            note="the ten sub-steps of an interval run in registers, so the state crosses HBM once per "
                 "interval; the kernel is bound by memory latency while the state in use outgrows the "
                 "Infinity Cache and by VALU issue once it fits, not by HBM bandwidth")
        if fresh:
            ops = kc["valu_lane_ops_per_segment"] * segs_launch
            roofline["valu_issue"] = dict(
                lane_instructions_per_launch=ops, achieved=ops / flight_s / 1e12, peak=ALU_PEAK_LANE_OPS / 1e12,
                unit="T lane-instr/s", frac_issue=ops / flight_s / ALU_PEAK_LANE_OPS,
                active_lane_fraction=kc.get("active_lane_fraction"),
                frac_useful=(ops * kc["active_lane_fraction"] / flight_s / ALU_PEAK_LANE_OPS
                             if kc.get("active_lane_fraction") else None),
                profile=kc["profile"], note=kc.get("note"))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": "half-nanowire GaN FinFET device MC, 10M superparticles, 3x6x100 subcells, "
                               "Vgs=0 V, Vds=5 V, 1e18 cm^-3, 300 K + 150 K drain hot spot, 1 fs x 10 per step",
                   "particles": args.particles, "substeps_per_step": K, "block": block, "tile": tile,
                   "graph": bool(args.graph), "variant": args.variant, "precision": args.precision},
        "flights_per_s": (proc + tal["selections"]) / wall,
        "real_events_per_s": real / wall,
        "electron_fs_per_s": proc * cfg["dt_fs"] * K / wall,
        "drain_current_A": tal["drain_current_A"],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
