"""Launch-shape autotuner for the particle kernel.

Times each candidate (workgroup size, tile size, kernel variant) on the
context's live state for a few flight intervals with HIP events, restoring a
checkpoint before every trial and at the end.  Results of the Monte Carlo do
not depend on the shape, so tuning leaves the simulation exactly where it
was.  Choices are cached per (mode, precision, instances, total slots).
"""
from __future__ import annotations

import json
import os

# (workgroup size, tile size, kernel variant).  Tile sizes step finely
# because the last round of resident workgroups is partly idle: the best
# tile is one whose tile count is just under a multiple of the resident count.
# The persistent variants (2, and 3 with staged slots) have no rounds: their
# grid is the resident count (one 1024-lane workgroup per compute unit, or
# two of 512), and their tile size only sets the contact refill's free-slot
# blocks.
DEFAULT_CANDIDATES = [
    (256, 1536, 0), (256, 2048, 0), (256, 2560, 0), (256, 3072, 0), (256, 4096, 0),
    (256, 5120, 0), (256, 6144, 0), (256, 8192, 0),
    (512, 2048, 0), (512, 2560, 0), (512, 3072, 0), (512, 4096, 0), (512, 8192, 0), (384, 3072, 0), (384, 6144, 0),
    (128, 2048, 0), (256, 4096, 1),
    (1024, 4096, 2), (1024, 8192, 2), (512, 4096, 2),
    (1024, 4096, 3), (1024, 8192, 3), (512, 4096, 3),
]
# FP32 state only: 1024-lane workgroups (16 wavefronts sharing one refill
# queue; FP64 state needs more registers than they leave each lane)
FP32_CANDIDATES = [(1024, 10240, 0), (1024, 13312, 0), (1024, 20480, 0)]

_cache: dict = {}


def round_candidates(ens, blocks=(256, 384, 512), max_rounds=8) -> list:
    """Tile sizes whose tile count just fills r whole rounds of resident
    workgroups (r = 1..max_rounds): with workgroups of similar length, a last
    round that is partly empty leaves compute units idle."""
    total = sum(int(c["capacity"]) for c in ens.cfgs)
    out = []
    for b in blocks:
        try:
            per_cu, n_cu = ens.mc_occupancy(b)
        except Exception:
            continue
        resident = per_cu * n_cu
        if resident <= 0:
            continue
        for r in range(1, max_rounds + 1):
            tile = -(-total // (r * resident))
            tile = -(-tile // b) * b
            if tile <= 65535:
                out.append((b, tile, 0))
    return out


def _key(ens) -> str:
    c = ens.cfgs[0]
    cap = sum(int(x["capacity"]) for x in ens.cfgs)
    return f"{c['mode']}/{c.get('precision', 'fp64')}/{len(ens.cfgs)}/{cap}"


def _time_candidate(ens, blob, block, tile, variant, intervals, K):
    """ms per interval of one shape over `intervals` flight intervals from
    the checkpoint `blob` (None if the shape is refused)."""
    ens.mc_restore(blob)
    try:
        ens.mc_set_launch(block, tile)
    except Exception:
        return None
    ens.mc_set_variant(variant)
    ens.mc_profile(True)
    ens.mc_profile_read(reset=True)
    ens.mc_step(intervals * K)
    p = ens.mc_profile_read(reset=True)
    ens.mc_profile(False)
    return (p["flight_ms"] + p["refresh_ms"]) / max(1, p["n_flight"]), p["flight_ms"] / max(1, p["n_flight"])


def autotune(ens, candidates=None, trials: int = 5, cache_file: str | None = None, log=None,
             refine: int = 4, retimes: int = 4) -> dict:
    """Pick the fastest launch shape for `ens` (a gfmc.Ensemble) and apply it.
    Every candidate is timed once over `trials` intervals; the `refine`
    fastest are timed `retimes` times more over twice as many intervals, and
    the lowest median of their timings wins (a single short timing can be
    off by several percent, and the staged variant's two tile sizes differ
    by about 1%)."""
    key = _key(ens)
    if cache_file and os.path.exists(cache_file) and not _cache:
        try:
            _cache.update(json.load(open(cache_file)))
        except (OSError, ValueError):
            pass
    if key in _cache:
        best = _cache[key]
        ens.mc_set_launch(best["block"], best["tile"])
        ens.mc_set_variant(best["variant"])
        return dict(best, cached=True)
    K = int(ens.cfgs[0]["substeps"])
    if candidates is None:
        fp32 = ens.cfgs[0].get("precision", "fp64") == "fp32"
        blocks = (256, 384, 512, 1024) if fp32 else (256, 384, 512)
        candidates = DEFAULT_CANDIDATES + (FP32_CANDIDATES if fp32 else [])
        candidates = list(dict.fromkeys(candidates + round_candidates(ens, blocks=blocks)))
        if not fp32:
            candidates = [c for c in candidates if c[0] <= 512]
    blob = ens.mc_checkpoint()
    results = []
    for block, tile, variant in candidates:
        t = _time_candidate(ens, blob, block, tile, variant, trials, K)
        if t is None:
            continue
        ms, fl = t
        results.append(dict(block=block, tile=tile, variant=variant, ms_per_interval=ms, flight_ms=fl))
        if log:
            log(f"  autotune block {block} tile {tile} variant {variant}: {ms:.3f} ms/interval")
    top = sorted(results, key=lambda r: r["ms_per_interval"])[:max(1, refine)]
    if refine > 1:
        for r in top:
            times = [r["ms_per_interval"]]
            for _ in range(retimes):
                t = _time_candidate(ens, blob, r["block"], r["tile"], r["variant"], 2 * trials, K)
                if t is not None:
                    times.append(t[0])
            r["refined_ms_per_interval"] = sorted(times)[len(times) // 2]
            if log:
                log(f"  autotune refine block {r['block']} tile {r['tile']} variant {r['variant']}: "
                    f"{', '.join(f'{x:.3f}' for x in times)} ms/interval")
        best = min(top, key=lambda r: r["refined_ms_per_interval"])
    else:
        best = top[0]
    ens.mc_restore(blob)
    ens.mc_set_launch(best["block"], best["tile"])
    ens.mc_set_variant(best["variant"])
    _cache[key] = best
    if cache_file:
        try:
            json.dump(_cache, open(cache_file, "w"))
        except OSError:
            pass
    return dict(best, cached=False, trials=results)
