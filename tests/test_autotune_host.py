"""Host logic of the launch-shape autotuner, on a stand-in context (no GPU):
candidate sets per precision, round-filling tile sizes, choice of the fastest
trial and restoration of the simulation state."""
import pytest

from paper_1707_09073_amd import autotune as A


class FakeEnsemble:
    """Times each (block, tile, variant) by a table; records every call."""

    def __init__(self, precision, capacity=13_000_000, per_cu=None, times=None):
        self.cfgs = [dict(mode="device", precision=precision, capacity=capacity, substeps=10)]
        self.per_cu = per_cu or {256: 4, 384: 3, 512: 2, 1024: 1}
        self.times = times or {}
        self.shape = (256, 8192, 0)
        self.state = 0            # advanced by mc_step, restored by mc_restore
        self.calls = []
        self._t = 0.0
        self._n = 0

    def mc_occupancy(self, block):
        return self.per_cu.get(block, 0), 256

    def mc_checkpoint(self):
        return self.state

    def mc_restore(self, blob):
        self.state = blob

    def mc_set_launch(self, block, tile):
        if block > 512 and self.cfgs[0]["precision"] != "fp32":
            raise RuntimeError("1024-lane workgroups need FP32 state")
        if tile % block or tile > 65535 or tile < 1024:
            raise RuntimeError("unsupported launch shape")
        self.shape = (block, tile, self.shape[2])
        self.calls.append(("launch", block, tile))

    def mc_set_variant(self, v):
        self.shape = (self.shape[0], self.shape[1], v)

    def mc_profile(self, on):
        pass

    def mc_step(self, n):
        self.state += n
        self._t += self.times.get(self.shape, 1.0) * (n // 10)
        self._n += n // 10

    def mc_profile_read(self, reset=True):
        r = dict(flight_ms=self._t, refresh_ms=0.0, n_flight=self._n, n_refresh=self._n)
        if reset:
            self._t, self._n = 0.0, 0
        return r


def test_round_candidates_fill_whole_rounds():
    e = FakeEnsemble("fp32")
    for block, tile, variant in A.round_candidates(e, blocks=(256, 512, 1024)):
        assert variant == 0 and tile % block == 0 and tile <= 65535
        resident = e.per_cu[block] * 256
        n_tiles = -(-13_000_000 // tile)
        r = -(-n_tiles // resident)          # rounds of resident workgroups
        # the last round is full up to the rounding of the tile to the block
        assert r <= 8 and n_tiles >= r * resident * (tile - block - 1) / tile


def test_fp64_contexts_never_try_1024_lane_workgroups():
    A._cache.clear()
    e = FakeEnsemble("fp64")
    r = A.autotune(e, trials=1)
    assert all(t["block"] <= 512 for t in r["trials"])


def test_fp32_contexts_try_1024_lane_workgroups_and_keep_the_fastest():
    A._cache.clear()
    fast = (1024, 20480, 0)
    e = FakeEnsemble("fp32", times={fast: 0.5, (1024, 8192, 2): 0.7})
    before = e.state
    r = A.autotune(e, trials=2)
    assert (r["block"], r["tile"], r["variant"]) == fast
    assert e.shape == fast
    assert e.state == before, "tuning must leave the simulation where it was"
    assert any(t["block"] == 1024 and t["variant"] == 2 for t in r["trials"])
    # cached: a second call applies the choice without new trials
    e.shape = (256, 4096, 0)
    r2 = A.autotune(e)
    assert r2["cached"] and e.shape == fast


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_unsupported_shapes_are_skipped_not_fatal(precision):
    A._cache.clear()
    e = FakeEnsemble(precision, capacity=50_000)
    r = A.autotune(e, trials=1)
    assert r["trials"], "some shape must be usable"
    assert all(t["tile"] % t["block"] == 0 for t in r["trials"])


class NoisyEnsemble(FakeEnsemble):
    """Per shape, a list of ms-per-interval figures, one taken per timing
    (the last figure repeats)."""

    def __init__(self, precision, seq):
        super().__init__(precision)
        self.seq = {k: list(v) for k, v in seq.items()}
        self.timings = {}

    def mc_step(self, n):
        s = self.seq.get(self.shape)
        if s is not None:
            i = self.timings.get(self.shape, 0)
            self.timings[self.shape] = i + 1
            self.times[self.shape] = s[min(i, len(s) - 1)]
        super().mc_step(n)


def test_refinement_takes_the_median_not_one_lucky_timing():
    A._cache.clear()
    lucky = (1024, 8192, 2)        # fast once, slow on the re-timings
    steady = (1024, 8192, 3)
    e = NoisyEnsemble("fp32", {lucky: [0.40, 0.60, 0.62], steady: [0.45, 0.46, 0.44]})
    before = e.state
    r = A.autotune(e, candidates=[lucky, steady, (512, 4096, 0)], trials=2, refine=2)
    assert (r["block"], r["tile"], r["variant"]) == steady
    # five timings: 0.45, 0.46, 0.44, 0.44, 0.44
    assert r["refined_ms_per_interval"] == pytest.approx(0.44)
    assert e.timings[lucky] == 5 and e.timings[steady] == 5
    # the third candidate (1.0 ms) is outside the top two: timed once only
    assert e.state == before and e.shape == steady


def test_refinement_resolves_a_small_steady_difference():
    A._cache.clear()
    a, b = (1024, 4096, 3), (1024, 8192, 3)
    # b is luckier on the first, short timing; a is 1% faster on most re-timings
    e = NoisyEnsemble("fp32", {a: [0.580, 0.574, 0.585, 0.573, 0.575], b: [0.575, 0.581, 0.579, 0.586, 0.580]})
    r = A.autotune(e, candidates=[a, b], trials=2, refine=2)
    assert (r["block"], r["tile"], r["variant"]) == a


def test_refinement_off_keeps_the_first_timing():
    A._cache.clear()
    lucky, steady = (1024, 8192, 2), (1024, 8192, 3)
    e = NoisyEnsemble("fp32", {lucky: [0.40, 0.60, 0.62], steady: [0.45, 0.46, 0.44]})
    r = A.autotune(e, candidates=[lucky, steady], trials=2, refine=1)
    assert (r["block"], r["tile"], r["variant"]) == lucky
    assert e.timings[lucky] == 1 and e.timings[steady] == 1
