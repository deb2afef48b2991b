"""Autotuner host logic on the CPU, with a stand-in for the library context
(the candidate set comes from what set_tuning accepts; times are given)."""

import json

import pytest

from paper_2011_05755_amd import autotune, mra


class FakeRefset:
    def __init__(self, L, r_max, K, T, precision):
        self.L, self.n_rings, self.K, self.shift_max, self.precision = L, r_max, K, T, precision


class FakeCtx:
    """Accepts variants {0, 2} and chunks >= 0, like an FP32 refset with R4 > 12."""

    def __init__(self):
        self.refsets = {3: FakeRefset(96, 46, 37, 2, "fp32")}
        self.tuning = {3: (2, 0)}
        self.run = {3: 0}

    def set_tuning(self, rid, corr_variant=-1, chunk_particles=0, run_tiles=0):
        v = 2 if corr_variant < 0 else corr_variant
        if v not in (0, 2) or chunk_particles < 0 or not 0 <= run_tiles <= 64:
            raise mra.MRAError(mra.MRA_E_INVAL, "variant cannot serve this geometry")
        self.tuning[rid] = (v, chunk_particles)
        self.run[rid] = run_tiles

    def get_tuning(self, rid):
        return self.tuning[rid]


class Parts:
    shape = (1000, 96, 96)


def test_k_bucket_and_key():
    assert [autotune.k_bucket(k) for k in (1, 8, 9, 100, 128, 129, 400)] == [8, 8, 16, 128, 128, 256, 512]
    assert autotune.tuning_key(76, 35, 100, 3, "bf16") == "L76-R35-K128-T3-bf16"


def test_candidates_are_what_the_library_accepts_and_tuning_is_restored():
    ctx = FakeCtx()
    ctx.set_tuning(3, corr_variant=0, chunk_particles=7)
    cand = autotune.candidates(ctx, 3, chunks=(0, 64))
    assert cand == [(0, 0), (0, 64), (2, 0), (2, 64)]
    assert ctx.get_tuning(3) == (0, 7)


def test_tune_picks_the_fastest_applies_it_and_caches(tmp_path):
    ctx = FakeCtx()
    cost = {(0, 0): 5.0, (0, 128): 4.0, (0, 512): 4.5, (2, 0): 3.0, (2, 128): 3.5, (2, 512): 3.0}
    seen = []

    run_cost = {1: 3.2, 2: 2.5, 4: 2.5, 8: 2.9, 16: 3.0, 32: 3.1, 48: 3.3}  # run 0 (the library's choice) costs cost[...]

    def timer(c, rid, parts, reps):
        r = c.run[rid]
        if r:
            assert c.get_tuning(rid) == (2, 0)     # run lengths are timed at the winner
            return run_cost[r]
        seen.append(c.get_tuning(rid))
        return cost[c.get_tuning(rid)]

    cache = autotune.Cache(str(tmp_path / "t.json"))
    e = autotune.tune(ctx, 3, Parts(), cache=cache, chunks=(0, 128, 512, 2048), timer=timer)
    assert sorted(seen) == sorted(cost)            # chunk 2048 >= sample size is skipped
    assert (e["corr_variant"], e["chunk_particles"]) == (2, 0)   # tie broken towards the smaller config
    assert e["run_tiles"] == 2 and e["ms"] == 2.5                # tie broken towards the shorter run
    assert ctx.get_tuning(3) == (2, 0) and ctx.run[3] == 2
    cache.save()
    data = json.loads((tmp_path / "t.json").read_text())
    assert data["L96-R46-K64-T2-fp32"]["candidates"]["0/128"] == 4.0

    assert data["L96-R46-K64-T2-fp32"]["runs"] == {"0": 3.0, "1": 3.2, "2": 2.5, "4": 2.5, "8": 2.9, "16": 3.0,
                                                   "32": 3.1, "48": 3.3}

    ctx2 = FakeCtx()
    ctx2.set_tuning(3, corr_variant=0)
    assert autotune.apply(ctx2, 3, autotune.Cache(str(tmp_path / "t.json")))
    assert ctx2.get_tuning(3) == (2, 0) and ctx2.run[3] == 2
    ctx2.refsets[3].K = 500
    assert not autotune.apply(ctx2, 3, autotune.Cache(str(tmp_path / "t.json")))


def test_cache_rejects_a_file_that_is_not_a_mapping(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("[1, 2]")
    with pytest.raises(ValueError):
        autotune.Cache(str(p))
