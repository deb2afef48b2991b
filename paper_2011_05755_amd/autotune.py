"""Autotuner for the tile configuration of the correlation kernel.

A refset's tile configuration is (corr_variant, chunk_particles, run_tiles);
see ``mra_tuning`` in include/mra.h.  No configuration changes any result,
only speed, so the tuner may pick freely among the ones the library accepts.
The tile itself (8 particle rows by 8 references) is fixed by the matrix-core
block, whose 16 columns are the 8 references' two spectrum combinations, and
by the LDS state of its 64 pairs; what a workgroup covers is tunable through
run_tiles, the number of consecutive row tiles it takes (they share the
particle thresholds of the pruning bound, and fewer, longer runs trade
launch tail for pruning reach).

Key:        (L, number of rings, K bucket, T, precision), where the K bucket is
            the smallest power of two >= K (at least 8, one reference tile).
Candidates: every variant that ``mra_set_tuning`` accepts for the refset,
            crossed with a few chunk sizes (0 = as large as the workspace
            allows; small chunks keep the particle operand of a chunk within
            the last-level cache), with the library's own run length; then,
            at the winner, a few run lengths (0 = the library's choice).
Measure:    the median wall time of ``mra_align`` on a sample stack,
            synchronised, after one untimed call per candidate.
Cache:      a JSON file, ``$MRA_AUTOTUNE_CACHE`` or
            ``~/.cache/paper_2011_05755_amd/autotune.json``; entries hold the
            winner and every candidate's time.

    python -m paper_2011_05755_amd.autotune --L 76 --rings 35 --K 100 --T 3 --precision fp32
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import tempfile
import time
from typing import Callable, Iterable

DEFAULT_CHUNKS = (0, 128, 512, 2048)
DEFAULT_RUNS = (0, 1, 2, 4, 8, 16, 32, 48)
MAX_VARIANT = 4   # variant ids are probed from 0 up to this bound


def k_bucket(K: int) -> int:
    b = 8
    while b < K:
        b *= 2
    return b


def tuning_key(L: int, n_rings: int, K: int, T: int, precision: str) -> str:
    return f"L{L}-R{n_rings}-K{k_bucket(K)}-T{T}-{precision}"


def refset_key(ctx, refset_id: int) -> str:
    rs = ctx.refsets[refset_id]
    return tuning_key(rs.L, rs.n_rings, rs.K, rs.shift_max, rs.precision)


def default_cache_path() -> str:
    env = os.environ.get("MRA_AUTOTUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2011_05755_amd", "autotune.json")


class Cache:
    """Key -> {"corr_variant", "chunk_particles", "ms", "candidates"}."""

    def __init__(self, path: str | None = None):
        self.path = path or default_cache_path()
        self.entries: dict[str, dict] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                data = json.load(f)
            if not isinstance(data, dict):
                raise ValueError(f"{self.path}: not a tuning cache")
            self.entries = data

    def get(self, key: str) -> dict | None:
        return self.entries.get(key)

    def put(self, key: str, entry: dict):
        self.entries[key] = entry

    def save(self):
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune.")
        with os.fdopen(fd, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def candidates(ctx, refset_id: int, chunks: Iterable[int] = DEFAULT_CHUNKS) -> list[tuple[int, int]]:
    """(variant, chunk) pairs the library accepts for the refset.  Leaves the
    refset's tuning as it was."""
    from .mra import MRAError, MRA_E_INVAL
    before = ctx.get_tuning(refset_id)
    variants = []
    for v in range(MAX_VARIANT + 1):
        try:
            ctx.set_tuning(refset_id, corr_variant=v)
        except MRAError as e:
            if e.code != MRA_E_INVAL:
                raise
            continue
        variants.append(v)
    ctx.set_tuning(refset_id, *before)
    return [(v, c) for v in variants for c in chunks]


def wall_ms(ctx, refset_id: int, parts, reps: int) -> float:
    """Median synchronised wall time of mra_align over `reps` calls."""
    import torch

    from .mra import AlignResult
    out = AlignResult.empty(parts.shape[0], parts.device)
    ctx.align(refset_id, parts, out=out)            # untimed: workspace growth, caches
    torch.cuda.synchronize(parts.device)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.align(refset_id, parts, out=out)
        torch.cuda.synchronize(parts.device)
        times.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(times)


def tune(ctx, refset_id: int, parts, reps: int = 3, cache: Cache | None = None,
         chunks: Iterable[int] = DEFAULT_CHUNKS, runs: Iterable[int] = DEFAULT_RUNS,
         timer: Callable[[object, int, object, int], float] = wall_ms, log=None) -> dict:
    """Time every candidate on `parts`, apply the fastest to the refset and
    record it in `cache` (if given; the caller saves).  Returns the entry."""
    key = refset_key(ctx, refset_id)
    n = parts.shape[0]
    cand = [(v, c) for v, c in candidates(ctx, refset_id, chunks) if c == 0 or c < n]
    times = {}
    for v, c in cand:
        ctx.set_tuning(refset_id, corr_variant=v, chunk_particles=c)
        times[(v, c)] = timer(ctx, refset_id, parts, reps)
        if log:
            log(f"{key}: variant {v} chunk {c}: {times[(v, c)]:.3f} ms")
    (bv, bc) = min(times, key=lambda vc: (times[vc], vc))
    # the run length at the winner (run_tiles 0, the library's choice, is the
    # time already taken)
    run_times = {0: times[(bv, bc)]}
    for r in runs:
        if r in run_times:
            continue
        ctx.set_tuning(refset_id, corr_variant=bv, chunk_particles=bc, run_tiles=r)
        run_times[r] = timer(ctx, refset_id, parts, reps)
        if log:
            log(f"{key}: variant {bv} chunk {bc} run {r}: {run_times[r]:.3f} ms")
    br = min(run_times, key=lambda r: (run_times[r], r))
    ctx.set_tuning(refset_id, corr_variant=bv, chunk_particles=bc, run_tiles=br)
    entry = dict(corr_variant=bv, chunk_particles=bc, run_tiles=br, ms=run_times[br], n_sample=n,
                 candidates={f"{v}/{c}": round(t, 4) for (v, c), t in sorted(times.items())},
                 runs={str(r): round(t, 4) for r, t in sorted(run_times.items())})
    if cache is not None:
        cache.put(key, entry)
    return entry


def apply(ctx, refset_id: int, cache: Cache) -> bool:
    """Set the refset's tuning from the cache; False if its key is absent."""
    e = cache.get(refset_key(ctx, refset_id))
    if e is None:
        return False
    ctx.set_tuning(refset_id, corr_variant=int(e["corr_variant"]), chunk_particles=int(e["chunk_particles"]),
                   run_tiles=int(e.get("run_tiles", 0)))
    return True


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", type=int, required=True)
    ap.add_argument("--rings", type=int, required=True, help="rings 1..rings")
    ap.add_argument("--K", type=int, required=True)
    ap.add_argument("--T", type=int, required=True)
    ap.add_argument("--precision", default="fp32", choices=("fp32", "bf16", "fp16"))
    ap.add_argument("--sample", type=int, default=4096, help="particles in the timed stack")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args(argv)

    import torch
    from . import mra, synth
    dev = torch.device("cuda", 0)
    blobs = synth.make_blobs(args.K, args.L, seed=(7, 0), rho_max=min(args.rings, args.L / 2 - 4))
    refs = synth.render_refs(blobs).to(dev)
    parts, _ = synth.make_particles(blobs, args.sample, args.T, 0.05, seed=(7, 1), device=dev)
    ctx = mra.Context(0)
    ctx.load_refs(0, refs, r_min=1, r_max=args.rings, shift_max=args.T, precision=args.precision)
    cache = Cache(args.cache)
    entry = tune(ctx, 0, parts, reps=args.reps, cache=cache, log=lambda m: print(m, flush=True))
    cache.save()
    print(json.dumps({refset_key(ctx, 0): entry}), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
