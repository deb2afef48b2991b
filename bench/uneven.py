"""Uneven stacks in one batched call, with autotuned tile configurations.

64 stacks drawn from the uneven-stack size distribution (box L in
{64, 76, 96, 128}, N uniform 2k..50k, K uniform 20..400, shifts +-2..+-5,
rings 1..L/2-2), each against its own resident refset.  For each precision:

1. every distinct tuning key is tuned on a sample of its first stack (or
   taken from the cache) and applied to the refsets with that key;
2. the whole batch is aligned in one ``mra_align_batch`` call (timed);
3. every stack is aligned by its own ``mra_align`` call (timed), and the two
   results are compared bit for bit.

Prints one JSON line per precision.

    python -m bench.uneven --precisions bf16,fp32
"""

from __future__ import annotations

import argparse
import json
import sys
import time


def log(msg):
    print(f"[uneven] {msg}", file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--stacks", type=int, default=64)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--precisions", default="bf16,fp32")
    ap.add_argument("--n-scale", type=float, default=1.0, help="scale of the stack sizes")
    ap.add_argument("--tune-sample", type=int, default=384)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cache", default=None, help="autotune cache (JSON)")
    ap.add_argument("--no-singles", action="store_true")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from paper_2011_05755_amd import autotune, mra, synth
    dev = torch.device("cuda", 0)
    specs = synth.uneven_stack_specs(args.stacks, seed=args.seed)
    t0 = time.perf_counter()
    data = []
    for i, sp in enumerate(specs):
        N = max(1, int(round(sp["N"] * args.n_scale)))
        blobs = synth.make_blobs(sp["K"], sp["L"], seed=sp["seed"], rho_max=sp["rho_max"])
        refs = synth.render_refs(blobs).to(dev)
        parts, _ = synth.make_particles(blobs, N, sp["shift_max"], sp["snr"], seed=(sp["seed"], 1), device=dev)
        data.append((sp, refs, parts))
        if (i + 1) % 16 == 0:
            log(f"generated {i + 1} stacks")
    torch.cuda.synchronize()
    n_total = sum(p.shape[0] for _, _, p in data)
    log(f"{len(data)} stacks, {n_total} particles generated in {time.perf_counter() - t0:.1f} s")

    ctx = mra.Context(0)
    cache = autotune.Cache(args.cache)
    for form in [f for f in args.precisions.split(",") if f]:
        base = {"fp32": 0, "bf16": 1000, "fp16": 2000}[form]
        for i, (sp, refs, parts) in enumerate(data):
            ctx.load_refs(base + i, refs, r_min=sp["r_min"], r_max=sp["r_max"], shift_max=sp["shift_max"],
                          precision=form)
        # 1. tuning, one key at a time
        tuned = {}
        t0 = time.perf_counter()
        if not args.no_tune:
            for i, (sp, refs, parts) in enumerate(data):
                key = autotune.refset_key(ctx, base + i)
                if key not in tuned:
                    e = cache.get(key)
                    if e is None:
                        e = autotune.tune(ctx, base + i, parts[:args.tune_sample], reps=2, cache=cache,
                                          chunks=(0, 128), log=log)
                    tuned[key] = e
                autotune.apply(ctx, base + i, cache)
            cache.save()
        t_tune = time.perf_counter() - t0
        log(f"{form}: {len(tuned)} keys tuned in {t_tune:.1f} s")

        # 2. one batched call
        outs = [mra.AlignResult.empty(p.shape[0], dev) for _, _, p in data]
        stacks = [(base + i, p, -1, o) for i, ((_, _, p), o) in enumerate(zip(data, outs))]
        ctx.align_batch(stacks[:8])         # warm: workspace growth to its cap
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.align_batch(stacks)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        log(f"{form}: batch {t_batch:.2f} s, {n_total / t_batch:.4g} particles/s")

        # 3. per-stack calls
        t_single, same = None, None
        if not args.no_singles:
            singles = [mra.AlignResult.empty(p.shape[0], dev) for _, _, p in data]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i, ((_, _, p), o) in enumerate(zip(data, singles)):
                ctx.align(base + i, p, out=o)
            torch.cuda.synchronize()
            t_single = time.perf_counter() - t0
            same = 0
            for a, b in zip(outs, singles):
                x, y = a.to_numpy(), b.to_numpy()
                same += all(np.array_equal(x[k], y[k]) for k in x)
            log(f"{form}: per-stack calls {t_single:.2f} s; identical results {same}/{len(data)}")
        variants = {}
        for i in range(len(data)):
            v, c = ctx.get_tuning(base + i)
            e = cache.get(autotune.refset_key(ctx, base + i)) or {}
            k = f"{v}/{c}/run{e.get('run_tiles', 0)}"
            variants[k] = variants.get(k, 0) + 1
        line = dict(workload=f"uneven stacks: {len(data)} stacks, L in {{64,76,96,128}}, N 2k..50k "
                             f"(x{args.n_scale}), K 20..400, shifts +-2..+-5, own refset each, seed {args.seed}",
                    precision=form, particles=n_total, batch_s=round(t_batch, 4),
                    particles_per_s=round(n_total / t_batch, 1),
                    per_stack_calls_s=None if t_single is None else round(t_single, 4),
                    identical_to_per_stack_calls=None if same is None else f"{same}/{len(data)}",
                    tuned_keys=len(tuned), tune_s=round(t_tune, 2), variant_chunk_run_counts=variants)
        print(json.dumps(line), flush=True)
        for i in range(len(data)):
            ctx.unload_refs(base + i)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
