"""Reference-free alignment (RFA) on a 100k-particle single-class stack.

100 000 particles of 76 px rendered from one blob reference (random
rotation, integer shift within the search range, mirror with p = 0.5, SNR
0.05), rings 1..35 x 256 angles.  For every search range T in --shifts the
single-reference pass (the fused K = 1 kernel) is timed against a resident
reference, kernel time from HIP events and wall time per pass, like the
paper's RFA timing over shift ranges (Fig. 5b); then one RFA loop from the
plain mean runs at T = 3.  One JSON line per measurement.

    python -m bench.rfa_bench --shifts 1,2,3,4,5
"""

from __future__ import annotations

import argparse
import json
import sys
import time


def log(msg):
    print(f"[rfa-bench] {msg}", file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=100000)
    ap.add_argument("--shifts", default="1,2,3,4,5")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--loop-iters", type=int, default=10)
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args(argv)

    import torch

    from paper_2011_05755_amd import mra, synth
    dev = torch.device("cuda", 0)
    L, r_min, r_max = 76, 1, 35
    Ts = [int(t) for t in args.shifts.split(",") if t]
    Tmax = max(Ts + [3])
    blobs = synth.make_blobs(1, L, seed=(args.seed, 0), rho_max=28.0)
    ref = synth.render_refs(blobs).to(dev)
    parts, _ = synth.make_particles(blobs, args.N, Tmax, 0.05, seed=(args.seed, 1), device=dev)
    torch.cuda.synchronize()
    log(f"{args.N} particles generated (shifts drawn within +-{Tmax})")

    ctx = mra.Context(0)
    for T in Ts:
        ctx.load_refs(0, ref, r_min=r_min, r_max=r_max, shift_max=T)
        out = mra.AlignResult.empty(args.N, dev, with_cc2=True)
        ctx.align(0, parts[:2048], out=out.narrow(0, 2048))   # warm-up
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.reps):
            ctx.align(0, parts, out=out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.reps
        ms, launches = ctx.profile_read("rfa")
        ctx.profile(False)
        kern = ms / launches
        S = (2 * T + 1) ** 2
        print(json.dumps(dict(
            workload=f"RFA pass: {args.N} particles, L={L}, one reference, shifts +-{T} ({S}), both mirrors, "
                     f"rings {r_min}..{r_max} x 256",
            shift_max=T, kernel_ms=round(kern, 3), wall_ms=round(wall * 1e3, 3),
            particles_per_s=round(args.N / wall, 1),
            candidates_per_s=round(args.N * S * 2 * 256 / wall, 1))), flush=True)
        log(f"T={T}: kernel {kern:.2f} ms, wall {wall * 1e3:.2f} ms")

    T = 3
    t0 = time.perf_counter()
    out, avg, n, changed = ctx.rfa(1, parts, r_min=r_min, r_max=r_max, shift_max=T, max_iter=args.loop_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps(dict(
        workload=f"RFA loop from the plain mean: {args.N} particles, L={L}, shifts +-{T}, rings {r_min}..{r_max}",
        passes=n, changed_per_pass=changed, total_s=round(dt, 3), s_per_pass=round(dt / n, 4))), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
