"""Iterative MRA (mra_classify) on the 100k-particle workload.

100 000 particles of 76 px from 100 classes (SNR 0.05, shifts +-3, rings
1..35, 256 angles).  The loop starts from K particles drawn at random as the
initial references (no knowledge of the classes), runs until at most
``--frac`` of the particles change class or ``--max-iter`` passes, and
prints one JSON line: passes, particles reassigned per pass, wall time per
pass, and how well the final classes recover the planted ones (the share of
particles whose final class holds a majority of their planted class).

    python -m bench.iterate --precision fp32
"""

from __future__ import annotations

import argparse
import json
import sys
import time


def log(msg):
    print(f"[iterate] {msg}", file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--max-iter", type=int, default=20)
    ap.add_argument("--frac", type=float, default=0.005)
    ap.add_argument("--n-scale", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from paper_2011_05755_amd import mra, synth
    dev = torch.device("cuda", 0)
    w = dict(synth.WORKLOADS["mra_c1"])
    N = max(w["K"], int(round(w["N"] * args.n_scale)))
    blobs = synth.make_blobs(w["K"], w["L"], seed=(w["seed"], 0), rho_max=w["rho_max"])
    parts, truth = synth.make_particles(blobs, N, w["shift_max"], w["snr"], seed=(w["seed"], 1), device=dev)
    pick = np.random.default_rng(args.seed).choice(N, w["K"], replace=False)
    start = parts[torch.as_tensor(pick, device=dev)].clone()
    torch.cuda.synchronize()
    log(f"{N} particles generated")

    ctx = mra.Context(0)
    # warm-up: one pass on a slice builds the kernels' state and the workspace
    warm = start.clone()
    ctx.classify(0, parts[:4096], warm, r_min=w["r_min"], r_max=w["r_max"], shift_max=w["shift_max"],
                 max_iter=1, precision=args.precision)
    torch.cuda.synchronize()
    avg = start.clone()
    t0 = time.perf_counter()
    out, counts, n_iter, changed = ctx.classify(0, parts, avg, r_min=w["r_min"], r_max=w["r_max"],
                                                shift_max=w["shift_max"], max_iter=args.max_iter,
                                                max_changed_frac=args.frac, precision=args.precision)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{n_iter} passes in {dt:.2f} s")

    # class recovery: for each final class, its majority planted class
    ref = out.ref.cpu().numpy()
    tab = np.zeros((w["K"], w["K"]), dtype=np.int64)
    np.add.at(tab, (ref, truth.ref), 1)
    recovered = tab.max(axis=1).sum() / N
    line = dict(workload=f"iterative MRA: {N} particles, L={w['L']}, K={w['K']}, shifts +-{w['shift_max']}, "
                         f"rings {w['r_min']}..{w['r_max']} x 256, SNR {w['snr']}, "
                         f"start from {w['K']} random particles",
                precision=args.precision, passes=n_iter, changed_per_pass=changed,
                stop_rule=f"changed <= {args.frac} N or {args.max_iter} passes",
                total_s=round(dt, 3), s_per_pass=round(dt / n_iter, 4),
                aligned_particles_per_s=round(N * n_iter / dt, 1),
                nonempty_classes=int((counts.cpu().numpy() > 0).sum()),
                majority_purity=round(float(recovered), 4))
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
