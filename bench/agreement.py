"""Arg-max agreement of the 16-bit forms, with and without top-k FP32
re-ranking, on the 100k-particle workload.

Aligns the 100 000 particles (L = 76, K = 100, shifts +-3, rings 1..35, SNR
0.05) with the FP32 form and with BF16 / FP16 at rescore_rows 1 and 4, and
prints one JSON line per 16-bit setting: the share of particles whose five
parameters equal the FP32 form's, the same share among particles whose FP32
top-two gap is at least 1e-4 of |cc|, and the pass time.  (Agreement with
the FP64 oracle itself is asserted by the GPU test suite on sampled
particles, not here.)

    python -m bench.agreement
"""

from __future__ import annotations

import argparse
import json
import sys
import time


def log(msg):
    print(f"[agreement] {msg}", file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--forms", default="bf16,fp16")
    ap.add_argument("--rows", default="1,4")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from paper_2011_05755_amd import mra, synth
    dev = torch.device("cuda", 0)
    w = synth.WORKLOADS["mra_c1"]
    blobs = synth.make_blobs(w["K"], w["L"], seed=(w["seed"], 0), rho_max=w["rho_max"])
    refs = synth.render_refs(blobs).to(dev)
    parts, _ = synth.make_particles(blobs, w["N"], w["shift_max"], w["snr"], seed=(w["seed"], 1), device=dev)
    torch.cuda.synchronize()
    keys = ("ref", "shift_x", "shift_y", "psi", "mirror")
    ctx = mra.Context(0)

    def run(form, rows):
        ctx.load_refs(0, refs, r_min=w["r_min"], r_max=w["r_max"], shift_max=w["shift_max"], precision=form,
                      rescore_rows=rows)
        out = mra.AlignResult.empty(w["N"], dev, with_cc2=(form == "fp32"))
        ctx.align(0, parts[:4096], out=out.narrow(0, 4096))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.align(0, parts, out=out)
        torch.cuda.synchronize()
        return out.to_numpy(), time.perf_counter() - t0

    f32, t32 = run("fp32", 0)
    log(f"fp32 pass {t32:.3f} s")
    gap = (f32["cc"] - f32["cc2"]) >= 1e-4 * np.abs(f32["cc"])
    for form in [f for f in args.forms.split(",") if f]:
        for rows in [int(r) for r in args.rows.split(",") if r]:
            res, t = run(form, rows)
            same = np.all([res[k] == f32[k] for k in keys], axis=0)
            line = dict(workload=f"mra_c1: N={w['N']} L={w['L']} K={w['K']} shifts +-{w['shift_max']} rings "
                                 f"{w['r_min']}..{w['r_max']}, SNR {w['snr']}",
                        form=form, rescore_rows=rows, pass_s=round(t, 4), fp32_pass_s=round(t32, 4),
                        agree_with_fp32=round(float(same.mean()), 5),
                        agree_with_fp32_where_fp32_gap_ge_1e4=round(float(same[gap].mean()), 5),
                        particles_with_fp32_gap_ge_1e4=int(gap.sum()))
            print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
