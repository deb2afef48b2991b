#!/usr/bin/env python3
"""Throughput of one multi-reference-alignment pass on one MI355X.

A step is one pass of the hot path over the 100k-particle workload
(N=100000, L=76, K=100 references, shifts +-3 px (49), both mirrors,
rings 1..35 x 256 angles, SNR 0.05): mra_align (polar resampling + ring
FFTs, correlation contraction on the matrix cores, inverse FFT over angle,
arg-max) followed by mra_update_averages.  References are loaded once
before timing; particles are resident in HBM when the timed region starts.

Prints one JSON line.  `value` is the FP32 form's aligned particles/s; the
BF16-matrix-core form (FP32 re-score of the winner) is reported beside it.
`roofline` covers the dominant kernel (the fused correlation kernel), timed
with HIP events on the library's stream; its `traffic` (HBM bytes per
launch) comes from the counter summary under profiles/ when that summary was
taken on the current kernel sources, else null.  `serving` runs the
continuous-batching server on a bounded trace (BF16, 8 resident refsets of
the uneven-stack distribution, Poisson arrivals at 20/s and at a rate one
GPU sustains) and reports p50/p99 latency and particles/s.  `cpu_baseline`
times the FP64 oracle on a sample of the same stack.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "aligned particles/s (L=76,K=100,±3px); FP32 vs BF16-MFMA; p50/p99 latency"
FP32_MATRIX_PEAK = 157.3   # TFLOP/s, MI355X dense FP32 matrix
BF16_MATRIX_PEAK = 2500.0  # TFLOP/s, dense
FP32_VECTOR_PEAK = 157.3   # TFLOP/s, MI355X FP32 vector (published; counts packed FP32)
# reachable without packed FP32 (which the library's compile flags disable): 256 CUs x 4 SIMDs
# x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VALU_PEAK = 78.6
HBM_PEAK = 8000.0          # GB/s
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "mra_c1_hbm_traffic.md")
CSRC = os.path.join(ROOT, "paper_2011_05755_amd", "csrc")
# sources each kernel's code is built from (a change to any of them voids
# counter figures taken before it)
KERNEL_SOURCES = {
    "k_corr": ["corr_impl.h", "k_corr.hip", "k_corr_fp32.hip", "k_corr_bf16.hip", "k_corr_fp16.hip", "mra_common.h",
               "mra_fft.h"],
    "k_polar_fft": ["k_polar.hip", "polar_impl.h", "mra_fft.h", "mra_common.h"],
    "k_avg": ["k_avg.hip", "mra_common.h"],
}


def kernel_sources_sha(kernel: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, form: str, workspace_gib: int):
    """HBM bytes per launch of `kernel` in `form` from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None
    when the summary is missing, was taken with another chunking, or on
    other kernel sources."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            m = re.search(r"<!-- traffic: (\{.*?\}) -->", f.read(), re.S)
        e = json.loads(m.group(1))[kernel][form]
    except (OSError, AttributeError, KeyError, ValueError):
        return None
    if e.get("sources_sha") != kernel_sources_sha(kernel) or e.get("workspace_gib") != workspace_gib:
        return None
    return float(e["bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def corr_flops_per_row_ref(R: int) -> float:
    # per (particle row, reference): 128 frequency slots x 4 real dot products
    # of length R (both mirrors), 2 flops per multiply-add
    return 128 * 4 * R * 2.0


def ifft_flops_per_row_ref() -> float:
    # 256-point complex inverse FFT as 16 x 16: 32 DFT16 (8 DFT4 = 128 adds,
    # 7 general complex products = 42 flops) + 225 inter-pass complex products
    return 32 * (128 + 42) + 225 * 6.0


def run_serving(args, bench_ctx, dev) -> dict:
    """Two bounded traces of the serving workload (8 resident BF16 refsets
    drawn from the uneven-stack distribution; request sizes N ~ U{2k..50k},
    each a slice of one pre-generated device stack per refset): Poisson 20/s,
    which offers more than one GPU serves, and a sustainable rate.  Latency
    is completion minus arrival; the first requests of each trace are not
    left out (the server starts empty)."""
    import torch
    from paper_2011_05755_amd import mra, serve
    ws = 8 << 30
    ctx = mra.Context(0, workspace_cap=ws)
    sets = serve.make_refsets(ctx, 8, seed=5, precision="bf16")
    out = {}
    legs = [(args.serve_rate, args.serve_requests), (args.serve_sustained_rate, args.serve_sustained)]
    for j, (rate, n_req) in enumerate(legs):
        if n_req <= 0:
            continue
        arrivals = serve.make_requests(sets, n_req, rate, seed=5 + j, device=dev, pool=True)
        torch.cuda.synchronize()
        srv = serve.Server(serve.AlignExecutor(ctx), hbm_budget=96 << 30, workspace_bytes=ws, step_rows=1 << 18)
        log(f"serving: {n_req} requests at Poisson {rate}/s")
        stats = serve.run_trace(srv, arrivals)
        torch.cuda.synchronize()
        offered = sum(r.N for _, r in arrivals) / max(arrivals[-1][0], 1e-9)
        out[f"poisson_{rate:g}_per_s"] = dict(
            requests=stats["requests"], failed=stats["failed_requests"], particles=stats["particles"],
            p50_latency_s=round(stats["p50_s"], 4), p99_latency_s=round(stats["p99_s"], 4),
            particles_per_s=round(stats["particles_per_s"], 1), offered_particles_per_s=round(offered, 1),
            makespan_s=round(stats["makespan_s"], 3), max_waiting=stats["max_waiting"])
        log(f"serving {rate}/s: p50 {stats['p50_s']:.3f} s, p99 {stats['p99_s']:.3f} s, "
            f"{stats['particles_per_s']:.4g} particles/s (offered {offered:.4g})")
        del arrivals, srv
    ctx.close()
    del sets
    torch.cuda.empty_cache()
    out["workload"] = ("8 resident refsets (uneven-stack distribution: L in {64,76,96,128}, K 20..400, shifts "
                       "+-2..+-5, rings 1..L/2-2), BF16 with FP32 re-ranking, request N ~ U{2000..50000} "
                       "(slices of one device-resident stack per refset), 96 GiB admission budget")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="fp32,bf16,fp16")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-h2d", action="store_true", help="skip the pinned-host-memory pass")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reads and writes MIB MiB), "
                         "a reference for hardware traffic counters")
    ap.add_argument("--workspace-gib", type=int, default=128,
                    help="library workspace cap (chunk size); 128 GiB of the GPU's 288 GB: a 100k pass in 3 FP32 / "
                         "2 16-bit chunks")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the 20/s serving leg (0: no serving legs)")
    ap.add_argument("--serve-sustained", type=int, default=16, help="requests of the sustainable-rate leg")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-sustained-rate", type=float, default=2.5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        return 2

    import torch
    from paper_2011_05755_amd import mra, synth

    dev = torch.device("cuda", 0)
    if args.copy_calibration > 0:
        n = args.copy_calibration << 18          # float32 elements
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del src, dst
    w = synth.WORKLOADS["mra_c1"]
    N, L, K, T, r_min, r_max = w["N"], w["L"], w["K"], w["shift_max"], w["r_min"], w["r_max"]
    R = r_max - r_min + 1
    S = (2 * T + 1) ** 2
    log(f"generating workload N={N} L={L} K={K} T={T}")
    blobs = synth.make_blobs(K, L, seed=(w["seed"], 0), rho_max=w["rho_max"])
    refs = synth.render_refs(blobs).to(dev)
    parts, truth = synth.make_particles(blobs, N, T, w["snr"], seed=(w["seed"], 1), device=dev)
    torch.cuda.synchronize()

    ctx = mra.Context(0, workspace_cap=args.workspace_gib << 30)
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    for i, form in enumerate(forms):
        ctx.load_refs(i, refs, r_min=r_min, r_max=r_max, shift_max=T, precision=form)
        out = mra.AlignResult.empty(N, dev)
        avg = refs.clone()

        def step():
            ctx.align(i, parts, out=out)
            ctx.update_averages(i, parts, out, avg)

        log(f"{form}: warmup {args.warmup}")
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ctx.profile(True)
        torch.cuda.synchronize()
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        marks[0].record(ctx.stream)
        for k in range(args.steps):
            step()
            marks[k + 1].record(ctx.stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per_step = [marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)]
        kern = {name: ctx.profile_read(name) for name in ("polar", "corr", "merge", "rescore", "averages")}
        ctx.profile(False)
        ms = dt * 1000.0 / args.steps
        log(f"{form}: {ms:.2f} ms/step (median {statistics.median(per_step):.2f}), {N / (ms / 1000):.4g} "
            "particles/s; kernels " + ", ".join(f"{k} {v[0] / args.steps:.2f} ms" for k, v in kern.items() if v[1]))
        results[form] = dict(ms=ms, median_ms=statistics.median(per_step), value=N / (ms / 1000.0), kern=kern,
                             out=out.to_numpy())

    # ---- the same pass with the particles in pinned host memory (H2D copy inside the timing) ----
    h2d = None
    if "fp32" in forms and not args.no_h2d:
        host = parts.cpu().pin_memory()
        i = forms.index("fp32")
        out = mra.AlignResult.empty(N, dev)
        avg = refs.clone()
        staged = torch.empty_like(parts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        staged.copy_(host, non_blocking=True)
        t1e = torch.cuda.Event(enable_timing=True)
        t0e = torch.cuda.Event(enable_timing=True)
        t0e.record(ctx.stream)
        ctx.align(i, staged, out=out)
        ctx.update_averages(i, staged, out, avg)
        t1e.record(ctx.stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h2d = dict(value=round(N / dt, 1), unit="particles/s", ms=round(dt * 1000, 3),
                   copy_gb=round(parts.numel() * 4 / 1e9, 3),
                   note="fp32 form; particles copied from pinned host memory before the pass (not overlapped)")
        log(f"fp32 with H2D: {dt * 1000:.1f} ms, {N / dt:.4g} particles/s")
        del host, staged

    # ---- roofline of the dominant kernel (fused correlation, FP32 form) ----
    head = "fp32" if "fp32" in results else forms[0]
    corr_ms, corr_n = results[head]["kern"]["corr"]
    corr_flops = corr_flops_per_row_ref(R) * N * S * K * args.steps
    achieved = corr_flops / (corr_ms / 1000.0) / 1e12
    peak = FP32_MATRIX_PEAK if head == "fp32" else BF16_MATRIX_PEAK
    R4 = (R + 3) // 4
    padded = corr_flops * (4 * R4) / R
    roofline = dict(bound="mfma", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4),
                    frac_padded=round(padded / (corr_ms / 1000.0) / 1e12 / peak, 4),
                    traffic=traffic_from_profile("k_corr", head, args.workspace_gib),
                    traffic_unit="bytes per launch (HBM, counter-measured)",
                    kernel="k_corr", launches_per_step=corr_n // args.steps,
                    avg_launch_ms=round(corr_ms / corr_n, 4),
                    flops_per_row_ref=corr_flops_per_row_ref(R))

    extra = {}
    for form in results:
        if form == head:
            continue
        r = results[form]
        cms, cn = r["kern"]["corr"]
        pms, _ = r["kern"]["polar"]
        # 16-bit forms: ring spectra written as 2-byte values
        pol16 = (N * L * L * 4 + N * S * 512 * R) * args.steps / (pms / 1000.0) / 1e9
        alu = ifft_flops_per_row_ref() * N * S * K * args.steps / (cms / 1000.0) / 1e12
        mf = corr_flops_per_row_ref(R) * N * S * K * args.steps / (cms / 1000.0) / 1e12
        extra[form] = dict(value=round(r["value"], 1), ms_per_step=round(r["ms"], 3),
                           median_ms_per_step=round(r["median_ms"], 3),
                           speedup_vs_fp32=round(results[head]["ms"] / r["ms"], 3) if head == "fp32" else None,
                           corr_avg_launch_ms=round(cms / cn, 4),
                           corr_matrix_tflops=round(mf, 2), corr_matrix_frac=round(mf / BF16_MATRIX_PEAK, 4),
                           corr_ifft_valu_tflops=round(alu, 2), corr_ifft_valu_frac=round(alu / FP32_VALU_PEAK, 4),
                           corr_traffic_bytes_per_launch=traffic_from_profile("k_corr", form, args.workspace_gib),
                           polar_hbm_gbps=round(pol16, 1), polar_hbm_frac=round(pol16 / HBM_PEAK, 4))

    kernels = {form: {k: round(v[0] / args.steps, 3) for k, v in r["kern"].items() if v[1]}
               for form, r in results.items()}

    # ---- the other kernels against their own rooflines (head form) ----
    def gbps(nbytes, key):
        t, n = results[head]["kern"][key]
        return nbytes * args.steps / (t / 1000.0) / 1e9 if n else float("nan")
    polar_bytes = N * L * L * 4 + N * S * 1024 * R        # images read + ring spectra written
    avg_bytes = N * L * L * 4 + 2 * K * L * L * 4         # images read + averages read and written
    ifft = ifft_flops_per_row_ref() * N * S * K * args.steps / (corr_ms / 1000.0) / 1e12
    rooflines = {
        "k_polar_fft": dict(bound="hbm", achieved=round(gbps(polar_bytes, "polar"), 1), peak=HBM_PEAK,
                            unit="GB/s", frac=round(gbps(polar_bytes, "polar") / HBM_PEAK, 4),
                            algorithmic_bytes_per_step=polar_bytes),
        "k_avg": dict(bound="hbm", achieved=round(gbps(avg_bytes, "averages"), 1), peak=HBM_PEAK, unit="GB/s",
                      frac=round(gbps(avg_bytes, "averages") / HBM_PEAK, 4), algorithmic_bytes_per_step=avg_bytes),
        "k_corr_ifft": dict(bound="alu", achieved=round(ifft, 2), peak=FP32_VALU_PEAK, unit="TFLOP/s",
                            frac=round(ifft / FP32_VALU_PEAK, 4), flops_per_row_ref=ifft_flops_per_row_ref(),
                            note="inverse FFT share of the fused correlation kernel, same launches"),
    }

    # ---- serving: continuous batching on bounded Poisson traces (BF16) ----
    serving = None
    if args.serve_requests > 0:
        serving = run_serving(args, ctx, dev)

    # ---- CPU baseline: the FP64 oracle on a sample of the same stack ----
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        ns = args.cpu_sample
        log(f"cpu baseline: oracle on {ns} particles")
        g = oracle.Geometry(L=L, r_min=r_min, r_max=r_max, n_phi=256, shift_max=T)
        p_host = parts[:ns].cpu().numpy()
        r_host = refs.cpu().numpy()
        t0 = time.perf_counter()
        qh, _ = oracle.reference_polar(r_host, g)
        bmat = oracle.rolled_reference_matrix(qh, g)
        t_prep = time.perf_counter() - t0
        t0 = time.perf_counter()
        want = oracle.align(p_host, r_host, g)
        t_all = time.perf_counter() - t0
        try:
            from threadpoolctl import threadpool_info
            threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
        except Exception:
            threads = len(os.sched_getaffinity(0))
        cpu_model = platform.processor() or "unknown"
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
        except (OSError, StopIteration):
            pass
        cpu = dict(value=round(ns / max(t_all - t_prep, 1e-9), 3), unit="particles/s",
                   cores=int(threads), kind="oracle",
                   sample=f"first {ns} particles of the same stack, FP64 direct ring sums "
                          f"({t_all:.1f} s incl. {t_prep:.1f} s reference preparation, which is excluded "
                          f"like mra_load_refs on the GPU)",
                   host=dict(cpu_model=cpu_model, affinity_cpus=len(os.sched_getaffinity(0)),
                             blas_threads=int(threads)))
        # (untimed) each sampled particle's gap from its best pose (reference,
        # mirror, shift) to the best of every other pose, from the oracle's
        # CC table: the 16-bit forms' decisions are checked where it is large
        pose_gap = np.empty(ns)
        for lo in range(0, ns, 8):
            tab = oracle.cc_table(p_host[lo:lo + 8], None, g, qhat=qh, bmat=bmat)
            per_pose = tab.reshape(tab.shape[0], -1, tab.shape[-1]).max(axis=2)
            top2 = np.sort(per_pose, axis=1)[:, -2:]
            pose_gap[lo:lo + tab.shape[0]] = top2[:, 1] - top2[:, 0]
        parity = {}
        for form, r in results.items():
            got = {k: v[:ns] for k, v in r["out"].items()}
            tol = 1e-5 if form == "fp32" else 2e-3
            rel = np.abs(got["cc"] - want["cc"]) / np.abs(want["cc"])
            decided = (want["cc"] - want["cc2"]) >= tol * np.abs(want["cc"])
            same = np.ones(ns, bool)
            for key in ("ref", "shift_x", "shift_y", "mirror", "psi"):
                same &= got[key] == want[key]
            pose_decided = pose_gap >= tol * np.abs(want["cc"])
            same_pose = np.ones(ns, bool)
            for key in ("ref", "shift_x", "shift_y", "mirror"):
                same_pose &= got[key] == want[key]
            dpsi = np.abs(((got["psi"] - want["psi"]) + 128) % 256 - 128)
            same_pose &= dpsi <= 1
            parity[form] = dict(sample=ns, max_rel_cc_err=float(rel.max()), argmax_agree=int(same.sum()),
                                decided=int(decided.sum()), decided_mismatch=int((decided & ~same).sum()),
                                pose_decided=int(pose_decided.sum()),
                                pose_mismatch=int((pose_decided & ~same_pose).sum()))
        log(f"parity sample: {parity}")

    line = {
        "metric": METRIC,
        "value": round(results[head]["value"], 1),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(results[head]["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else head,
        "data": "synthetic",
        "config": {"workload": f"mra_c1: N={N} L={L} K={K} shifts +-{T} (S={S}) mirror rings "
                               f"{r_min}..{r_max} x 256 angles, SNR {w['snr']}, blob references, seed {w['seed']}",
                   "step": "mra_align + mra_update_averages, references resident",
                   "workspace_gib": args.workspace_gib,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "median_ms_per_step": round(results[head]["median_ms"], 3),
        "rooflines_other_kernels": rooflines,
        "kernels_ms_per_step": kernels,
        "with_h2d": h2d,
        "serving": serving,
    }
    line.update(extra)
    if parity is not None:
        line["parity_sample"] = parity
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
