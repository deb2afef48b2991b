"""The serving loop on the GPU: requests of uneven size against several
resident refsets, arriving while others run (device- and host-resident
particles), give the same result bit for bit as each request aligned alone,
and every request agrees with the FP64 oracle (one alignment pass of
Algorithm 1 per request) at its form's tolerance.  A request against a refset
that is not loaded fails on its own while the others complete."""

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import serve, synth
from parity import check_align, check_rescored_cc

ORACLE_PER_REQUEST = 16     # particles of each request checked against the oracle

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-serve] {msg}", flush=True)


@pytest.mark.parametrize("precision,host", [("bf16", False), ("fp32", True)])
def test_results_are_the_same_alone_and_in_the_mix(precision, host):
    from paper_2011_05755_amd import mra
    log(f"{precision}, host inputs {host}")
    ctx = mra.Context(0, workspace_cap=1 << 30)
    specs = [dict(L=64, K=9, shift_max=2, r_min=1, r_max=30, n_phi=256, snr=0.1, rho_max=28.0),
             dict(L=76, K=20, shift_max=1, r_min=1, r_max=35, n_phi=256, snr=0.1, rho_max=34.0),
             dict(L=96, K=5, shift_max=3, r_min=1, r_max=46, n_phi=256, snr=0.1, rho_max=44.0)]
    sets = serve.make_refsets(ctx, 3, seed=11, precision=precision, specs=specs)
    rng = np.random.default_rng(12)
    arrivals, t = [], 0.0
    for j in range(10):
        t += rng.exponential(0.002)
        s = sets[int(rng.integers(3))]
        N = int(rng.integers(1, 40))
        parts, _ = synth.make_particles(s["blobs"], N, s["shift_max"], s["snr"], seed=(12, j), device=DEV)
        if host:
            parts = parts.cpu().pin_memory()
        arrivals.append((t, serve.Request(refset_id=s["id"], N=N, L=s["L"], shift_max=s["shift_max"],
                                          parts=parts, out=mra.AlignResult.empty(N, DEV))))
    # one request against a refset id that is not loaded, in the middle of the trace
    bad_parts, _ = synth.make_particles(sets[0]["blobs"], 7, 2, 0.1, seed=(12, 99), device=DEV)
    bad = serve.Request(refset_id=77, N=7, L=64, shift_max=2, parts=bad_parts.cpu().pin_memory() if host else bad_parts,
                        out=mra.AlignResult.empty(7, DEV))
    ctx.refsets[77] = ctx.refsets[0]          # the binding accepts it; the library refuses refset 77
    arrivals.insert(5, (arrivals[4][0], bad))
    fp = max(r.footprint() for _, r in arrivals)
    srv = serve.Server(serve.AlignExecutor(ctx), hbm_budget=(1 << 30) + 3 * fp, workspace_bytes=1 << 30,
                       step_rows=2000)
    stats = serve.run_trace(srv, arrivals)
    torch.cuda.synchronize()
    log(f"stats {stats}")
    assert stats["requests"] == 10 and stats["steps"] > 1 and stats["failed_requests"] == 1
    assert bad.error is not None and "not loaded" in bad.error, bad.error
    del ctx.refsets[77]
    assert srv.peak_used <= srv.budget and srv.used == 0
    by_id = {x["id"]: x for x in sets}
    tol = 1e-5 if precision == "fp32" else 2e-3
    for _, r in arrivals:
        if r is bad:
            continue
        alone = ctx.align(r.refset_id, r.parts.to(DEV)).to_numpy()
        got = r.out.to_numpy()
        for key in alone:
            np.testing.assert_array_equal(got[key], alone[key], err_msg=f"request {r.rid}: {key}")
        sp = by_id[r.refset_id]
        g = oracle.Geometry(L=sp["L"], r_min=sp["r_min"], r_max=sp["r_max"], n_phi=256, shift_max=r.shift_max)
        n = min(r.N, ORACLE_PER_REQUEST)
        pn, rn = r.parts[:n].cpu().numpy(), sp["refs"].cpu().numpy()
        want = oracle.align(pn, rn, g)
        sub = {k: v[:n] for k, v in got.items()}
        err, frac = check_align(sub, want, tol)
        if precision != "fp32":
            qhat, _ = oracle.reference_polar(rn, g)
            check_rescored_cc(sub, pn, qhat, g)
        log(f"request {r.rid} (L={r.L} N={r.N} T={r.shift_max}): oracle on {n}, max rel CC err {err:.2e}")
    ctx.close()
