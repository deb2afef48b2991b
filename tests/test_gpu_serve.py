"""The serving loop on the GPU: requests of uneven size against several
resident refsets, arriving while others run (device- and host-resident
particles), give the same result bit for bit as each request aligned alone."""

import numpy as np
import pytest
import torch

from paper_2011_05755_amd import serve, synth

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
    fp = max(r.footprint() for _, r in arrivals)
    srv = serve.Server(serve.AlignExecutor(ctx), hbm_budget=(1 << 30) + 3 * fp, workspace_bytes=1 << 30,
                       step_rows=2000)
    stats = serve.run_trace(srv, arrivals)
    torch.cuda.synchronize()
    log(f"stats {stats}")
    assert stats["requests"] == 10 and stats["steps"] > 1
    assert srv.peak_used <= srv.budget
    for _, r in arrivals:
        alone = ctx.align(r.refset_id, r.parts.to(DEV)).to_numpy()
        got = r.out.to_numpy()
        for key in alone:
            np.testing.assert_array_equal(got[key], alone[key], err_msg=f"request {r.rid}: {key}")
    ctx.close()
