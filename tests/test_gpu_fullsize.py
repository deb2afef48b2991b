"""The 100k-particle workload (N=100000, L=76, K=100, shifts +-3, rings 1..35)
at full size, in the launch configuration bench.py times.

The FP64 oracle checks sampled particles (the first and last, both sides of
chunk boundaries, and random ones); every one of the 100k outputs is checked
against properties that hold at any size: parameter ranges, the flat index
decoding to the reported parameters, cc2 <= cc, and the BF16 form choosing
the FP32 form's parameters wherever FP32's own top-two gap exceeds the BF16
tolerance.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-fullsize] {msg}", flush=True)


@pytest.fixture(scope="module")
def workload():
    w = synth.WORKLOADS["mra_c1"]
    blobs = synth.make_blobs(w["K"], w["L"], seed=(w["seed"], 0), rho_max=w["rho_max"])
    refs = synth.render_refs(blobs).to(DEV)
    parts, truth = synth.make_particles(blobs, w["N"], w["shift_max"], w["snr"], seed=(w["seed"], 1), device=DEV)
    torch.cuda.synchronize()
    return w, refs, parts


def decode_ok(res, w):
    S1 = 2 * w["shift_max"] + 1
    M = 2
    ang = (256 - res["psi"]) % 256
    flat = ((((res["ref"] * M + res["mirror"]) * S1 + res["shift_y"] + w["shift_max"]) * S1
             + res["shift_x"] + w["shift_max"]) * 256 + ang)
    return flat == res["flat_index"]


def test_full_size_sampled_parity_and_properties(workload):
    from paper_2011_05755_amd import mra
    w, refs, parts = workload
    N, K, T = w["N"], w["K"], w["shift_max"]
    ctx = mra.Context(0)
    out = {}
    for i, form in enumerate(("fp32", "bf16")):
        log(f"{form}: aligning {N} particles")
        ctx.load_refs(i, refs, r_min=w["r_min"], r_max=w["r_max"], shift_max=T, precision=form)
        out[form] = ctx.align(i, parts, with_cc2=(form == "fp32")).to_numpy()
    torch.cuda.synchronize()

    # properties of every output
    for form, res in out.items():
        assert np.all((res["ref"] >= 0) & (res["ref"] < K)), form
        for key in ("shift_x", "shift_y"):
            assert np.all(np.abs(res[key]) <= T), (form, key)
        assert np.all((res["psi"] >= 0) & (res["psi"] < 256)) and np.all((res["mirror"] == 0) | (res["mirror"] == 1))
        assert np.all(np.isfinite(res["cc"])), form
        assert np.all(decode_ok(res, w)), form
    f32, b16 = out["fp32"], out["bf16"]
    assert np.all(f32["cc2"] <= f32["cc"])
    decided = (f32["cc"] - f32["cc2"]) >= 2e-3 * np.abs(f32["cc"])
    for key in ("ref", "shift_x", "shift_y", "mirror", "psi"):
        bad = np.nonzero((f32[key] != b16[key]) & decided)[0]
        assert bad.size == 0, f"bf16 {key} differs from fp32 at decided particles {bad[:10]}"
    log(f"fp32-decided at the bf16 tolerance: {decided.sum()} of {N}")

    # sampled particles against the oracle
    rng = np.random.default_rng(9)
    idx = {0, 1, N - 2, N - 1}
    # around chunk boundaries of the default workspace (32 GiB, half of it for
    # the particle operand of 128 slots x 4 ceil(R/4) rings x 16 floats per 8 rows)
    R4 = (w["r_max"] - w["r_min"] + 4) // 4
    chunk = (32 << 30) // 2 // ((2 * T + 1) ** 2 * 128 * R4 * 64 * 4 // 8)
    for b in (chunk, 2 * chunk, 50000):
        idx.update({b - 1, b})
    idx.update(int(i) for i in rng.integers(0, N, 6))
    idx = np.array(sorted(idx))
    g = oracle.Geometry(L=w["L"], r_min=w["r_min"], r_max=w["r_max"], n_phi=256, shift_max=T)
    want = oracle.align(parts[torch.as_tensor(idx, device=DEV)].cpu().numpy(), refs.cpu().numpy(), g)
    for form, tol in (("fp32", 1e-5), ("bf16", 2e-3)):
        got = {k: v[idx] for k, v in out[form].items()}
        rel = np.abs(got["cc"] - want["cc"]) / np.abs(want["cc"])
        assert rel.max() <= tol, f"{form}: max rel cc err {rel.max():.3g}"
        ok = (want["cc"] - want["cc2"]) >= tol * np.abs(want["cc"])
        for key in ("ref", "shift_x", "shift_y", "mirror", "psi"):
            bad = np.nonzero((got[key] != want[key]) & ok)[0]
            assert bad.size == 0, f"{form} {key} differs at sampled particles {idx[bad]}"
        if form == "fp32":
            rel2 = np.abs(got["cc2"] - want["cc2"]) / np.abs(want["cc"])
            assert rel2.max() <= 1e-5
        log(f"{form}: {len(idx)} sampled particles, max rel cc err {rel.max():.2e}, decided {ok.sum()}")
    ctx.close()
