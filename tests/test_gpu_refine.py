"""Sub-step angle refinement on the GPU (mra_result.psi_frac) against the
oracle's parabola (oracle.refine_psi) and against planted rotations.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
L, K, T = 64, 5, 2


def log(msg):
    print(f"[gpu-refine] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


def circ(x):
    return np.abs((np.asarray(x, dtype=np.float64) + 128.0) % 256.0 - 128.0)


def setup(seed, N, snr, K=K):
    blobs = synth.make_blobs(K, L, seed=(seed, 0), rho_max=28)
    refs = synth.render_refs(blobs)
    parts, truth = synth.make_particles(blobs, N, T, snr, seed=(seed, 1))
    g = oracle.Geometry(L=L, r_min=1, r_max=30, n_phi=256, shift_max=T)
    return refs, parts, truth, g


@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_psi_frac_matches_the_oracle_parabola(ctx, form):
    refs, parts, _, g = setup(210, 40, 0.2)
    ctx.load_refs(100, refs.to(DEV), r_min=1, r_max=30, shift_max=T, precision=form)
    got = ctx.align(100, parts.to(DEV), with_psi_frac=True).to_numpy()
    want = oracle.refine_psi(parts.numpy(), refs.numpy(), g, got)   # the oracle at the GPU's parameters
    err = circ(got["psi_frac"] - want)
    assert err.max() <= 0.01, err.max()
    assert np.all(circ(got["psi_frac"] - got["psi"]) <= 0.5 + 1e-6)
    log(f"{form}: max |psi_frac - oracle| {err.max():.2e} steps")


def test_psi_frac_recovers_planted_off_grid_rotations(ctx):
    refs, parts, truth, g = setup(211, 24, None)
    ctx.load_refs(101, refs.to(DEV), r_min=1, r_max=30, shift_max=T)
    got = ctx.align(101, parts.to(DEV), with_psi_frac=True).to_numpy()
    np.testing.assert_array_equal(got["ref"], truth.ref)
    true_steps = (truth.alpha * 256.0 / (2.0 * math.pi)) % 256.0
    assert circ(got["psi_frac"] - true_steps).max() <= 0.02
    assert circ(got["psi"] - true_steps).max() <= 0.5 + 1e-6


def test_psi_frac_changes_nothing_else_in_every_path(ctx):
    from paper_2011_05755_amd import mra
    refs, parts, _, g = setup(212, 29, 0.1)
    p = parts.to(DEV)
    for rid, k in ((102, K), (103, 1)):       # the MRA path and the fused single-reference path
        ctx.load_refs(rid, refs[:k].to(DEV), r_min=1, r_max=30, shift_max=T, precision="bf16")
        plain = ctx.align(rid, p).to_numpy()
        full = ctx.align(rid, p, with_psi_frac=True).to_numpy()
        for key in plain:
            np.testing.assert_array_equal(plain[key], full[key], err_msg=(rid, key))
        assert np.all(np.isfinite(full["psi_frac"]))
        # inside a batch the stack takes the per-chunk path and gives the same
        o = mra.AlignResult.empty(29, DEV, with_psi_frac=True)
        o2 = mra.AlignResult.empty(7, DEV)
        ctx.align_batch([(rid, p, -1, o), (rid, p[:7], -1, o2)])
        for key, v in o.to_numpy().items():
            np.testing.assert_array_equal(v, full[key], err_msg=(rid, "batch", key))
