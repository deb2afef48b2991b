"""Exact pruning of the inverse FFT in the correlation kernel.

A (particle row, reference) pair whose upper bound on the CC over all angles
lies below the row's best so far is skipped; the bound is a theorem about
the spectra, inflated against rounding, so every result must be bit for bit
the one without pruning.  Checked for every precision and tile variant, for
the runner-up pass (cc2), the batched persistent launch and a near-noise-free
case (where most pairs are pruned) next to a pure-noise one (where few are).
"""

import numpy as np
import pytest
import torch

from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-prune] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


def same(x, y, what):
    for key in x:
        np.testing.assert_array_equal(x[key], y[key], err_msg=f"{what}: {key}")


def run_both(ctx, rid, parts, with_cc2, variant=-1):
    outs = []
    for prune in (0, 1):
        ctx.set_tuning(rid, corr_variant=variant, prune=prune)
        assert ctx.get_prune(rid) == bool(prune)
        outs.append(ctx.align(rid, parts, with_cc2=with_cc2).to_numpy())
    return outs


@pytest.mark.parametrize("form,variants", [("fp32", (0, 1, 2)), ("bf16", (0, 1)), ("fp16", (0, 1))])
@pytest.mark.parametrize("snr", [None, 0.05])
def test_pruning_changes_no_result(ctx, form, variants, snr):
    L, K, T, N = 64, 21, 2, 29          # 3 reference tiles, the last ragged; ragged row tiles
    blobs = synth.make_blobs(K, L, seed=(90, 0), rho_max=28)
    refs = synth.render_refs(blobs).to(DEV)
    parts = synth.make_particles(blobs, N, T, snr, seed=(90, 1), device=DEV)[0]
    ctx.load_refs(80, refs, r_min=1, r_max=30, shift_max=T, precision=form)
    for v in variants:
        log(f"{form} variant {v} snr {snr}")
        off, on = run_both(ctx, 80, parts, with_cc2=True, variant=v)
        same(off, on, f"{form} v{v}")


@pytest.mark.parametrize("mirror,normalize,r_min", [(False, True, 1), (True, False, 3)])
def test_pruning_without_mirror_or_normalisation(ctx, mirror, normalize, r_min):
    L, K, T, N = 48, 13, 1, 19
    blobs = synth.make_blobs(K, L, seed=(93, 0), rho_max=20)
    refs = synth.render_refs(blobs).to(DEV)
    parts = synth.make_particles(blobs, N, T, 0.2, seed=(93, 1), device=DEV, mirror=mirror)[0]
    for form in ("fp32", "bf16"):
        ctx.load_refs(86, refs, r_min=r_min, r_max=20, shift_max=T, precision=form, mirror=mirror,
                      normalize=normalize)
        off, on = run_both(ctx, 86, parts, with_cc2=True)
        same(off, on, f"{form} mirror={mirror} normalize={normalize}")


def test_pruning_in_the_batched_launch(ctx):
    from paper_2011_05755_amd import mra
    stacks, want = [], []
    for i, (L, K, T, N, r_max) in enumerate([(64, 10, 2, 17, 30), (48, 5, 1, 9, 20), (76, 12, 3, 11, 35)]):
        blobs = synth.make_blobs(K, L, seed=(91, i), rho_max=L / 2 - 4)
        refs = synth.render_refs(blobs).to(DEV)
        parts = synth.make_particles(blobs, N, T, 0.1, seed=(91, i + 10), device=DEV)[0]
        ctx.load_refs(81 + i, refs, r_min=1, r_max=r_max, shift_max=T, precision="bf16")
        ctx.set_tuning(81 + i, prune=0)
        want.append(ctx.align(81 + i, parts).to_numpy())
        ctx.set_tuning(81 + i, prune=1)
        stacks.append((81 + i, parts, -1, mra.AlignResult.empty(N, DEV)))
    ctx.align_batch(stacks)
    for (_, _, _, o), w in zip(stacks, want):
        same(o.to_numpy(), w, "batch")


def test_prune_setting_is_validated(ctx):
    from paper_2011_05755_amd import mra
    blobs = synth.make_blobs(3, 32, seed=(92, 0), rho_max=12)
    ctx.load_refs(85, synth.render_refs(blobs).to(DEV), r_min=1, r_max=13, shift_max=1)
    with pytest.raises(mra.MRAError):
        ctx.set_tuning(85, prune=2)
    assert ctx.get_prune(85)        # on by default
