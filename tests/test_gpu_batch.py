"""Uneven stacks in one persistent launch, and tile configurations.

Every stack's result from mra_align_batch must equal, bit for bit, its
result from mra_align alone; the tile variant and the chunk size must not
change any result either.  Stacks mix box sizes whose ring counts fall in
every operand bucket of the correlation kernel (R4 = 8, 9, 12, 16), shift
ranges, reference counts, empty stacks and per-stack shift overrides.  Every
non-empty stack is also checked against the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)

# (L, K, T, N, seed): rings 1..L/2-2 -> R4 = 8, 9, 12, 16
STACKS = [(64, 7, 2, 5, 60), (76, 12, 1, 9, 61), (96, 3, 3, 4, 62), (128, 5, 1, 3, 63),
          (64, 20, 1, 0, 64), (76, 9, 2, 6, 65)]


def log(msg):
    print(f"[gpu-batch] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def data():
    out = []
    for L, K, T, N, seed in STACKS:
        blobs = synth.make_blobs(K, L, seed=(seed, 0), rho_max=L / 2 - 4)
        refs = synth.render_refs(blobs).to(DEV)
        if N:
            parts, _ = synth.make_particles(blobs, N, T, 0.1, seed=(seed, 1), device=DEV)
        else:
            parts = torch.empty((0, L, L), device=DEV)
        out.append((refs, parts))
    return out


def same(a, b, what):
    for key in b:
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{what}: {key}")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_batch_of_mixed_ring_buckets_equals_single_runs(ctx, data, precision):
    from paper_2011_05755_amd import mra
    log(f"{precision}: batch of {len(STACKS)} uneven stacks")
    base = {"fp32": 100, "bf16": 200, "fp16": 300}[precision]
    stacks, singles = [], []
    for i, ((L, K, T, N, _), (refs, parts)) in enumerate(zip(STACKS, data)):
        rid = base + i
        ctx.load_refs(rid, refs, r_min=1, r_max=L // 2 - 2, shift_max=T, precision=precision)
        T_run = T - 1 if i == len(STACKS) - 1 else -1      # last stack: per-stack shift override
        if N:
            if T_run >= 0:
                ctx.load_refs(rid + 50, refs, r_min=1, r_max=L // 2 - 2, shift_max=T_run, precision=precision)
                singles.append(ctx.align(rid + 50, parts).to_numpy())
            else:
                singles.append(ctx.align(rid, parts).to_numpy())
        else:
            singles.append(None)
        stacks.append((rid, parts, T_run, mra.AlignResult.empty(N, DEV)))
    ctx.align_batch(stacks)
    torch.cuda.synchronize()
    for (rid, parts, _, out), single in zip(stacks, singles):
        if single is not None:
            same(out.to_numpy(), single, f"stack {rid}")

    # every stack (every ring bucket, and both widths of the 16-bit
    # reference operand's last step) against the oracle
    tol = 1e-5 if precision == "fp32" else 2e-3
    for i, ((L, K, T, N, _), (refs, parts)) in enumerate(zip(STACKS, data)):
        if not N:
            continue
        T_eff = stacks[i][2] if stacks[i][2] >= 0 else T
        g = oracle.Geometry(L=L, r_min=1, r_max=L // 2 - 2, n_phi=256, shift_max=T_eff)
        want = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(), g)
        got = stacks[i][3].to_numpy()
        rel = np.abs(got["cc"] - want["cc"]) / np.abs(want["cc"])
        assert rel.max() <= tol, f"stack {i}"
        decided = (want["cc"] - want["cc2"]) >= tol * np.abs(want["cc"])
        for key in ("ref", "shift_x", "shift_y", "mirror", "psi"):
            assert np.all((got[key] == want[key]) | ~decided), f"stack {i}: {key}"


@pytest.mark.parametrize("precision,variants", [("fp32", (0, 1, 2)), ("bf16", (0, 1)), ("fp16", (0, 1))])
def test_tile_variants_and_chunk_sizes_do_not_change_results(ctx, data, precision, variants):
    from paper_2011_05755_amd import mra
    log(f"{precision}: variants {variants} x chunk sizes")
    L, K, T, N, _ = STACKS[1]
    refs, parts = data[1]
    rid = 400 + variants[-1] * 10 + len(precision)
    ctx.load_refs(rid, refs, r_min=1, r_max=L // 2 - 2, shift_max=T, precision=precision)
    want = ctx.align(rid, parts).to_numpy()
    # the runner-up pass re-reads the particle operand in the layout the
    # variant's first pass had written
    want2 = ctx.align(rid, parts, with_cc2=True).to_numpy()
    for v in variants:
        for chunk in (0, 1, 4):
            ctx.set_tuning(rid, corr_variant=v, chunk_particles=chunk)
            assert ctx.get_tuning(rid) == (v, chunk)
            same(ctx.align(rid, parts).to_numpy(), want, f"variant {v} chunk {chunk}")
            same(ctx.align(rid, parts, with_cc2=True).to_numpy(), want2, f"cc2, variant {v} chunk {chunk}")
            out = mra.AlignResult.empty(N, DEV)
            ctx.align_batch([(rid, parts, -1, out)])
            same(out.to_numpy(), want, f"batch, variant {v} chunk {chunk}")
    ctx.set_tuning(rid)   # back to the default


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_run_length_does_not_change_results(ctx, precision):
    """A workgroup's run of consecutive row tiles carries each particle's best
    from one tile to the next as a pruning threshold; no run length (one tile
    each, odd lengths that end inside a particle, the whole chunk) may change
    any result, in the single, runner-up and batched launches."""
    from paper_2011_05755_amd import mra
    L, K, T, N = 64, 21, 2, 37            # 925 rows: 116 row tiles, the last ragged
    log(f"{precision}: run lengths")
    blobs = synth.make_blobs(K, L, seed=(66, 0), rho_max=28)
    refs = synth.render_refs(blobs).to(DEV)
    parts = synth.make_particles(blobs, N, T, 0.05, seed=(66, 1), device=DEV)[0]
    rid = 480 + len(precision)
    ctx.load_refs(rid, refs, r_min=1, r_max=30, shift_max=T, precision=precision)
    want = ctx.align(rid, parts).to_numpy()
    want2 = ctx.align(rid, parts, with_cc2=True).to_numpy()
    for run in (1, 2, 3, 7, 64):
        ctx.set_tuning(rid, run_tiles=run)
        same(ctx.align(rid, parts).to_numpy(), want, f"run {run}")
        same(ctx.align(rid, parts, with_cc2=True).to_numpy(), want2, f"cc2, run {run}")
        out = mra.AlignResult.empty(N, DEV)
        ctx.align_batch([(rid, parts, -1, out)])
        same(out.to_numpy(), want, f"batch, run {run}")
    ctx.set_tuning(rid)
    g = oracle.Geometry(L=L, r_min=1, r_max=30, n_phi=256, shift_max=T)
    ref = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(), g)
    tol = 1e-5 if precision == "fp32" else 2e-3
    assert (np.abs(want["cc"] - ref["cc"]) / np.abs(ref["cc"])).max() <= tol


def test_batch_cut_into_many_pieces_and_waves(ctx, data):
    from paper_2011_05755_amd import mra
    log("batch cut into more pieces than one launch holds")
    stacks, singles = [], []
    for i in (0, 1, 5):
        L, K, T, N, _ = STACKS[i]
        refs, parts = data[i]
        rid = 500 + i
        ctx.load_refs(rid, refs, r_min=1, r_max=L // 2 - 2, shift_max=T, precision="bf16")
        singles.append(ctx.align(rid, parts).to_numpy())
        ctx.set_tuning(rid, chunk_particles=1)     # one piece per particle: 20 pieces
        stacks.append((rid, parts, -1, mra.AlignResult.empty(N, DEV)))
    ctx.align_batch(stacks)
    torch.cuda.synchronize()
    for (rid, _, _, out), single in zip(stacks, singles):
        same(out.to_numpy(), single, f"stack {rid}")


def test_invalid_tuning_is_rejected(ctx, data):
    from paper_2011_05755_amd import mra
    L, K, T, N, _ = STACKS[3]
    refs, _ = data[3]
    ctx.load_refs(600, refs, r_min=1, r_max=L // 2 - 2, shift_max=T, precision="fp32")
    for v in (0, 1, 7):   # resident FP32 variants cannot hold R4 = 16
        with pytest.raises(mra.MRAError) as e:
            ctx.set_tuning(600, corr_variant=v)
        assert e.value.code == mra.MRA_E_INVAL
    with pytest.raises(mra.MRAError) as e:
        ctx.set_tuning(600, corr_variant=2, chunk_particles=-1)
    assert e.value.code == mra.MRA_E_INVAL
    ctx.set_tuning(600, corr_variant=2)
    assert ctx.get_tuning(600) == (2, 0)
