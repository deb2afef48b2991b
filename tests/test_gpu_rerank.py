"""Top-k FP32 re-ranking of the 16-bit forms (mra_geom.rescore_rows).

The 16-bit pass picks each row's best in 16-bit precision; with
rescore_rows = k the winners of the particle's k best rows and their
neighbours one angle step either side are re-scored in FP32 and the best
becomes the result.  Checked against the oracle: the reported CC is the
oracle's CC of the reported candidate (FP32 re-score, 1e-5), the chosen
candidate is never worse in the oracle than the plain 16-bit winner (beyond
FP32 rounding), agreement with the oracle's parameters does not drop, and
results are the same in a batched launch.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-rerank] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


def case(seed, N=160, L=64, K=10, T=2, snr=0.1):
    blobs = synth.make_blobs(K, L, seed=(seed, 0), rho_max=L / 2 - 4)
    refs = synth.render_refs(blobs)
    parts, _ = synth.make_particles(blobs, N, T, snr, seed=(seed, 1))
    g = oracle.Geometry(L=L, r_min=1, r_max=30, n_phi=256, shift_max=T)
    return refs, parts, g


def oracle_cc_of(table, res, g):
    """Oracle CC of each particle's reported candidate (from the full table)."""
    S1 = 2 * g.shift_max + 1
    out = np.empty(len(res["ref"]))
    for n in range(len(out)):
        a = (256 - res["psi"][n]) % 256
        out[n] = table[n, res["ref"][n], res["mirror"][n], res["shift_y"][n] + g.shift_max,
                       res["shift_x"][n] + g.shift_max, a]
    return out


@pytest.mark.parametrize("form", ["bf16", "fp16"])
def test_reranked_winner_is_never_worse_and_reports_its_fp32_cc(ctx, form):
    refs, parts, g = case(95)
    table = oracle.cc_table(parts.numpy(), refs.numpy(), g)   # [N, K, M, S1, S1, 256]
    want = oracle.align(parts.numpy(), refs.numpy(), g)
    got = {}
    # 2, 3 and 8 rows as well: odd candidate counts end in a single-candidate
    # pass after the pairs
    for rows in (1, 2, 3, 4, 8):
        ctx.load_refs(90, refs.to(DEV), r_min=1, r_max=30, shift_max=g.shift_max, precision=form,
                      rescore_rows=rows)
        got[rows] = ctx.align(90, parts.to(DEV)).to_numpy()
    for rows, res in got.items():
        tcc = oracle_cc_of(table, res, g)
        assert (np.abs(res["cc"] - tcc) / np.abs(want["cc"])).max() <= 1e-5, rows
    # more rows re-score a superset of candidates: the winner never gets worse
    cc_of = {r: oracle_cc_of(table, got[r], g) for r in got}
    order = sorted(got)
    for lo, hi in zip(order, order[1:]):
        assert np.all(cc_of[hi] >= cc_of[lo] - 2e-5 * np.abs(want["cc"])), (lo, hi)
    c1, c4 = cc_of[1], cc_of[4]
    same = {r: int(np.sum(np.all([got[r][k] == want[k] for k in ("ref", "shift_x", "shift_y", "psi", "mirror")],
                                   axis=0))) for r in got}
    assert same[4] >= same[1]
    log(f"{form}: oracle parameters matched {same[1]} -> {same[4]} of {len(c1)} with 4-row re-ranking")


def mirror_symmetric(parts, L):
    """Each image made symmetric about the mirror axis, the horizontal line
    through the sampling centre (row L // 2): rows y and L - y averaged, row 0
    (whose partner lies outside the box, where images are zero) cleared."""
    c = L // 2
    ys = torch.arange(1, L)
    p = parts.clone()
    p[:, 1:, :] = 0.5 * (parts[:, ys, :] + parts[:, 2 * c - ys, :])
    p[:, 0, :] = 0
    return p


@pytest.mark.parametrize("form", ["bf16", "fp16"])
def test_mirror_symmetric_particles_rerank_candidates_of_both_mirrors(ctx, form):
    """Particles symmetric about the mirror axis: every mirrored row ties with
    the unmirrored row at the opposite vertical shift, so a particle's best
    rows come in pairs of both mirrors and the re-ranking evaluates candidates
    of both mirrors side by side.  Each reported CC is still the oracle's CC of
    the reported candidate, and the re-ranked winner is never worse."""
    refs, parts, g = case(99, N=48)
    sym = mirror_symmetric(parts, g.L)
    table = oracle.cc_table(sym.numpy(), refs.numpy(), g)   # [N, K, M, S1 (sy), S1 (sx), 256]
    want = oracle.align(sym.numpy(), refs.numpy(), g)
    scale = np.abs(want["cc"])
    # the construction: mirror 1 at (sx, sy) equals mirror 0 at (sx, -sy)
    np.testing.assert_allclose(table[:, :, 1], table[:, :, 0, ::-1], rtol=0, atol=1e-9 * scale.max())
    got = {}
    for rows in (1, 4):
        ctx.load_refs(94, refs.to(DEV), r_min=1, r_max=30, shift_max=g.shift_max, precision=form,
                      rescore_rows=rows)
        got[rows] = ctx.align(94, sym.to(DEV), with_cc2=True).to_numpy()
    for rows, res in got.items():
        tcc = oracle_cc_of(table, res, g)
        assert (np.abs(res["cc"] - tcc) / scale).max() <= 1e-5, rows
    # the GPU sees the tie too: the best candidate other than the winner (its
    # mirror partner) is within the 16-bit tolerance of the winner
    assert np.all(np.abs(got[4]["cc2"] - got[4]["cc"]) <= 2e-3 * scale)
    c1, c4 = oracle_cc_of(table, got[1], g), oracle_cc_of(table, got[4], g)
    assert np.all(c4 >= c1 - 2e-5 * scale)
    best = {r: int(np.sum(np.abs(oracle_cc_of(table, got[r], g) - want["cc"]) <= 2e-5 * scale)) for r in got}
    assert best[4] >= best[1]
    log(f"{form} symmetric: oracle's best CC reached {best[1]} -> {best[4]} of {len(c1)}; "
        f"mirror 1 reported for {int(np.sum(got[4]['mirror']))}")


def test_rescore_rows_one_is_the_plain_rescore_and_batch_matches(ctx):
    from paper_2011_05755_amd import mra
    refs, parts, g = case(96, N=37)
    p = parts.to(DEV)
    outs = {}
    for rows in (0, 1, 4):
        ctx.load_refs(91, refs.to(DEV), r_min=1, r_max=30, shift_max=g.shift_max, precision="bf16",
                      rescore_rows=rows)
        outs[rows] = ctx.align(91, p).to_numpy()
    for key in outs[0]:
        np.testing.assert_array_equal(outs[0][key], outs[1][key], err_msg=key)
    # batched launch of two pieces with re-ranking equals the single call
    o = mra.AlignResult.empty(37, DEV)
    o2 = mra.AlignResult.empty(20, DEV)
    ctx.align_batch([(91, p, -1, o), (91, p[:20], -1, o2)])
    for key, v in o.to_numpy().items():
        np.testing.assert_array_equal(v, outs[4][key], err_msg=key)
    for key, v in o2.to_numpy().items():
        np.testing.assert_array_equal(v, outs[4][key][:20], err_msg=key)


def test_runner_up_excludes_the_reranked_winner(ctx):
    refs, parts, g = case(97, N=24)
    ctx.load_refs(92, refs.to(DEV), r_min=1, r_max=30, shift_max=g.shift_max, precision="bf16", rescore_rows=4)
    res = ctx.align(92, parts.to(DEV), with_cc2=True).to_numpy()
    assert np.all(np.isfinite(res["cc2"]))
    table = oracle.cc_table(parts.numpy(), refs.numpy(), g).reshape(24, -1)
    # the runner-up is a 16-bit value of some other candidate: within the
    # 16-bit tolerance of the oracle's best over everything but the winner
    for n in range(24):
        t = table[n].copy()
        t[res["flat_index"][n]] = -np.inf
        assert abs(res["cc2"][n] - t.max()) <= 2e-3 * abs(res["cc"][n])


def test_rescore_rows_is_validated(ctx):
    from paper_2011_05755_amd import mra
    refs, _, g = case(98, N=1)
    with pytest.raises(mra.MRAError):
        ctx.load_refs(93, refs.to(DEV), r_min=1, r_max=30, shift_max=g.shift_max, precision="bf16", rescore_rows=9)
