"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative CC error against the oracle's best): FP32 <= 1e-5;
BF16 / FP16 contraction <= 2e-3, and the reported CC (the FP32 re-score of
the chosen candidate) equals the oracle's value of that same candidate to
1e-5.  Alignment parameters must equal the oracle's except where the
oracle's own top-two gap is below the tolerance.  Averages: <= 1e-5 of the
largest |Y'| given identical parameters.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth
from parity import agreement, check_align, check_pose, pose_gap

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-parity] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


def make_case(L, K, T, N, snr, seed, rho=None, r_max=None, mirror=True, n_phi_grid=None):
    blobs = synth.make_blobs(K, L, seed=(seed, 0), rho_max=rho if rho else L / 2 - 4)
    refs = synth.render_refs(blobs).to(DEV)
    parts, truth = synth.make_particles(blobs, N, T, snr, seed=(seed, 1), device=DEV, mirror=mirror,
                                        n_phi_grid=n_phi_grid)
    return refs, parts, truth


def geom(L, r_max, T, mirror=True, normalize=True, r_min=1):
    return oracle.Geometry(L=L, r_min=r_min, r_max=r_max, n_phi=256, shift_max=T, mirror=int(mirror),
                           normalize=int(normalize))


def test_reference_preparation(ctx):
    log("reference polar samples and norms")
    L, K, T = 64, 10, 2
    refs, _, _ = make_case(L, K, T, 1, 0.1, 20)
    ctx.load_refs(1, refs, r_min=1, r_max=30, shift_max=T)
    qhat, norm = ctx.debug_refs(1)
    torch.cuda.synchronize()
    q_o, nu_o = oracle.reference_polar(refs.cpu().numpy(), geom(L, 30, T))
    np.testing.assert_allclose(norm.cpu().numpy(), nu_o, rtol=1e-12)
    np.testing.assert_allclose(qhat.cpu().numpy(), q_o, rtol=0, atol=2e-7 * np.abs(q_o).max())


@pytest.mark.parametrize("L,r_max,T", [(64, 30, 2), (76, 35, 3), (33, 14, 1)])
def test_polar_samples(ctx, L, r_max, T):
    log(f"polar samples L={L} r_max={r_max} T={T}")
    refs, parts, _ = make_case(L, 3, T, 3, 0.1, 21, rho=L / 2 - 4)
    ctx.load_refs(2, refs, r_min=1, r_max=r_max, shift_max=T)
    got = ctx.debug_polar(2, parts).cpu().numpy()
    g = geom(L, r_max, T)
    S1 = 2 * T + 1
    for n in range(parts.shape[0]):
        want = oracle.particle_polar(parts[n].cpu().numpy(), g)[0].reshape(S1 * S1, g.n_rings, 256)
        np.testing.assert_allclose(got[n], want, rtol=0, atol=2e-6 * np.abs(want).max())


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-3)])
def test_largest_geometry(ctx, precision, tol):
    # the largest box, ring count and search range the C ABI admits: 160 px,
    # rings 1..64 (R4 = 16), shifts +-8 (289 rows per mirror)
    log(f"largest geometry L=160 r_max=64 T=8 {precision}")
    L, r_max, T, K, N = 160, 64, 8, 3, 3
    refs, parts, _ = make_case(L, K, T, N, 0.1, 47)
    ctx.load_refs(36, refs, r_min=1, r_max=r_max, shift_max=T, precision=precision)
    g = geom(L, r_max, T)
    if precision == "fp32":
        got = ctx.debug_polar(36, parts[:1]).cpu().numpy()
        want = oracle.particle_polar(parts[0].cpu().numpy(), g)[0].reshape((2 * T + 1) ** 2, g.n_rings, 256)
        np.testing.assert_allclose(got[0], want, rtol=0, atol=2e-6 * np.abs(want).max())
    res = ctx.align(36, parts).to_numpy()
    want = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(), g)
    err, _ = check_align(res, want, tol)
    if precision != "fp32":   # the reported CC is the FP32 re-score of the chosen candidate
        qhat, _ = oracle.reference_polar(refs.cpu().numpy(), g)
        for n in range(N):
            v = oracle.candidate_cc(parts[n].cpu().numpy(), qhat[res["ref"][n]], g, res["shift_x"][n],
                                    res["shift_y"][n], res["mirror"][n], (256 - res["psi"][n]) % 256)
            assert abs(res["cc"][n] - v) <= 1e-5 * abs(v), (n, res["cc"][n], v)
    log(f"  max rel CC err {err:.2e}")
    ctx.unload_refs(36)


def test_ring_spectra_match_numpy_rfft_of_the_same_samples(ctx):
    log("ring spectra vs numpy rfft")
    L, T = 64, 2
    refs, parts, _ = make_case(L, 3, T, 3, 0.1, 22)
    ctx.load_refs(3, refs, r_min=1, r_max=30, shift_max=T)
    samples = ctx.debug_polar(3, parts).cpu().numpy().astype(np.float64)
    spec = ctx.debug_spectra(3, parts).cpu().numpy()
    ref = np.fft.rfft(samples, axis=-1)
    got = spec[..., 0] + 1j * spec[..., 1]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err


# rings 1..r_max: R4 = 8, 9, 12, 16 (one step of 8 rings per lane group; two
# with the 16-bit reference operand's last step 2, 4 or 8 wide)
@pytest.mark.parametrize("L,r_max", [(64, 30), (76, 35), (96, 46), (128, 62)])
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-3), ("fp16", 2e-3)])
def test_full_cc_table(ctx, precision, tol, L, r_max):
    log(f"full CC table {precision} L={L} rings 1..{r_max}")
    K, T, N = 10, 2, 5
    refs, parts, _ = make_case(L, K, T, N, 0.1, 23)
    ctx.load_refs(4, refs, r_min=1, r_max=r_max, shift_max=T, precision=precision)
    got = ctx.debug_cctable(4, parts).cpu().numpy()
    want = oracle.cc_table(parts.cpu().numpy(), refs.cpu().numpy(), geom(L, r_max, T))
    for n in range(N):
        scale = np.abs(want[n]).max()
        err = np.abs(got[n] - want[n]).max() / scale
        assert err <= tol, f"particle {n}: {err:.3g}"


@pytest.mark.parametrize("N", [1, 3, 61])
def test_align_fp32_small_shapes_and_ragged_sizes(ctx, N):
    log(f"align fp32 L=64 K=10 T=2 N={N}")
    L, K, T = 64, 10, 2
    refs, parts, _ = make_case(L, K, T, N, 0.1, 24 + N)
    ctx.load_refs(5, refs, r_min=1, r_max=30, shift_max=T)
    res = ctx.align(5, parts).to_numpy()
    want = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(), geom(L, 30, T))
    err, _ = check_align(res, want, 1e-5)
    flat = oracle.flat_index(geom(L, 30, T), want["ref"], want["mirror"], want["shift_x"], want["shift_y"],
                             (256 - want["psi"]) % 256)
    gap = (want["cc"] - want["cc2"]) >= 1e-5 * np.abs(want["cc"])
    np.testing.assert_array_equal(res["flat_index"][gap], flat[gap])
    log(f"  max rel CC err {err:.2e}")


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-3), ("fp16", 2e-3)])
def test_runner_up_cc2(ctx, precision, tol):
    """cc2 (best over every candidate but the winner, from the second pass)
    against the oracle's, relative to |cc|; the other outputs are those of a
    run without cc2; batch and single agree."""
    from paper_2011_05755_amd import mra
    log(f"runner-up cc2 {precision}")
    L, K, T, N = 64, 10, 2, 23
    refs, parts, _ = make_case(L, K, T, N, 0.1, 70)
    ctx.load_refs(40, refs, r_min=1, r_max=30, shift_max=T, precision=precision)
    res = ctx.align(40, parts, with_cc2=True).to_numpy()
    want = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(), geom(L, 30, T))
    rel = np.abs(res["cc2"] - want["cc2"]) / np.abs(want["cc"])
    assert rel.max() <= tol, f"max rel cc2 err {rel.max():.3g}"
    if precision == "fp32":
        assert np.all(res["cc2"] <= res["cc"])
    plain = ctx.align(40, parts).to_numpy()
    for key in plain:
        np.testing.assert_array_equal(res[key], plain[key])
    out = mra.AlignResult.empty(N, DEV, with_cc2=True)
    ctx.align_batch([(40, parts, -1, out)])
    got = out.to_numpy()
    for key in res:
        np.testing.assert_array_equal(got[key], res[key])
    log(f"  max rel cc2 err {rel.max():.2e}")


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_align_mixed_precision_with_fp32_rescore(ctx, precision):
    log(f"align {precision} L=64 K=10 T=2 N=48")
    L, K, T, N = 64, 10, 2, 48
    refs, parts, _ = make_case(L, K, T, N, 0.1, 30)
    ctx.load_refs(6, refs, r_min=1, r_max=30, shift_max=T, precision=precision)
    res = ctx.align(6, parts).to_numpy()
    g = geom(L, 30, T)
    pn, rn = parts.cpu().numpy(), refs.cpu().numpy()
    want = oracle.align(pn, rn, g)
    # CC within 2e-3 of the oracle's best; parameters equal wherever the
    # oracle's top-two gap is at least 2e-3
    err, frac = check_align(res, want, 2e-3)
    # the teeth: the pose (reference, shifts, mirror) equal and psi within one
    # step wherever every other pose is 2e-3 below the winner in the oracle
    gap = pose_gap(oracle.cc_table(pn, rn, g))
    n_pose = check_pose(res, want, gap, 2e-3, min_decided=N // 4)
    # the reported CC is the FP32 re-score of the chosen candidate: equal to
    # the oracle's value of that same candidate to FP32 accuracy
    qhat, _ = oracle.reference_polar(rn, g)
    for n in range(N):
        a = (256 - res["psi"][n]) % 256
        v = oracle.candidate_cc(pn[n], qhat[res["ref"][n]], g, res["shift_x"][n], res["shift_y"][n],
                                res["mirror"][n], a)
        assert abs(res["cc"][n] - v) <= 1e-5 * abs(v), (n, res["cc"][n], v)
    agree = int(agreement(res, want).sum())
    log(f"  max rel CC err {err:.2e}; argmax agreement {agree}/{N}; decided by the top-two gap {frac:.3f}, "
        f"by pose {n_pose}/{N}")
    # with the default FP32 re-ranking of the 4 best rows the 16-bit forms
    # pick the oracle's exact winner for nearly every particle
    assert agree >= 0.9 * N, f"argmax agreement {agree}/{N}"


def test_align_mirror_off_normalize_off_no_shift(ctx):
    log("align fp32 mirror=0 normalize=0 T=0, K=1 and K=9")
    for K in (1, 9):
        L, T, N = 48, 0, 7
        refs, parts, _ = make_case(L, K, T, N, 0.2, 31 + K, mirror=False)
        ctx.load_refs(7, refs, r_min=2, r_max=20, shift_max=T, mirror=False, normalize=False)
        res = ctx.align(7, parts).to_numpy()
        want = oracle.align(parts.cpu().numpy(), refs.cpu().numpy(),
                            geom(L, 20, T, mirror=False, normalize=False, r_min=2))
        check_align(res, want, 1e-5)
        assert np.all(res["mirror"] == 0)


def test_noise_free_planted_recovery(ctx):
    log("noise-free planted parameters")
    L, K, T, N = 64, 6, 2, 40
    refs, parts, truth = make_case(L, K, T, N, None, 32, rho=28.0, n_phi_grid=256)
    ctx.load_refs(8, refs, r_min=1, r_max=30, shift_max=T)
    res = ctx.align(8, parts).to_numpy()
    np.testing.assert_array_equal(res["ref"], truth.ref)
    np.testing.assert_array_equal(res["shift_x"], truth.shift_x)
    np.testing.assert_array_equal(res["shift_y"], truth.shift_y)
    np.testing.assert_array_equal(res["mirror"], truth.mirror)
    np.testing.assert_array_equal(res["psi"], truth.psi_index)


def test_averages_match_oracle_given_identical_parameters(ctx):
    log("class averages")
    from paper_2011_05755_amd import mra
    L, K, T, N = 64, 10, 2, 300
    refs, parts, truth = make_case(L, K, T, N, 0.1, 33)
    ctx.load_refs(9, refs, r_min=1, r_max=30, shift_max=T)
    rng = np.random.default_rng(3)
    ref = rng.integers(0, K - 1, N)      # class K-1 stays empty
    params = dict(ref=ref, shift_x=rng.integers(-T, T + 1, N), shift_y=rng.integers(-T, T + 1, N),
                  psi=rng.integers(0, 256, N), mirror=rng.integers(0, 2, N))
    res = mra.AlignResult.empty(N, DEV)
    for key, val in params.items():
        getattr(res, key).copy_(torch.as_tensor(val, dtype=torch.int32))
    avg = refs.clone()
    counts = ctx.update_averages(9, parts, res, avg)
    torch.cuda.synchronize()
    want, cnt = oracle.averages(parts.cpu().numpy(), params, refs.cpu().numpy(), geom(L, 30, T))
    np.testing.assert_array_equal(counts.cpu().numpy(), cnt)
    got = avg.cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-5, err
    assert torch.equal(avg[K - 1], refs[K - 1])
    avg2 = refs.clone()
    ctx.update_averages(9, parts, res, avg2)
    assert torch.equal(avg, avg2)   # fixed summation order


@pytest.mark.parametrize("K", [300, 2100])
def test_averages_many_classes_and_blocks(ctx, K):
    """More than one 1024-particle block of the class scatter, and K on both
    sides of the scatter's LDS limit (16 K ints: one workgroup per block up
    to K = 2048, one wave per block above)."""
    log(f"class averages, K={K}")
    from paper_2011_05755_amd import mra
    L, T, N = 16, 1, 2500
    refs, parts, _ = make_case(L, K, T, N, 0.1, 34)
    ctx.load_refs(10, refs, r_min=1, r_max=L // 2 - 2, shift_max=T)
    rng = np.random.default_rng(4)
    ref = rng.integers(0, K, N)
    params = dict(ref=ref, shift_x=rng.integers(-T, T + 1, N), shift_y=rng.integers(-T, T + 1, N),
                  psi=rng.integers(0, 256, N), mirror=rng.integers(0, 2, N))
    res = mra.AlignResult.empty(N, DEV)
    for key, val in params.items():
        getattr(res, key).copy_(torch.as_tensor(val, dtype=torch.int32))
    avg = refs.clone()
    counts = ctx.update_averages(10, parts, res, avg)
    torch.cuda.synchronize()
    want, cnt = oracle.averages(parts.cpu().numpy(), params, refs.cpu().numpy(), geom(L, L // 2 - 2, T))
    np.testing.assert_array_equal(counts.cpu().numpy(), cnt)
    err = np.abs(avg.cpu().numpy() - want).max() / np.abs(want).max()
    assert err <= 1e-5, err
    ctx.unload_refs(10)


def test_batch_equals_individual_runs_and_runs_are_deterministic(ctx):
    log("align_batch vs individual")
    from paper_2011_05755_amd import mra
    cases = [(64, 10, 2, 17, 40), (48, 5, 1, 9, 41), (76, 12, 3, 11, 42)]
    stacks, singles = [], []
    for i, (L, K, T, N, seed) in enumerate(cases):
        refs, parts, _ = make_case(L, K, T, N, 0.1, seed)
        rid = 20 + i
        ctx.load_refs(rid, refs, r_min=1, r_max=L // 2 - 2, shift_max=T)
        singles.append(ctx.align(rid, parts).to_numpy())
        out = mra.AlignResult.empty(N, DEV)
        stacks.append((rid, parts, -1, out))
    ctx.align_batch(stacks)
    torch.cuda.synchronize()
    for (rid, parts, _, out), single in zip(stacks, singles):
        got = out.to_numpy()
        for key in single:
            np.testing.assert_array_equal(got[key], single[key])
        again = ctx.align(rid, parts).to_numpy()
        for key in single:
            np.testing.assert_array_equal(again[key], single[key])


def test_error_codes(ctx):
    log("error codes")
    from paper_2011_05755_amd import mra
    refs, parts, _ = make_case(32, 2, 1, 2, 0.1, 43)
    with pytest.raises(mra.MRAError) as e:
        ctx.load_refs(30, refs, r_min=0, r_max=10, shift_max=1)
    assert e.value.code == mra.MRA_E_INVAL
    with pytest.raises(mra.MRAError) as e:
        ctx.load_refs(30, refs, r_min=1, r_max=10, shift_max=1, n_phi=128)
    assert e.value.code == mra.MRA_E_INVAL
    zero = torch.zeros_like(refs)
    with pytest.raises(mra.MRAError) as e:
        ctx.load_refs(31, zero, r_min=1, r_max=10, shift_max=1)
    assert e.value.code == mra.MRA_E_DEGENERATE
    ctx.load_refs(32, refs, r_min=1, r_max=10, shift_max=1)
    ctx.unload_refs(32)
    lib = mra.load_library()
    out = mra.AlignResult.empty(2, DEV)
    r = out.c_struct()
    import ctypes
    assert lib.mra_align(ctx._h, 32, ctypes.c_void_p(parts.data_ptr()), 2, ctypes.byref(r)) == mra.MRA_E_NOREF
    ctx.load_refs(33, refs, r_min=1, r_max=10, shift_max=1)
    empty = torch.empty((0, 32, 32), device=DEV)
    ctx.align(33, empty, out=mra.AlignResult.empty(0, DEV))    # N = 0 is a no-op
    small = mra.Context(0, workspace_cap=1 << 16)     # 64 KiB: less than one row tile of the operand (98 KiB)
    with pytest.raises(mra.MRAError) as e:            # reference preparation or the alignment runs out
        small.load_refs(0, refs, r_min=1, r_max=10, shift_max=1)
        small.align(0, parts)
    assert e.value.code == mra.MRA_E_NOMEM
    small.close()
    bad = mra.AlignResult.empty(2, DEV)
    bad.cc = None
    r = bad.c_struct()
    assert lib.mra_align(ctx._h, 33, ctypes.c_void_p(parts.data_ptr()), 2, ctypes.byref(r)) == mra.MRA_E_INVAL
