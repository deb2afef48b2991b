"""Single-reference alignment (K = 1, the fused kernel) and reference-free
alignment (mra_rfa) on the GPU against the oracle.

The single-reference pass is held to the FP32 bar: CC within 1e-5 of the
oracle's (relative), parameters equal wherever the oracle's top-two gap is
at least that, cc2 within 1e-5 of |cc|.  The RFA loop is compared on cases
where every pass is decided (gap >= 3e-5 at every pass), so the HIP loop
must take the oracle's trajectory: same passes, same changed counts, same
final parameters, averages within 1e-5 of their largest value.  Inputs are
generated on the CPU and copied to the device.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-rfa] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_05755_amd import mra
    c = mra.Context(0)
    yield c
    c.close()


def one_class(L, T, N, snr, seed, n_phi_grid=None, mirror=True):
    blobs = synth.make_blobs(1, L, seed=(seed, 0), rho_max=L / 2 - 4)
    ref = synth.render_refs(blobs)
    parts, truth = synth.make_particles(blobs, N, T, snr, seed=(seed, 1), n_phi_grid=n_phi_grid, mirror=mirror)
    return ref, parts, truth


def check_pass(got, want, tol=1e-5):
    rel = np.abs(got["cc"] - want["cc"]) / np.abs(want["cc"])
    assert rel.max() <= tol, f"max rel CC err {rel.max():.3g}"
    rel2 = np.abs(got["cc2"] - want["cc2"]) / np.abs(want["cc"])
    assert rel2.max() <= tol, f"max rel cc2 err {rel2.max():.3g}"
    decided = (want["cc"] - want["cc2"]) >= tol * np.abs(want["cc"])
    for key in ("ref", "shift_x", "shift_y", "mirror", "psi", "flat_index"):
        bad = np.nonzero((got[key] != want[key]) & decided)[0]
        assert bad.size == 0, f"{key} differs at {bad[:10]}"
    return rel.max(), decided.mean()


@pytest.mark.parametrize("L,T,r_min,r_max,mirror,N,seed", [
    (64, 2, 1, 30, True, 37, 60),     # 25 shifts: four 8-row groups, the last one ragged
    (48, 0, 1, 20, True, 11, 61),     # one shift: seven idle rows in the group
    (76, 5, 3, 35, True, 9, 62),      # 121 shifts, 16 groups, rings from 3
    (32, 3, 1, 13, False, 21, 63),    # no mirror search
    (76, 3, 1, 35, True, 30, 64),     # the 100k workload's geometry
])
def test_single_reference_pass_matches_oracle(ctx, L, T, r_min, r_max, mirror, N, seed):
    log(f"K=1 pass L={L} T={T} rings {r_min}..{r_max} mirror={mirror} N={N}")
    from paper_2011_05755_amd import mra
    ref, parts, _ = one_class(L, T, N, 0.1, seed, mirror=mirror)
    g = oracle.Geometry(L=L, r_min=r_min, r_max=r_max, n_phi=256, shift_max=T, mirror=int(mirror))
    want = oracle.align(parts.numpy(), ref.numpy(), g)
    ctx.load_refs(70, ref.to(DEV), r_min=r_min, r_max=r_max, shift_max=T, mirror=mirror)
    out = ctx.align(70, parts.to(DEV), with_cc2=True)
    got = out.to_numpy()
    err, dec = check_pass(got, want)
    assert np.all(got["ref"] == 0)
    if not mirror:
        assert np.all(got["mirror"] == 0)
    # every precision runs the same FP32 kernel for one reference
    ctx.load_refs(71, ref.to(DEV), r_min=r_min, r_max=r_max, shift_max=T, mirror=mirror, precision="bf16")
    o16 = ctx.align(71, parts.to(DEV), out=mra.AlignResult.empty(N, DEV, with_cc2=True)).to_numpy()
    for key in got:
        np.testing.assert_array_equal(o16[key], got[key], err_msg=key)
    log(f"max rel cc err {err:.2e}, decided {dec:.2f}")


def test_planted_particles_are_recovered_with_one_reference(ctx):
    ref, parts, truth = one_class(64, 3, 24, None, 65, n_phi_grid=256)
    ctx.load_refs(72, ref.to(DEV), r_min=1, r_max=30, shift_max=3)
    got = ctx.align(72, parts.to(DEV)).to_numpy()
    np.testing.assert_array_equal(got["shift_x"], truth.shift_x)
    np.testing.assert_array_equal(got["shift_y"], truth.shift_y)
    np.testing.assert_array_equal(got["mirror"], truth.mirror)
    np.testing.assert_array_equal(got["psi"], truth.psi_index)


def test_single_reference_stacks_in_a_batch_equal_single_calls(ctx):
    from paper_2011_05755_amd import mra
    ref1, p1, _ = one_class(64, 2, 13, 0.1, 66)
    blobs = synth.make_blobs(6, 48, seed=(67, 0), rho_max=20)
    refs6 = synth.render_refs(blobs).to(DEV)
    p2 = synth.make_particles(blobs, 17, 2, 0.1, seed=(67, 1), device=DEV)[0]
    p1 = p1.to(DEV)
    ctx.load_refs(73, ref1.to(DEV), r_min=1, r_max=30, shift_max=2)
    ctx.load_refs(74, refs6, r_min=1, r_max=20, shift_max=2)
    o1, o2 = mra.AlignResult.empty(13, DEV), mra.AlignResult.empty(17, DEV)
    ctx.align_batch([(73, p1, -1, o1), (74, p2, -1, o2), (73, p1[:0], -1, mra.AlignResult.empty(0, DEV))])
    s1, s2 = ctx.align(73, p1), ctx.align(74, p2)
    for a, b in ((o1, s1), (o2, s2)):
        x, y = a.to_numpy(), b.to_numpy()
        for key in x:
            np.testing.assert_array_equal(x[key], y[key], err_msg=key)


def rfa_case(seed):
    L, T, N = 32, 2, 20
    blobs = synth.make_blobs(1, L, seed=(seed, 0), rho_max=12.0)
    parts = synth.make_particles(blobs, N, T, 0.2, seed=(seed, 1), n_phi_grid=256)[0].numpy()
    return parts, oracle.Geometry(L=L, r_min=1, r_max=13, n_phi=256, shift_max=T)


@pytest.mark.parametrize("seed,start", [(150, "mean"), (183, "mean"), (195, "p0"), (165, "p0")])
def test_rfa_follows_the_oracle(ctx, seed, start):
    log(f"rfa seed {seed} start {start}")
    parts, g = rfa_case(seed)
    N = parts.shape[0]
    init = None if start == "mean" else parts[0]
    want, Yw, nw, fw = oracle.rfa(parts, g, max_iter=8, init=init)
    avg = None if init is None else torch.as_tensor(init).to(DEV).contiguous()
    out, avg, n, changed = ctx.rfa(75, torch.as_tensor(parts).to(DEV), r_min=1, r_max=13, shift_max=2,
                                   average=avg, max_iter=8)
    got = out.to_numpy()
    assert n == nw and changed[0] == N and changed[1:] == [round(f * N) for f in fw], (n, changed, fw)
    for key in ("ref", "shift_x", "shift_y", "psi", "mirror", "flat_index"):
        np.testing.assert_array_equal(got[key], want[key], err_msg=key)
    assert (np.abs(got["cc"] - want["cc"]) / np.abs(want["cc"])).max() <= 1e-5
    err = np.abs(avg.cpu().numpy() - Yw).max() / np.abs(Yw).max()
    assert err <= 1e-5, err
    log(f"passes {n}, changed {changed}, average rel err {err:.2e}")


def test_rfa_from_the_true_reference_converges_at_once(ctx):
    ref, parts, truth = one_class(48, 2, 16, None, 68, n_phi_grid=256)
    out, avg, n, changed = ctx.rfa(76, parts.to(DEV), r_min=1, r_max=20, shift_max=2,
                                   average=ref[0].to(DEV).contiguous(), max_iter=5)
    got = out.to_numpy()
    assert n == 2 and changed == [16, 0]
    np.testing.assert_array_equal(got["psi"], truth.psi_index)
    np.testing.assert_array_equal(got["shift_x"], truth.shift_x)
    np.testing.assert_array_equal(got["mirror"], truth.mirror)


def test_rfa_argument_errors(ctx):
    from paper_2011_05755_amd import mra
    lib = mra.load_library()
    parts, _ = rfa_case(150)
    p = torch.as_tensor(parts).to(DEV)
    avg = torch.zeros((32, 32), dtype=torch.float32, device=DEV)
    out = mra.AlignResult.empty(20, DEV)
    g = mra.Geom(32, 1, 13, 256, 2, 1, 0, 1)
    n_iter = ctypes.c_int32()

    def call(n=20, max_iter=3, frac=0.0, a=avg):
        res = out.c_struct()
        return lib.mra_rfa(ctx._h, 77, ctypes.byref(g), mra._ptr(p), n, mra._ptr(a), 1, max_iter, frac,
                           ctypes.byref(res), ctypes.byref(n_iter), None)

    assert call(n=0) == mra.MRA_E_INVAL
    assert call(max_iter=0) == mra.MRA_E_INVAL
    assert call(frac=-0.1) == mra.MRA_E_INVAL
    assert call(a=None) == mra.MRA_E_INVAL
    assert call() == mra.MRA_OK and n_iter.value >= 1
