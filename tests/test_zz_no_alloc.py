"""mra_align_noalloc (the alignment entry point for callers that cannot
allocate) through the C ABI: on two calls in a row, the second with fewer
particles, its results equal mra_align's on the same input bit for bit (the
same kernels; only where the chunk buffers live differs), for every
contraction precision with the runner-up pass, and for the single-reference
kernel; the calls leave the device's free memory unchanged."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2011_05755_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def log(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(DEV)[0]


@pytest.mark.parametrize("precision,K", [("fp32", 24), ("bf16", 24), ("fp16", 24), ("fp32", 1)])
def test_noalloc_equals_align_on_two_calls(precision, K):
    from paper_2011_05755_amd import mra
    L, T, r_max = 76, 3, 35
    log(f"{precision} K={K} L={L} T={T} rings 1..{r_max}")
    blobs = synth.make_blobs(K, L, seed=(90, K), rho_max=28.0)
    refs = synth.render_refs(blobs).to(DEV)
    # 300 particles need three chunks of the 256 MiB scratch at this geometry
    parts, _ = synth.make_particles(blobs, 300, T, 0.05, seed=(90, 1), device=DEV)
    lib = mra.load_library()
    plain = mra.Context(0)
    plain.load_refs(0, refs, r_min=1, r_max=r_max, shift_max=T, precision=precision)
    ctx = mra.Context(0)
    ctx.load_refs(0, refs, r_min=1, r_max=r_max, shift_max=T, precision=precision)
    xs = {300: parts[:300], 37: parts[200:237].contiguous()}
    wants = {n: plain.align(0, x, with_cc2=True).to_numpy() for n, x in xs.items()}
    outs = {n: mra.AlignResult.empty(n, DEV, with_cc2=True) for n in (300, 37, 5)}
    # first launch of every kernel on this context (code objects load)
    c = outs[5].c_struct()
    assert lib.mra_align_noalloc(ctx._h, 0, ctypes.c_void_p(parts.data_ptr()), 5, ctypes.byref(c)) == mra.MRA_OK
    before = free_bytes()
    for n, x in xs.items():
        c = outs[n].c_struct()
        rc = lib.mra_align_noalloc(ctx._h, 0, ctypes.c_void_p(x.data_ptr()), n, ctypes.byref(c))
        assert rc == mra.MRA_OK, lib.mra_last_error(ctx._h)
        assert free_bytes() == before, "mra_align_noalloc changed the device's free memory"
        got = outs[n].to_numpy()
        for key in wants[n]:
            np.testing.assert_array_equal(got[key], wants[n][key], err_msg=f"N={n}: {key}")
        log(f"  N={n}: equal to mra_align")
    # errors: unknown refset, NULL result arrays
    assert lib.mra_align_noalloc(ctx._h, 9, ctypes.c_void_p(parts.data_ptr()), 5, ctypes.byref(c)) == mra.MRA_E_NOREF
    assert lib.mra_align_noalloc(ctx._h, 0, ctypes.c_void_p(parts.data_ptr()), 5, None) == mra.MRA_E_INVAL
    ctx.close()
    plain.close()
