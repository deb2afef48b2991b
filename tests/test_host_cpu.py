"""Host-side checks that need no GPU: the C ABI library loads and exports
every symbol the header declares, error paths return codes, and the
register-level FFT building blocks pass their CPU check."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mra.h")


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (binds the HIP runtime the way the binding does)
    from paper_2011_05755_amd import mra

    if not os.path.exists(mra.LIB_PATH):
        from paper_2011_05755_amd import build

        build.build()
    return mra.load_library()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mra_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2011_05755_amd import mra
    assert set(mra.EXPORTS) == set(syms)


def test_strerror_and_null_context(lib):
    assert lib.mra_strerror(0) == b"ok"
    assert lib.mra_strerror(-5).startswith(b"degenerate")
    assert lib.mra_strerror(-99) == b"unknown error"
    assert lib.mra_last_error(None) == b"NULL context"
    assert lib.mra_align(None, 0, None, 0, None) == -1
    assert lib.mra_destroy(None) == -1


def test_create_without_a_device_returns_an_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.mra_create(ctypes.byref(h), 0, None, 0) == -1
    assert not h.value


def test_register_fft_building_blocks_on_cpu(tmp_path):
    exe = tmp_path / "fft_check"
    src = os.path.join(ROOT, "tests", "cpu", "fft_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), src], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"


def test_geometry_validation_needs_no_device(lib):
    """mra_check_geom: the ranges of mra_geom, and the int32 flat candidate
    index (K * M * (2T+1)^2 * n_phi below 2^31)."""
    from paper_2011_05755_amd import mra
    ok = dict(L=76, r_min=1, r_max=35, shift_max=3, K=100)
    assert mra.check_geom(**ok) == mra.MRA_OK
    assert mra.check_geom(L=160, r_min=1, r_max=64, shift_max=8, K=3, precision="bf16", rescore_rows=8) == mra.MRA_OK
    for bad in (dict(n_phi=128), dict(r_min=0), dict(L=7), dict(L=161), dict(r_max=65), dict(shift_max=9),
                dict(K=0), dict(rescore_rows=9), dict(r_min=36)):
        assert mra.check_geom(**{**ok, **bad}) == mra.MRA_E_INVAL, bad
    # the largest reference counts whose candidate index fits an int32
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=14513) == mra.MRA_OK
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=14514) == mra.MRA_E_INVAL
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=15000) == mra.MRA_E_INVAL
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=15000, mirror=False) == mra.MRA_OK
    assert mra.check_geom(L=76, r_min=1, r_max=35, shift_max=3, K=85598) == mra.MRA_OK
    assert mra.check_geom(L=76, r_min=1, r_max=35, shift_max=3, K=85599) == mra.MRA_E_INVAL
    # a per-call search range is checked the same way
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=3, K=15000, search_shift=8) == mra.MRA_E_INVAL
    assert lib.mra_check_geom(None, 10, -1) == mra.MRA_E_INVAL


def test_result_arrays_are_checked_before_the_call(lib):
    """The binding rejects result tensors the kernels would write out of
    bounds or misread: short, wrong dtype, strided, on another device, or a
    required field missing (cc2, flat_index, psi_frac are optional)."""
    import torch
    from paper_2011_05755_amd import mra
    cpu = torch.device("cpu")
    out = mra.AlignResult.empty(10, cpu, with_cc2=True)
    mra._check_result(out, 10, cpu)
    mra._check_result(out, 7, cpu)                       # longer than N is fine
    with pytest.raises(ValueError, match="length >= 11"):
        mra._check_result(out, 11, cpu)
    for field, bad in (("ref", torch.zeros(10, dtype=torch.int64)), ("cc", torch.zeros(10, dtype=torch.float64)),
                       ("psi", torch.zeros(20, dtype=torch.int32)[::2]), ("cc2", torch.zeros(9)),
                       ("flat_index", torch.zeros(10, 1, dtype=torch.int32))):
        o = mra.AlignResult.empty(10, cpu, with_cc2=True)
        setattr(o, field, bad)
        with pytest.raises(ValueError, match=field):
            mra._check_result(o, 10, cpu)
    o = mra.AlignResult.empty(10, cpu)
    o.mirror = None
    with pytest.raises(ValueError, match="mirror is required"):
        mra._check_result(o, 10, cpu)
    with pytest.raises(ValueError, match="on cuda:0"):
        mra._check_result(mra.AlignResult.empty(10, cpu), 10, torch.device("cuda", 0))
    o = mra.AlignResult.empty(10, cpu)
    o.cc = None                                           # the average update reads no CC
    mra._check_result(o, 10, cpu, required=mra._REQUIRED[:5])
