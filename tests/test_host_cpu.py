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
