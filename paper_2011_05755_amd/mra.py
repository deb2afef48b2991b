"""Thin ctypes binding over libmra.so (C ABI declared in include/mra.h).

Argument marshalling only: every step of the alignment runs in the HIP
kernels of libmra.so.  PyTorch provides device memory and the stream; the
library is bound to torch's HIP runtime by importing torch first.  If the
library has not been built, every call fails loudly.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmra.so")

MRA_OK, MRA_E_INVAL, MRA_E_NOREF, MRA_E_NOMEM, MRA_E_DEVICE, MRA_E_DEGENERATE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
# 16-bit forms: rows whose winners are re-ranked in FP32 unless a caller says
# otherwise (on the 100k-particle workload it lifts BF16's agreement with the
# FP32 form's parameters from 96.2 % to 99.99 % for 2 % more time)
DEFAULT_RESCORE_ROWS = 4

EXPORTS = (
    "mra_create", "mra_destroy", "mra_load_refs", "mra_check_geom", "mra_unload_refs", "mra_refset_info",
    "mra_align", "mra_align_noalloc", "mra_update_averages", "mra_classify", "mra_rfa", "mra_align_batch", "mra_set_tuning", "mra_get_tuning",
    "mra_debug_polar",
    "mra_debug_spectra", "mra_debug_cctable", "mra_debug_refs", "mra_profile", "mra_profile_read",
    "mra_last_error", "mra_strerror",
)


class Geom(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("L", "r_min", "r_max", "n_phi", "shift_max", "mirror", "precision", "normalize", "rescore_rows")]


class Result(ctypes.Structure):
    _fields_ = [("ref", ctypes.c_void_p), ("shift_x", ctypes.c_void_p), ("shift_y", ctypes.c_void_p),
                ("psi", ctypes.c_void_p), ("mirror", ctypes.c_void_p), ("cc", ctypes.c_void_p),
                ("cc2", ctypes.c_void_p), ("flat_index", ctypes.c_void_p), ("psi_frac", ctypes.c_void_p)]


class Stack(ctypes.Structure):
    _fields_ = [("refset_id", ctypes.c_int32), ("parts", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("shift_max", ctypes.c_int32), ("out", Result)]


class Tuning(ctypes.Structure):
    _fields_ = [("corr_variant", ctypes.c_int32), ("chunk_particles", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("run_tiles", ctypes.c_int32)]


class MRAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libmra.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_05755_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "mra_create": [ctypes.POINTER(vp), ctypes.c_int, vp, u64],
        "mra_destroy": [vp],
        "mra_load_refs": [vp, i32, vp, i32, ctypes.POINTER(Geom)],
        "mra_check_geom": [ctypes.POINTER(Geom), i32, i32],
        "mra_unload_refs": [vp, i32],
        "mra_refset_info": [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(Geom)],
        "mra_align": [vp, i32, vp, i64, ctypes.POINTER(Result)],
        "mra_align_noalloc": [vp, i32, vp, i64, ctypes.POINTER(Result)],
        "mra_update_averages": [vp, i32, vp, i64, ctypes.POINTER(Result), vp, vp],
        "mra_classify": [vp, i32, ctypes.POINTER(Geom), vp, i64, vp, i32, i32, ctypes.c_double,
                         ctypes.POINTER(Result), vp, ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "mra_rfa": [vp, i32, ctypes.POINTER(Geom), vp, i64, vp, i32, i32, ctypes.c_double, ctypes.POINTER(Result),
                    ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "mra_align_batch": [vp, ctypes.POINTER(Stack), i32],
        "mra_set_tuning": [vp, i32, ctypes.POINTER(Tuning)],
        "mra_get_tuning": [vp, i32, ctypes.POINTER(Tuning)],
        "mra_debug_polar": [vp, i32, vp, i64, vp],
        "mra_debug_spectra": [vp, i32, vp, i64, vp],
        "mra_debug_cctable": [vp, i32, vp, i64, vp],
        "mra_debug_refs": [vp, i32, vp, vp],
        "mra_profile": [vp, ctypes.c_int],
        "mra_profile_read": [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mra_last_error.argtypes = [vp]
    lib.mra_last_error.restype = ctypes.c_char_p
    lib.mra_strerror.argtypes = [ctypes.c_int]
    lib.mra_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class AlignResult:
    """Per-particle alignment parameters (device tensors of length N)."""

    ref: torch.Tensor
    shift_x: torch.Tensor
    shift_y: torch.Tensor
    psi: torch.Tensor
    mirror: torch.Tensor
    cc: torch.Tensor
    cc2: torch.Tensor | None = None
    flat_index: torch.Tensor | None = None
    psi_frac: torch.Tensor | None = None

    @classmethod
    def empty(cls, N: int, device, with_cc2=False, with_flat=True, with_psi_frac=False):
        i = dict(dtype=torch.int32, device=device)
        f = dict(dtype=torch.float32, device=device)
        return cls(ref=torch.empty(N, **i), shift_x=torch.empty(N, **i), shift_y=torch.empty(N, **i),
                   psi=torch.empty(N, **i), mirror=torch.empty(N, **i),
                   cc=torch.empty(N, **f),
                   cc2=torch.empty(N, **f) if with_cc2 else None,
                   flat_index=torch.empty(N, **i) if with_flat else None,
                   psi_frac=torch.empty(N, **f) if with_psi_frac else None)

    def c_struct(self) -> Result:
        return Result(*(_ptr(getattr(self, f)) for f in
                        ("ref", "shift_x", "shift_y", "psi", "mirror", "cc", "cc2", "flat_index", "psi_frac")))

    def narrow(self, lo: int, n: int) -> "AlignResult":
        return AlignResult(**{f.name: (None if getattr(self, f.name) is None else getattr(self, f.name)[lo:lo + n])
                              for f in dataclasses.fields(self)})

    def to_numpy(self) -> dict:
        return {f.name: getattr(self, f.name).cpu().numpy() for f in dataclasses.fields(self)
                if getattr(self, f.name) is not None}


@dataclasses.dataclass
class Refset:
    id: int
    K: int
    L: int
    r_min: int
    r_max: int
    n_phi: int
    shift_max: int
    mirror: int
    precision: str
    normalize: int

    @property
    def n_rings(self):
        return self.r_max - self.r_min + 1


_RESULT_DTYPES = dict(ref=torch.int32, shift_x=torch.int32, shift_y=torch.int32, psi=torch.int32,
                      mirror=torch.int32, cc=torch.float32, cc2=torch.float32, flat_index=torch.int32,
                      psi_frac=torch.float32)
_REQUIRED = ("ref", "shift_x", "shift_y", "psi", "mirror", "cc")


def _check_result(out: "AlignResult", N: int, device: torch.device, name: str = "out",
                  required=_REQUIRED):
    """Every array the library will write (or read) must be a contiguous 1-D
    tensor of the field's dtype with at least N elements on `device`: the C
    ABI takes raw pointers and cannot check lengths itself."""
    for field, dtype in _RESULT_DTYPES.items():
        t = getattr(out, field)
        if t is None:
            if field in required:
                raise ValueError(f"{name}.{field} is required")
            continue
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.dim() != 1 or t.shape[0] < N \
                or not t.is_contiguous() or t.device != device:
            raise ValueError(f"{name}.{field} must be a contiguous 1-D {dtype} tensor of length >= {N} "
                             f"on {device}")


def check_geom(L: int, r_min: int, r_max: int, shift_max: int, K: int, n_phi: int = 256, mirror: bool = True,
               precision: str = "fp32", normalize: bool = True, rescore_rows: int = 0,
               search_shift: int = -1) -> int:
    """mra_check_geom: MRA_OK when the library accepts the geometry for K
    references (searched at search_shift, or shift_max when negative),
    else the error code.  Needs no device."""
    lib = load_library()
    g = Geom(L, r_min, r_max, n_phi, shift_max, int(mirror), PRECISIONS[precision], int(normalize), rescore_rows)
    return lib.mra_check_geom(ctypes.byref(g), K, search_shift)


def _check_images(x: torch.Tensor, L: int, name: str):
    if not (x.is_cuda and x.dtype == torch.float32 and x.dim() == 3 and x.shape[1] == L
            and x.shape[2] == L and x.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor [N, {L}, {L}]")


class Context:
    """One libmra context bound to a device and a stream (default: torch's
    current stream on that device)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, workspace_cap: int = 0):
        self.lib = load_library()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        rc = self.lib.mra_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.c_uint64(workspace_cap))
        if rc != MRA_OK:
            raise MRAError(rc, "mra_create failed: " + self.lib.mra_strerror(rc).decode())
        self._h = h
        self.refsets: dict[int, Refset] = {}

    def _check(self, rc: int):
        if rc != MRA_OK:
            raise MRAError(rc, self.lib.mra_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mra_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- reference sets ----
    def load_refs(self, refset_id: int, refs: torch.Tensor, r_min: int, r_max: int, shift_max: int,
                  n_phi: int = 256, mirror: bool = True, precision: str = "fp32", normalize: bool = True,
                  rescore_rows: int | None = None) -> Refset:
        """rescore_rows (16-bit forms): re-rank the winners of that many best
        rows (and their +-1 angle neighbours) in FP32; 0/1: the winner only.
        None: DEFAULT_RESCORE_ROWS for BF16/FP16."""
        if rescore_rows is None:
            rescore_rows = DEFAULT_RESCORE_ROWS if precision != "fp32" else 0
        L = refs.shape[-1]
        _check_images(refs, L, "refs")
        g = Geom(L, r_min, r_max, n_phi, shift_max, int(mirror), PRECISIONS[precision], int(normalize),
                 rescore_rows)
        self._check(self.lib.mra_load_refs(self._h, refset_id, _ptr(refs), refs.shape[0], ctypes.byref(g)))
        rs = Refset(refset_id, refs.shape[0], L, r_min, r_max, n_phi, shift_max, int(mirror), precision,
                    int(normalize))
        self.refsets[refset_id] = rs
        return rs

    def unload_refs(self, refset_id: int):
        self._check(self.lib.mra_unload_refs(self._h, refset_id))
        self.refsets.pop(refset_id, None)

    # ---- alignment ----
    def align(self, refset_id: int, parts: torch.Tensor, out: AlignResult | None = None,
              with_cc2: bool = False, with_psi_frac: bool = False) -> AlignResult:
        rs = self.refsets[refset_id]
        _check_images(parts, rs.L, "parts")
        N = parts.shape[0]
        if out is None:
            out = AlignResult.empty(N, parts.device, with_cc2=with_cc2, with_psi_frac=with_psi_frac)
        _check_result(out, N, parts.device)
        res = out.c_struct()
        self._check(self.lib.mra_align(self._h, refset_id, _ptr(parts), N, ctypes.byref(res)))
        return out

    def align_noalloc(self, refset_id: int, parts: torch.Tensor, out: AlignResult) -> AlignResult:
        """mra_align_noalloc: as align, with the library's fixed device
        scratch instead of its workspace; `out` must be given (nothing is
        allocated by this call)."""
        rs = self.refsets[refset_id]
        _check_images(parts, rs.L, "parts")
        N = parts.shape[0]
        _check_result(out, N, parts.device)
        res = out.c_struct()
        self._check(self.lib.mra_align_noalloc(self._h, refset_id, _ptr(parts), N, ctypes.byref(res)))
        return out

    def align_batch(self, stacks: list[tuple[int, torch.Tensor, int, AlignResult]]):
        """stacks: list of (refset_id, parts, shift_max (-1: refset's), out)."""
        arr = (Stack * len(stacks))()
        for i, (rid, parts, T, out) in enumerate(stacks):
            _check_images(parts, self.refsets[rid].L, "parts")
            _check_result(out, parts.shape[0], parts.device, name=f"stacks[{i}].out")
            arr[i] = Stack(rid, parts.data_ptr(), parts.shape[0], T, out.c_struct())
        self._check(self.lib.mra_align_batch(self._h, arr, len(stacks)))

    def update_averages(self, refset_id: int, parts: torch.Tensor, params: AlignResult,
                        averages: torch.Tensor) -> torch.Tensor:
        """In place: averages [K, L, L] (previous Y in, Y' out).  Returns counts [K]."""
        rs = self.refsets[refset_id]
        _check_images(parts, rs.L, "parts")
        _check_images(averages, rs.L, "averages")
        if averages.shape[0] != rs.K:
            raise ValueError("averages must have K images")
        _check_result(params, parts.shape[0], parts.device, name="params", required=_REQUIRED[:5])
        counts = torch.empty(rs.K, dtype=torch.int32, device=parts.device)
        p = params.c_struct()
        self._check(self.lib.mra_update_averages(self._h, refset_id, _ptr(parts), parts.shape[0],
                                                 ctypes.byref(p), _ptr(averages), _ptr(counts)))
        return counts

    def classify(self, refset_id: int, parts: torch.Tensor, averages: torch.Tensor, r_min: int, r_max: int,
                 shift_max: int, max_iter: int = 20, max_changed_frac: float = 0.005, n_phi: int = 256,
                 mirror: bool = True, precision: str = "fp32", normalize: bool = True,
                 out: AlignResult | None = None, with_cc2: bool = False, rescore_rows: int | None = None):
        """Iterative MRA (mra_classify): averages [K, L, L] in place (initial
        references in, final averages out).  Returns (params of the last
        pass, counts [K], passes run, changed-per-pass list)."""
        L = averages.shape[-1]
        _check_images(parts, L, "parts")
        _check_images(averages, L, "averages")
        N, K = parts.shape[0], averages.shape[0]
        if out is None:
            out = AlignResult.empty(N, parts.device, with_cc2=with_cc2)
        _check_result(out, N, parts.device)
        counts = torch.empty(K, dtype=torch.int32, device=parts.device)
        if rescore_rows is None:
            rescore_rows = DEFAULT_RESCORE_ROWS if precision != "fp32" else 0
        g = Geom(L, r_min, r_max, n_phi, shift_max, int(mirror), PRECISIONS[precision], int(normalize),
                 rescore_rows)
        res = out.c_struct()
        n_iter = ctypes.c_int32()
        changed = (ctypes.c_int64 * max(1, max_iter))()
        self._check(self.lib.mra_classify(self._h, refset_id, ctypes.byref(g), _ptr(parts), N, _ptr(averages), K,
                                          max_iter, max_changed_frac, ctypes.byref(res), _ptr(counts),
                                          ctypes.byref(n_iter), changed))
        self.refsets[refset_id] = Refset(refset_id, K, L, r_min, r_max, n_phi, shift_max, int(mirror), precision,
                                         int(normalize))
        return out, counts, n_iter.value, list(changed[:n_iter.value])

    def rfa(self, refset_id: int, parts: torch.Tensor, r_min: int, r_max: int, shift_max: int,
            average: torch.Tensor | None = None, max_iter: int = 10, max_changed_frac: float = 0.0,
            n_phi: int = 256, mirror: bool = True, normalize: bool = True, out: AlignResult | None = None,
            with_cc2: bool = True):
        """Reference-free alignment (mra_rfa).  average [L, L]: the starting
        reference, updated in place; None starts from the plain mean.
        Returns (params of the last pass, average, passes run, changed-per-pass list)."""
        L = parts.shape[-1]
        _check_images(parts, L, "parts")
        N = parts.shape[0]
        start_from_mean = average is None
        if average is None:
            average = torch.empty((L, L), dtype=torch.float32, device=parts.device)
        if not (average.is_cuda and average.dtype == torch.float32 and tuple(average.shape) == (L, L)
                and average.is_contiguous()):
            raise ValueError(f"average must be a contiguous float32 CUDA tensor [{L}, {L}]")
        if out is None:
            out = AlignResult.empty(N, parts.device, with_cc2=with_cc2)
        _check_result(out, N, parts.device)
        g = Geom(L, r_min, r_max, n_phi, shift_max, int(mirror), 0, int(normalize))
        res = out.c_struct()
        n_iter = ctypes.c_int32()
        changed = (ctypes.c_int64 * max(1, max_iter))()
        self._check(self.lib.mra_rfa(self._h, refset_id, ctypes.byref(g), _ptr(parts), N, _ptr(average),
                                     int(start_from_mean), max_iter, max_changed_frac, ctypes.byref(res),
                                     ctypes.byref(n_iter), changed))
        self.refsets[refset_id] = Refset(refset_id, 1, L, r_min, r_max, n_phi, shift_max, int(mirror), "fp32",
                                         int(normalize))
        return out, average, n_iter.value, list(changed[:n_iter.value])

    # ---- tile configuration (see include/mra.h, mra_tuning) ----
    def set_tuning(self, refset_id: int, corr_variant: int = -1, chunk_particles: int = 0, prune: int = -1,
                   run_tiles: int = 0):
        t = Tuning(corr_variant, chunk_particles, prune, run_tiles)
        self._check(self.lib.mra_set_tuning(self._h, refset_id, ctypes.byref(t)))

    def get_tuning(self, refset_id: int) -> tuple[int, int]:
        """(corr_variant, chunk_particles) of a refset."""
        t = Tuning()
        self._check(self.lib.mra_get_tuning(self._h, refset_id, ctypes.byref(t)))
        return t.corr_variant, t.chunk_particles

    def get_prune(self, refset_id: int) -> bool:
        t = Tuning()
        self._check(self.lib.mra_get_tuning(self._h, refset_id, ctypes.byref(t)))
        return bool(t.prune)

    # ---- kernel timing ----
    def profile(self, enable: bool):
        self._check(self.lib.mra_profile(self._h, int(enable)))

    def profile_read(self, kernel: str) -> tuple[float, int]:
        """(summed device milliseconds, launches) of a kernel group since profile(True)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.mra_profile_read(self._h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ---- debug exports ----
    def debug_polar(self, refset_id: int, parts: torch.Tensor) -> torch.Tensor:
        rs = self.refsets[refset_id]
        S = (2 * rs.shift_max + 1) ** 2
        out = torch.empty((parts.shape[0], S, rs.n_rings, rs.n_phi), dtype=torch.float32, device=parts.device)
        self._check(self.lib.mra_debug_polar(self._h, refset_id, _ptr(parts), parts.shape[0], _ptr(out)))
        return out

    def debug_spectra(self, refset_id: int, parts: torch.Tensor) -> torch.Tensor:
        rs = self.refsets[refset_id]
        S = (2 * rs.shift_max + 1) ** 2
        out = torch.empty((parts.shape[0], S, rs.n_rings, rs.n_phi // 2 + 1, 2), dtype=torch.float32,
                          device=parts.device)
        self._check(self.lib.mra_debug_spectra(self._h, refset_id, _ptr(parts), parts.shape[0], _ptr(out)))
        return out

    def debug_cctable(self, refset_id: int, parts: torch.Tensor) -> torch.Tensor:
        rs = self.refsets[refset_id]
        S1 = 2 * rs.shift_max + 1
        M = 2 if rs.mirror else 1
        out = torch.empty((parts.shape[0], rs.K, M, S1, S1, rs.n_phi), dtype=torch.float32, device=parts.device)
        self._check(self.lib.mra_debug_cctable(self._h, refset_id, _ptr(parts), parts.shape[0], _ptr(out)))
        return out

    def debug_refs(self, refset_id: int):
        rs = self.refsets[refset_id]
        dev = torch.device("cuda", self.device)
        qhat = torch.empty((rs.K, rs.n_rings, rs.n_phi), dtype=torch.float32, device=dev)
        norm = torch.empty(rs.K, dtype=torch.float64, device=dev)
        self._check(self.lib.mra_debug_refs(self._h, refset_id, _ptr(qhat), _ptr(norm)))
        return qhat, norm
