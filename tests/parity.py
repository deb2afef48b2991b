"""Comparison rules between the HIP path and the FP64 oracle, shared by the
GPU tests (a helper module: pytest collects nothing from it).

The bar (one alignment pass, Algorithm 1):
  * relative CC error of the reported winner against the oracle's best:
    <= 1e-5 for FP32, <= 2e-3 for the BF16 / FP16 contractions;
  * the five parameters equal the oracle's wherever the oracle's own top-two
    gap (cc - cc2, cc2 over every other candidate) is at least tol * |cc|;
  * for the 16-bit forms, whose contraction rounding mostly decides between
    neighbouring angles of one pose (cc2 is then the adjacent angle and the
    rule above checks nothing), also: reference, shifts and mirror equal and
    psi within one step wherever the oracle's best candidate of any OTHER
    pose (reference, mirror, shift) is below the winner by tol * |cc|.
"""

from __future__ import annotations

import numpy as np

import oracle

KEYS = ("ref", "shift_x", "shift_y", "mirror", "psi")


def check_align(got, want, tol, cc_tol=None):
    """Returns (max relative CC error, fraction of decided particles)."""
    cc_tol = tol if cc_tol is None else cc_tol
    rel = np.abs(got["cc"] - want["cc"]) / np.abs(want["cc"])
    assert rel.max() <= cc_tol, f"max rel CC err {rel.max():.3g}"
    ok_gap = (want["cc"] - want["cc2"]) >= tol * np.abs(want["cc"])
    for key in KEYS:
        bad = np.nonzero((got[key] != want[key]) & ok_gap)[0]
        assert bad.size == 0, f"{key} differs at {bad[:10]}: got {got[key][bad[:5]]} want {want[key][bad[:5]]}"
    return rel.max(), ok_gap.mean()


def pose_gap(table: np.ndarray) -> np.ndarray:
    """Per particle of an oracle CC table [N, K, M, S1, S1, n_phi]: the best
    CC minus the best CC of every other pose (reference, mirror, shift)."""
    N, n_phi = table.shape[0], table.shape[-1]
    per_pose = table.reshape(N, -1, n_phi).max(axis=2)        # [N, poses]
    out = np.empty(N)
    for i in range(N):
        p = per_pose[i]
        best = int(np.argmax(p))
        out[i] = p[best] - np.delete(p, best).max() if p.size > 1 else np.inf
    return out


def check_pose(got, want, gap, tol, n_phi=256, min_decided=1):
    """Reference, shifts and mirror equal, psi within one step, wherever the
    oracle's gap to every other pose is at least tol * |cc|; at least
    `min_decided` particles must be decided that way (a check that compares
    nothing fails).  Returns the number of such particles."""
    decided = gap >= tol * np.abs(want["cc"])
    assert decided.sum() >= min_decided, f"only {decided.sum()} particles decided by pose"
    for key in ("ref", "shift_x", "shift_y", "mirror"):
        bad = np.nonzero((got[key] != want[key]) & decided)[0]
        assert bad.size == 0, f"pose {key} differs at {bad[:10]}"
    d = np.abs(((got["psi"] - want["psi"]) + n_phi // 2) % n_phi - n_phi // 2)
    bad = np.nonzero((d > 1) & decided)[0]
    assert bad.size == 0, f"psi more than one step off at {bad[:10]}: got {got['psi'][bad[:5]]} want {want['psi'][bad[:5]]}"
    return int(decided.sum())


def agreement(got, want) -> np.ndarray:
    return np.all([np.asarray(got[k]) == np.asarray(want[k]) for k in KEYS], axis=0)


def check_rescored_cc(got, parts: np.ndarray, qhat: np.ndarray, g, tol=1e-5):
    """16-bit forms report the FP32 re-score of the chosen candidate: it must
    equal the oracle's direct sum for that same candidate."""
    for n in range(parts.shape[0]):
        a = (g.n_phi - int(got["psi"][n])) % g.n_phi
        v = oracle.candidate_cc(parts[n], qhat[int(got["ref"][n])], g, int(got["shift_x"][n]),
                                int(got["shift_y"][n]), int(got["mirror"][n]), a)
        assert abs(got["cc"][n] - v) <= tol * abs(v), (n, got["cc"][n], v)
