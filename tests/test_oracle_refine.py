"""Pins of the oracle's sub-step angle refinement (a parabola through the CC
at the winning angle step and its two neighbours).

Noise-free particles rotated by angles off the 256-step grid: the refined
angle must land within 0.02 steps of the true rotation (the integer search
is off by up to half a step), and particles rotated exactly onto the grid
keep their angle to within a few hundredths of a step.
"""

import math

import numpy as np

import oracle
from paper_2011_05755_amd import synth

L, K, T = 64, 5, 2


def circ(x):
    return np.abs((np.asarray(x) + 128.0) % 256.0 - 128.0)


def setup(seed, n_phi_grid=None):
    blobs = synth.make_blobs(K, L, seed=(seed, 0), rho_max=28)
    refs = synth.render_refs(blobs).numpy()
    parts, truth = synth.make_particles(blobs, 24, T, None, seed=(seed, 1), n_phi_grid=n_phi_grid)
    g = oracle.Geometry(L=L, r_min=1, r_max=30, n_phi=256, shift_max=T)
    return refs, parts.numpy(), truth, g


def test_refined_angle_recovers_off_grid_rotations():
    refs, parts, truth, g = setup(200)
    res = oracle.align(parts, refs, g)
    np.testing.assert_array_equal(res["ref"], truth.ref)
    frac = oracle.refine_psi(parts, refs, g, res)
    true_steps = (truth.alpha * 256.0 / (2.0 * math.pi)) % 256.0
    err_int, err_frac = circ(res["psi"] - true_steps), circ(frac - true_steps)
    assert err_int.max() <= 0.5 + 1e-9
    assert err_frac.max() <= 0.02, err_frac.max()
    assert err_frac.mean() < 0.1 * err_int.mean()


def test_on_grid_rotations_stay_on_the_grid():
    refs, parts, truth, g = setup(201, n_phi_grid=256)
    res = oracle.align(parts, refs, g)
    frac = oracle.refine_psi(parts, refs, g, res)
    np.testing.assert_array_equal(res["psi"], truth.psi_index)
    assert circ(frac - res["psi"]).max() <= 0.05
