"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins catch each one.  Every mutation is undone by monkeypatch afterwards."""

import numpy as np
import pytest

import oracle
from oracle import mra_oracle

import test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_unit_ring_weights_are_caught(monkeypatch):
    monkeypatch.setattr(mra_oracle, "ring_weights", lambda g: np.ones(g.n_rings))
    assert _fails(pins.test_cc_of_linear_images_closed_form, 0, 0)


def test_reversed_lag_is_caught(monkeypatch):
    orig = mra_oracle.rolled_reference_matrix

    def reversed_lag(qhat, g):
        return orig(qhat[:, :, ::-1].copy(), g)   # reads q[-(j+a)] instead of q[j+a]

    monkeypatch.setattr(mra_oracle, "rolled_reference_matrix", reversed_lag)
    assert _fails(pins.test_cc_of_linear_images_closed_form, 0, 1)


def test_x_flip_mirror_is_caught(monkeypatch):
    def xflip(g, sx, sy, m):
        cx, cy = mra_oracle.centre(g.L)
        r = mra_oracle.ring_radii(g)[:, None]
        th = 2.0 * np.pi * np.arange(g.n_phi)[None, :] / g.n_phi
        return cx + sx + (1 - 2 * m) * r * np.cos(th), cy + sy + r * np.sin(th)

    monkeypatch.setattr(mra_oracle, "polar_positions", xflip)
    assert _fails(pins.test_linear_image_samples_closed_form, 1)
    assert _fails(pins.test_cc_of_linear_images_closed_form, 1, 1)


def test_half_pixel_centre_is_caught(monkeypatch):
    monkeypatch.setattr(mra_oracle, "centre", lambda L: (L / 2 - 0.5, L / 2 - 0.5))
    assert _fails(pins.test_linear_image_samples_closed_form, 0)


def test_missing_normalisation_is_caught(monkeypatch):
    orig = mra_oracle.reference_polar

    def unnormalised(refs, g):
        q, nu = orig(refs, mra_oracle.Geometry(**{**g.__dict__, "normalize": 0}))
        return q, nu

    monkeypatch.setattr(mra_oracle, "reference_polar", unnormalised)
    assert _fails(pins.test_self_cc_is_the_weighted_ring_norm, 1)


def test_unnegated_psi_is_caught(monkeypatch):
    orig = mra_oracle.align

    def wrong_psi(parts, refs, g, batch=8):
        res = orig(parts, refs, g, batch)
        res["psi"] = (g.n_phi - res["psi"]) % g.n_phi
        return res

    monkeypatch.setattr(oracle, "align", wrong_psi)
    assert _fails(pins.test_noise_free_planted_particles_are_recovered_exactly)


def test_wrong_average_rotation_sense_is_caught(monkeypatch):
    orig = mra_oracle.averages

    def negated(parts, params, prev, g):
        p = dict(params)
        p["psi"] = (g.n_phi - np.asarray(params["psi"])) % g.n_phi
        return orig(parts, p, prev, g)

    monkeypatch.setattr(oracle, "averages", negated)
    assert _fails(pins.test_averages_undo_quarter_turns_shifts_and_mirrors_exactly)


def test_runner_up_that_keeps_the_winner_is_caught(monkeypatch):
    """cc2 taken over the whole table (winner included) equals cc."""
    orig = mra_oracle.align

    def winner_kept(parts, refs, g, batch=8):
        res = orig(parts, refs, g, batch)
        res["cc2"] = res["cc"].copy()
        return res

    monkeypatch.setattr(oracle, "align", winner_kept)
    assert _fails(pins.test_winner_and_runner_up_of_linear_images_closed_form, 1)
    assert _fails(pins.test_winner_and_runner_up_of_linear_images_closed_form, 0)


def test_runner_up_of_the_wrong_order_is_caught(monkeypatch):
    """A cc2 read from the third-best candidate (or any other than the
    second) is caught as well."""
    orig = mra_oracle.align

    def third(parts, refs, g, batch=8):
        res = orig(parts, refs, g, batch)
        tab = oracle.cc_table(parts, refs, g)
        for i in range(len(res["cc2"])):
            res["cc2"][i] = np.sort(tab[i].reshape(-1))[-3]
        return res

    monkeypatch.setattr(oracle, "align", third)
    assert _fails(pins.test_winner_and_runner_up_of_linear_images_closed_form, 1)
