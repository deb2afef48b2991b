"""Pins of the oracle's reference-free alignment (RFA): the MRA pass and the
average update with one running average as the only reference.

What RFA adds to the pinned pass and update is the starting reference (the
plain mean), the single-reference loop and its stop rule on changed
parameters; these tests fix them against cases whose answer is known
without the oracle: identical copies of one image align to the identity and
average back to the image exactly, planted transforms of a known image are
recovered, and one pass is one alignment against the plain mean.
"""

import numpy as np

import oracle
from paper_2011_05755_amd import synth

L, T = 32, 2


def geom(mirror=1):
    return oracle.Geometry(L=L, r_min=1, r_max=13, n_phi=256, shift_max=T, mirror=mirror)


def image(seed):
    blobs = synth.make_blobs(1, L, seed=(seed, 0), rho_max=12.0)
    return blobs, synth.render_refs(blobs).numpy()


def test_identical_copies_align_to_the_identity_and_average_back_exactly():
    _, ref = image(70)
    parts = np.repeat(ref, 9, axis=0)
    params, avg, n, fracs = oracle.rfa(parts, geom(), max_iter=5)
    assert n == 2 and fracs == [0.0]
    for key in ("shift_x", "shift_y", "psi", "mirror", "ref"):
        assert np.all(params[key] == 0), key
    np.testing.assert_array_equal(avg, ref[0])        # mean of equal images, identity warp
    # the winner is the self-correlation: the weighted ring norm of the image
    p = oracle.particle_polar(ref[0], geom())[0, T, T]   # no mirror, zero shift
    w = oracle.ring_weights(geom())
    assert np.allclose(params["cc"], np.sqrt(np.sum(w[:, None] * p * p)), rtol=1e-12)


def test_planted_transforms_of_a_known_image_are_recovered():
    blobs, ref = image(71)
    parts, truth = synth.make_particles(blobs, 12, T, None, seed=(71, 1), n_phi_grid=256)
    params, avg, n, fracs = oracle.rfa(parts.numpy(), geom(), max_iter=4, init=ref[0])
    assert n == 2 and fracs == [0.0]
    np.testing.assert_array_equal(params["shift_x"], truth.shift_x)
    np.testing.assert_array_equal(params["shift_y"], truth.shift_y)
    np.testing.assert_array_equal(params["mirror"], truth.mirror)
    np.testing.assert_array_equal(params["psi"], truth.psi_index)
    assert np.all(params["ref"] == 0)


def test_one_pass_aligns_against_the_plain_mean():
    blobs, _ = image(72)
    parts = synth.make_particles(blobs, 7, T, 0.5, seed=(72, 1))[0].numpy()
    params, avg, n, fracs = oracle.rfa(parts, geom(), max_iter=1)
    mean = parts.astype(np.float64).mean(axis=0).astype(np.float32)[None]
    want = oracle.align(parts, mean, geom())
    Yw, _ = oracle.averages(parts, want, mean, geom())
    assert n == 1 and fracs == []
    for key in want:
        np.testing.assert_array_equal(params[key], want[key])
    np.testing.assert_array_equal(avg, Yw[0].astype(np.float32))


def test_stop_rule_counts_particles_with_any_changed_parameter():
    blobs, _ = image(73)
    parts = synth.make_particles(blobs, 10, T, 0.3, seed=(73, 1))[0].numpy()
    _, _, n, fracs = oracle.rfa(parts, geom(), max_iter=6, max_changed_frac=0.0)
    # from the plain mean the parameters settle over several passes
    assert n == 5 and fracs == [0.2, 0.1, 0.1, 0.0]
    _, _, n1, f1 = oracle.rfa(parts, geom(), max_iter=6, max_changed_frac=1.0)
    assert n1 == 2 and len(f1) == 1
    # without the mirror search every parameter set has mirror 0
    p0, _, _, _ = oracle.rfa(parts, geom(mirror=0), max_iter=2)
    assert np.all(p0["mirror"] == 0)
