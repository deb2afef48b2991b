"""Checks of the seeded input generator (CPU only)."""

import math

import numpy as np
import torch

from paper_2011_05755_amd import synth


def test_same_seed_same_stack_and_different_seed_differs():
    b1 = synth.make_blobs(5, 48, seed=(0, 0), rho_max=20.0)
    b2 = synth.make_blobs(5, 48, seed=(0, 0), rho_max=20.0)
    np.testing.assert_array_equal(b1.centres, b2.centres)
    p1, t1 = synth.make_particles(b1, 20, 2, 0.1, seed=(0, 1))
    p2, t2 = synth.make_particles(b2, 20, 2, 0.1, seed=(0, 1))
    assert torch.equal(p1, p2)
    np.testing.assert_array_equal(t1.alpha, t2.alpha)
    p3, _ = synth.make_particles(b1, 20, 2, 0.1, seed=(0, 2))
    assert not torch.equal(p1, p3)


def test_blobs_stay_inside_rho_max():
    L = 64
    b = synth.make_blobs(50, L, seed=1, rho_max=28.0)
    c = L // 2
    used = b.amp > 0
    rad = np.hypot(b.centres[..., 0] - c, b.centres[..., 1] - c)
    assert np.all(rad[used] + 2 * b.sigma[used] <= 28.0 + 1e-12)
    nb = used.sum(axis=1)
    assert nb.min() >= 8 and nb.max() <= 20
    assert b.sigma[used].min() >= 2.0 and b.sigma[used].max() <= 6.0
    assert b.amp[used].min() >= 0.5 and b.amp[used].max() <= 1.5


def test_noise_level_matches_the_snr_definition():
    b = synth.make_blobs(3, 64, seed=2, rho_max=28.0)
    clean, truth0 = synth.make_particles(b, 200, 2, None, seed=(2, 1))
    noisy, truth = synth.make_particles(b, 200, 2, 0.05, seed=(2, 1))
    np.testing.assert_array_equal(truth0.alpha, truth.alpha)   # same planted draw
    noise = (noisy - clean).double()
    var_clean = clean.double().reshape(200, -1).var(dim=1, unbiased=False).numpy()
    np.testing.assert_allclose(truth.noise_sigma ** 2, var_clean / 0.05, rtol=1e-5)
    emp = noise.reshape(200, -1).var(dim=1).numpy()
    ratio = emp / truth.noise_sigma ** 2
    assert abs(ratio.mean() - 1.0) < 0.01
    assert np.all(np.abs(ratio - 1.0) < 0.1)


def test_identity_transform_renders_the_reference():
    b = synth.make_blobs(2, 40, seed=3, rho_max=16.0)
    refs = synth.render_refs(b)
    parts, truth = synth.make_particles(b, 30, 0, None, seed=4, mirror=False, n_phi_grid=1)
    assert np.all(truth.psi_index == 0) and np.all(truth.mirror == 0)
    for n in range(30):
        torch.testing.assert_close(parts[n], refs[truth.ref[n]], rtol=0, atol=1e-6)


def test_planted_parameters_are_in_range():
    b = synth.make_blobs(7, 64, seed=5, rho_max=28.0)
    _, t = synth.make_particles(b, 500, 3, 0.1, seed=6, n_phi_grid=256)
    assert t.ref.min() >= 0 and t.ref.max() < 7
    assert t.shift_x.min() >= -3 and t.shift_x.max() <= 3
    assert t.shift_y.min() >= -3 and t.shift_y.max() <= 3
    assert set(np.unique(t.mirror)) <= {0, 1}
    np.testing.assert_allclose(t.alpha, t.psi_index * 2 * math.pi / 256)


def test_mirror_and_rotation_move_the_blob_centres_as_stated():
    """A single narrow blob lands where Shift_t o Mir^m o Rot_alpha puts it."""
    L = 64
    b = synth.BlobSet(centres=np.array([[[42.0, 32.0]] + [[0.0, 0.0]] * 19]),
                      sigma=np.ones((1, 20)), amp=np.array([[1.0] + [0.0] * 19]), L=L)
    parts, t = synth.make_particles(b, 40, 2, None, seed=7, n_phi_grid=4)
    for n in range(40):
        img = parts[n].numpy()
        y, x = np.unravel_index(np.argmax(img), img.shape)
        quarter = int(t.psi_index[n])
        vx, vy = [(10, 0), (0, 10), (-10, 0), (0, -10)][quarter]
        if t.mirror[n]:
            vy = -vy
        assert (x, y) == (32 + t.shift_x[n] + vx, 32 + t.shift_y[n] + vy)


def test_workload_recipes_and_uneven_specs():
    c1 = synth.WORKLOADS["mra_c1"]
    assert (c1["N"], c1["L"], c1["K"], c1["shift_max"], c1["r_max"]) == (100000, 76, 100, 3, 35)
    specs = synth.uneven_stack_specs()
    assert len(specs) == 64
    for s in specs:
        assert s["L"] in (64, 76, 96, 128)
        assert 2000 <= s["N"] <= 50000 and 20 <= s["K"] <= 400 and 2 <= s["shift_max"] <= 5
        assert s["r_max"] == s["L"] // 2 - 2
