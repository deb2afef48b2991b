"""Pins of the oracle's iterative MRA (the outer loop of Algorithm 1).

The loop is a composition of the pinned pass (oracle.align) and the pinned
average update (oracle.averages); these tests pin what the loop adds: one
pass equals one align + average update, planted noise-free particles keep
their classes so the loop stops at the second pass, the convergence rule
reads the fraction of reassigned particles, and a run started from
particles as references reaches a fixed point of the pass.
"""

import numpy as np

import oracle
from paper_2011_05755_amd import synth


def case(N, snr, seed, on_grid=True):
    L, K, T = 32, 3, 1
    blobs = synth.make_blobs(K, L, seed=(seed, 0), rho_max=12.0)
    refs = synth.render_refs(blobs).numpy()
    parts, truth = synth.make_particles(blobs, N, T, snr, seed=(seed, 1),
                                        n_phi_grid=4 if on_grid else None)
    g = oracle.Geometry(L=L, r_min=1, r_max=13, n_phi=256, shift_max=T)
    return g, refs, parts.numpy(), truth


def test_one_pass_is_one_alignment_and_one_average_update():
    g, refs, parts, _ = case(6, 1e6, 80)
    params, Y, counts, n, fracs = oracle.classify(parts, refs, g, max_iter=1)
    want = oracle.align(parts, refs.astype(np.float32), g)
    Yw, cw = oracle.averages(parts, want, refs.astype(np.float32), g)
    assert n == 1 and fracs == []
    for key in want:
        np.testing.assert_array_equal(params[key], want[key])
    np.testing.assert_array_equal(Y, Yw.astype(np.float32))
    np.testing.assert_array_equal(counts, cw)


def test_planted_classes_are_kept_and_the_loop_stops_at_the_second_pass():
    g, refs, parts, truth = case(9, 1e6, 81)
    params, Y, counts, n, fracs = oracle.classify(parts, refs, g, max_iter=10, max_changed_frac=0.0)
    assert n == 2 and fracs == [0.0]
    np.testing.assert_array_equal(params["ref"], truth.ref)
    np.testing.assert_array_equal(counts, np.bincount(truth.ref, minlength=3))


def test_convergence_rule_reads_the_reassigned_fraction():
    g, refs, parts, _ = case(8, 0.5, 82, on_grid=False)
    start = parts[[0, 3, 5]]                      # particles as the first references
    params, Y, counts, n, fracs = oracle.classify(parts, start, g, max_iter=6, max_changed_frac=0.0)
    assert len(fracs) == n - 1
    assert all(f > 0.0 for f in fracs[:-1])       # it only stopped when nothing changed ...
    if n < 6:
        assert fracs[-1] == 0.0
        # ... and then the last averages are a fixed point of the pass
        again = oracle.align(parts, Y, g)
        np.testing.assert_array_equal(again["ref"], params["ref"])
    p1, _, _, n1, f1 = oracle.classify(parts, start, g, max_iter=6, max_changed_frac=1.0)
    assert n1 == 2 and len(f1) == 1               # any fraction is at most 1: stop at pass 2
