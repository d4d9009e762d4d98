"""CPU checks of the seeded workload generators used by the tracking loop."""
import numpy as np

from paper_1705_03524_amd import synth


def test_track_sequence_is_seeded_and_in_frame():
    a, ta, side = synth.track_sequence(11, 20, 200, 260, side=21, ndistract=2)
    b, tb, _ = synth.track_sequence(11, 20, 200, 260, side=21, ndistract=2)
    assert np.array_equal(ta, tb) and all(np.array_equal(x, y) for x, y in zip(a, b))
    r = (side - 1) // 2
    assert ta[:, 0].min() >= r and ta[:, 0].max() <= 259 - r
    assert ta[:, 1].min() >= r and ta[:, 1].max() <= 199 - r
    steps = np.abs(np.diff(ta, axis=0)).max()
    assert 0 < steps <= 16           # smooth motion, a few pixels per frame


def test_distractor_has_the_targets_values_in_another_arrangement():
    t, d = synth._patch_pair(synth.rng(3), 31)
    assert np.array_equal(np.sort(t.ravel()), np.sort(d.ravel()))   # same plain histogram
    assert t[15, 15] == t.max() and d[15, 15] == d.min()               # brightest / darkest centre
    assert not np.array_equal(t, d)


def test_target_drawn_at_truth():
    fr, tr, side = synth.track_sequence(5, 10, ndistract=0)
    t, _ = synth._patch_pair(synth.rng(5), side)
    r = (side - 1) // 2
    for f, (x, y) in zip(fr, tr):
        assert np.array_equal(f[y - r:y + r + 1, x - r:x + r + 1], t)
