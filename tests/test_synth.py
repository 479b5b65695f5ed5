"""The seeded generators are deterministic and have the stated shapes and ranges."""

import numpy as np

import synth


def test_uniform_deterministic():
    a = synth.uniform(33, 17, 5)
    b = synth.uniform(33, 17, 5)
    assert synth.sha256(a) == synth.sha256(b)
    assert synth.sha256(a) != synth.sha256(synth.uniform(33, 17, 6))
    assert a.dtype == np.uint8 and a.shape == (33, 17)


def test_smooth_range_and_determinism():
    a = synth.smooth(128, 96, 4.0, 1)
    assert a.min() == 0 and a.max() == 255
    assert np.array_equal(a, synth.smooth(128, 96, 4.0, 1))
    u = synth.smooth(64, 64, 2.0, 2, np.uint16, noise_frac=0.05)
    assert u.dtype == np.uint16


def test_smooth_is_smoother_than_uniform():
    s = synth.smooth(256, 256, 8.0, 3).astype(np.int32)
    u = synth.uniform(256, 256, 3).astype(np.int32)
    assert np.abs(np.diff(s, axis=1)).mean() < 0.1 * np.abs(np.diff(u, axis=1)).mean()


def test_offsets_for_eq2_directions():
    assert synth.offsets_for([1]) == [(1, 0), (-1, 1), (0, 1), (1, 1)]
    assert len(synth.offsets_for([1, 2, 4])) == 12


def test_checkerboard_pattern():
    c = synth.checkerboard(3, 4, 1, 9)
    assert c.tolist() == [[1, 9, 1, 9], [9, 1, 9, 1], [1, 9, 1, 9]]


def test_batch_tiles_recipe():
    w = synth.batch_tiles(64)
    imgs = w["images"]
    assert len(imgs) == 64 and w["N"] == 16 and len(w["offsets"]) == 4
    for im in imgs:
        assert im.dtype == np.uint8 and 32 <= im.shape[0] <= 512 and 32 <= im.shape[1] <= 512
    # deterministic
    again = synth.batch_tiles(64)["images"]
    assert all(np.array_equal(a, b) for a, b in zip(imgs, again))
