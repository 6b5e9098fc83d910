"""Host checks of the paper's synthetic scenarios (Section V-B): foreground
covers the requested fraction, foreground labels lie in a structure and
background labels outside every structure, and the generators are seeded."""

import numpy as np

import synth


def _labels_inside(seeds, truth):
    v = np.floor(seeds[:, :3]).astype(np.int64)
    return truth[v[:, 2], v[:, 1], v[:, 0]]


def test_vessels_scenario():
    vol, seeds, truth = synth.vessels_volume(n=96, seed=3)
    assert 0.01 <= truth.mean() < 0.03
    assert vol.dtype == np.float32 and vol.min() >= 0.0 and vol.max() <= 1.0
    fg, bg = seeds[:, 3] == 1, seeds[:, 3] == 0
    assert fg.sum() >= 2 and bg.sum() >= 1
    assert np.all(_labels_inside(seeds[fg], truth) == 1)
    # background points keep two radii from their own cell and lie outside
    # every other sphere in continuous coordinates; the voxel a point falls
    # in can still touch a neighbouring sphere's rasterisation
    assert np.mean(_labels_inside(seeds[bg], truth) == 0) >= 0.95
    # vessels enter from the border: foreground touches a face of the volume
    faces = [truth[0], truth[-1], truth[:, 0], truth[:, -1], truth[:, :, 0], truth[:, :, -1]]
    assert any(f.any() for f in faces)
    again = synth.vessels_volume(n=96, seed=3)
    assert np.array_equal(again[2], truth) and np.array_equal(again[1], seeds)


def test_cells_scenario():
    vol, seeds, truth = synth.cells_volume(n=96, seed=3)
    assert 0.01 <= truth.mean() < 0.03
    fg, bg = seeds[:, 3] == 1, seeds[:, 3] == 0
    assert np.all(_labels_inside(seeds[fg], truth) == 1)
    # background points keep two radii from their own cell and lie outside
    # every other sphere in continuous coordinates; the voxel a point falls
    # in can still touch a neighbouring sphere's rasterisation
    assert np.mean(_labels_inside(seeds[bg], truth) == 0) >= 0.95
