"""Input generators: seeds, shapes, dtypes and the recipe's stated magnitudes."""
import numpy as np

import synthetic as G


def test_pairs_are_reproducible_and_float32():
    a = G.phantom_pair((40, 56), 7, 0.5, 3.0)
    b = G.phantom_pair((40, 56), 7, 0.5, 3.0)
    for x, y in ((a.source, b.source), (a.target, b.target), (a.p0, b.p0)):
        assert x.dtype == np.float32 and x.flags.c_contiguous
        np.testing.assert_array_equal(x, y)
    c = G.phantom_pair((40, 56), 8, 0.5, 3.0)
    assert not np.array_equal(a.target, c.target)


def test_warp_magnitude_and_phantom_levels():
    rng = np.random.default_rng(0)
    u = G.smooth_warp((64, 80), 20.0, 6.0, rng)
    assert abs(np.sqrt((u ** 2).sum(0)).max() - 6.0) < 1e-12
    img = G.phantom((120, 120), np.random.default_rng(1))
    assert 0.7 < img[60, 60] < 0.9           # inner shell 0.8 (+ noise)
    assert abs(img[0, 0]) < 1e-6              # background
    noise = G.gradient_noise((50, 50), 6.0, np.random.default_rng(2))
    assert abs(np.abs(noise).max() - 1.0) < 1e-12


def test_disk_workload():
    w = G.workload("c1")
    p = w.pairs[0]
    assert p.shape == (64, 64) and w.T == 10
    assert abs(p.rho - 0.5) < 1e-7 and abs(p.sigma - 3.0) < 1e-7
    assert 0.005 < p.p0.std() < 0.015
    assert p.target.max() > 1.5               # disk + blob


def test_ragged_2d_batch_recipe():
    w = G.workload("c3", n_pairs=12)
    assert w.T == 20 and len(w.pairs) == 12
    for p in w.pairs:
        assert p.shape[0] in G.SIZES_2D and p.shape[1] in G.SIZES_2D
        assert 0.05 <= p.rho <= 1.0 and 2.0 <= p.sigma <= 6.0
        assert p.lam == G.LAMBDA
    assert len({p.shape for p in w.pairs}) > 3


def test_lesion_lies_inside_the_phantom():
    p = G.phantom_pair((96, 128), 11, 0.5, 3.0, p0_kind="zero")
    diff = p.target - p.source
    peak = np.unravel_index(np.argmax(diff), diff.shape)
    assert 0.25 * 96 < peak[0] < 0.75 * 96 and 0.25 * 128 < peak[1] < 0.75 * 128
    np.testing.assert_array_equal(p.p0, 0.0)


def test_golden_fixture_holds_the_papers_fig1_time_steps():
    """The fixture states the paper's printed time steps: Eulerian 1/38,
    semi-Lagrangian 1/20 (Results, Fig. 1)."""
    from golden_fixtures import fig1_steps
    assert fig1_steps() == (38, 20)
