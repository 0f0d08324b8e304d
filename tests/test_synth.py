"""The seeded input generators: determinism, shapes, ranges and structure."""
import numpy as np

from synth_mrf import CONFIGS, make_batch_configs, make_config, make_stereo, sha256_of


def test_deterministic_and_seed_sensitive():
    a = make_stereo(20, 24, 16, 0.05, 4.0, "rectangles", 0)[0]
    b = make_stereo(20, 24, 16, 0.05, 4.0, "rectangles", 0)[0]
    c = make_stereo(20, 24, 16, 0.05, 4.0, "rectangles", 1)[0]
    assert sha256_of(a) == sha256_of(b) != sha256_of(c)


def test_shapes_ranges_and_truth():
    cfg = CONFIGS["stereo16"]
    g, D = make_config(cfg)
    assert g.shape == (16, 16, 16) and g.dtype == np.float32
    assert np.all(g > 0) and np.all(g <= 1)
    assert D.min() >= 0 and D.max() < cfg.M
    g2, D2, L, R = make_stereo(40, 50, 32, 0.03, 6.0, "slanted", 2)
    assert D2.min() >= 0 and D2.max() < 32 and g2.shape == (40, 50, 32)


def test_true_disparity_matches_best():
    """Without noise the true disparity has |L - R| = 0 wherever it is visible."""
    g, D, L, R = make_stereo(30, 40, 8, 0.05, 0.0, "rectangles", 3)
    r, c = np.mgrid[0:30, 0:40]
    g_true = g[r, c, D]
    visible = c - D >= 0
    # the paste order lets nearer surfaces overwrite, so most (not all) pixels match
    assert np.mean(g_true[visible] == 1.0) > 0.5


def test_batch_configs():
    insts = make_batch_configs()
    assert len(insts) == 32
    for it in insts:
        assert 64 <= it.H <= 512 and 64 <= it.W <= 512
        assert it.M in (16, 32, 64, 128)
        assert 1 <= it.T <= 8
        assert 0.3 <= it.alpha < 1.5
    assert make_batch_configs() == insts
