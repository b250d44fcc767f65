"""Seeded input generators: determinism and loose statistics."""
import numpy as np

from paper_2509_01416_amd import inputs as I


def test_grf_seeded_and_statistics():
    a = I.grf_2d(64, 10.0, seed=5)
    b = I.grf_2d(64, 10.0, seed=5)
    assert np.array_equal(a, b)
    samples = np.stack([I.grf_2d(64, 10.0, seed=s, clip_min=None) for s in range(40)])
    assert abs(samples.mean() - 1.0) < 0.03
    assert abs(samples.std() - 0.3) < 0.03
    # squared-exponential correlation at a lag of 1 correlation length
    # (6.4 cells of 0.15625 mfp): exp(-1/2) ~= 0.607
    d = samples - 1.0
    lag = 6
    r = np.mean(d[:, :, :-lag] * d[:, :, lag:]) / np.mean(d * d)
    assert abs(r - np.exp(-0.5 * (lag * 10.0 / 64) ** 2)) < 0.08


def test_named_workloads_shapes():
    wl = I.slab_1d()
    assert wl.instances[0].nx == 200 and wl.quad.n_dir == 8
    wl = I.sinusoid_128()
    assert wl.quad.n_dir == 40 and wl.instances[0].cells == 128 * 128
    wl = I.batched_uneven(16)
    assert all(i.nx in (32, 48, 64, 96, 128) for i in wl.instances)
    assert all(np.all(i.sigma_s <= i.sigma_t) for i in wl.instances)
    wl = I.hard_two_region(2, 32)
    st = wl.instances[0].sigma_t
    assert set(np.unique(st)) == {1.0, 5.0}
    assert wl.quad.n_dir == 144


def test_random_line_masks_differ_by_seed():
    a = I.random_line_mask(32, 32, 10, 10, 1)
    b = I.random_line_mask(32, 32, 10, 10, 2)
    assert a.any() and (~a).any() and not np.array_equal(a, b)
