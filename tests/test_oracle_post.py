"""Pins of the oracle's sinogram post-processing (sensitivity multiply and
Gaussian smoothing) against library routines and closed forms."""
import numpy as np
import pytest
from scipy.ndimage import gaussian_filter1d

from oracle import post


def rand_sino(shape=(3, 5, 8, 9), seed=0):
    return np.random.default_rng(seed).uniform(0, 10, shape)


@pytest.mark.parametrize("sigma", [0.7, 2.0, 3.3])
def test_radial_and_planar_smoothing_match_scipy_reflect(sigma):
    x = rand_sino()
    got = post.gaussian_smooth(x, (sigma, 0, 0))
    ref = gaussian_filter1d(x, sigma, axis=3, mode="reflect", truncate=4.0)
    assert np.max(np.abs(got - ref)) < 1e-12
    got = post.gaussian_smooth(x, (0, 0, sigma))
    ref = gaussian_filter1d(x, sigma, axis=1, mode="reflect", truncate=4.0)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("sigma", [0.9, 2.0, 5.0])
def test_view_smoothing_is_circular_over_the_doubled_sinogram(sigma):
    """Views cover [0, pi); continuing past pi revisits the same LORs from
    the other end (radial and TOF axes reversed).  Concatenating the sinogram
    with its flipped copy gives a 2*n_view periodic signal, smoothed with
    scipy's wrap mode."""
    x = rand_sino((3, 2, 7, 5), seed=1)
    doubled = np.concatenate([x, x[::-1, :, :, ::-1]], axis=2)
    ref = gaussian_filter1d(doubled, sigma, axis=2, mode="wrap", truncate=4.0)[:, :, :7, :]
    got = post.gaussian_smooth(x, (0, sigma, 0))
    assert np.max(np.abs(got - ref)) < 1e-12


def test_smoothing_keeps_constants_and_mass_on_symmetric_input():
    x = np.full((2, 4, 6, 7), 3.25)
    assert np.max(np.abs(post.gaussian_smooth(x, (2.0, 2.0, 2.0)) - 3.25)) < 1e-12


def test_separable_passes_commute():
    x = rand_sino((3, 6, 8, 9), seed=2)
    a = post.gaussian_smooth(post.gaussian_smooth(x, (1.5, 0, 0)), (0, 2.0, 1.0))
    b = post.gaussian_smooth(post.gaussian_smooth(x, (0, 2.0, 1.0)), (1.5, 0, 0))
    assert np.max(np.abs(a - b)) < 1e-12


def test_apply_sensitivity_broadcast_and_rounding():
    rng = np.random.default_rng(3)
    w = rng.integers(0, 50, size=(4, 3, 5, 7)).astype(np.float64)
    sens = rng.uniform(0.5, 1.5, size=(3, 5, 7)).astype(np.float32)
    a = post.apply_sensitivity(w, 0.25, sens)
    b = post.apply_sensitivity(w, 0.25, np.broadcast_to(sens, w.shape))
    assert a.dtype == np.float32 and np.array_equal(a, b)
    # scale 1 and sens 1: the weights themselves, rounded once to binary32
    one = post.apply_sensitivity(w / 3.0, 1.0, np.ones(w.shape, np.float32))
    assert np.array_equal(one, (w / 3.0).astype(np.float32))


def test_emission_scale():
    act = np.ones((2, 3, 4), np.float32) * 2.0
    # 24 voxels of 1000 mm^3 = 1 ml each at 2 Bq/ml for 10 s over 100 histories
    assert post.emission_scale(act, (10.0, 10.0, 10.0), 100, acq_seconds=10.0) == pytest.approx(24 * 2 * 10 / 100)
