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


# ---------------------------------------------------------------------------
# smoothing normalisation (Methods, "Known activity distribution, very
# limited simulation time")
# ---------------------------------------------------------------------------

def _structured(shape, seed):
    """A smooth field F and a high-frequency multiplicative detector pattern P
    (per radial bin and per view, like crystal efficiencies) on a
    [tof][plane][view][rad] grid."""
    rng = np.random.default_rng(seed)
    nt, npl, nv, nr = shape
    t, p, v, r = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    F = np.exp(-((r - nr / 2) / (0.35 * nr)) ** 2 - ((p - npl / 2) / npl) ** 2 - ((t - nt / 2) / nt) ** 2)
    F = F * (1.0 + 0.3 * np.cos(2 * np.pi * v / nv))
    P = (1.0 + 0.3 * rng.uniform(-1, 1, nr))[None, None, None, :] * (1.0 + 0.2 * rng.uniform(-1, 1, nv))[None, None, :, None]
    return F, np.broadcast_to(P, shape).copy()


FWHM_PAPER = np.array([9.0, 6.0, 10.5]) / 2.35482


def test_unit_normalisation_is_the_plain_finalize():
    F, P = _structured((3, 7, 32, 63), 0)
    sens = np.random.default_rng(1).uniform(0.5, 1.5, F.shape)
    W = P * F
    got = post.finalize_normalised(W, 0.7, np.ones_like(W), (2.0, 1.5, 2.5), sens)
    ref = post.gaussian_smooth(0.7 * W, (2.0, 1.5, 2.5)) * sens
    assert np.array_equal(got, ref)


def test_smoothing_normalisation_definition():
    F, P = _structured((3, 7, 32, 63), 2)
    S = P * F
    S[0, 0, 0, :5] = 0.0                       # empty bins
    N = post.smoothing_normalisation(S, 1.0, 3 * FWHM_PAPER)
    G = post.gaussian_smooth(S, 3 * FWHM_PAPER)
    ok = S > 0
    assert np.allclose(N[ok] * S[ok], G[ok], rtol=1e-13)
    assert np.all(N[~ok] == 1.0)
    Nc = post.smoothing_normalisation(np.full(S.shape, 2.5), 1.0, FWHM_PAPER)
    assert np.abs(Nc - 1.0).max() < 1e-12     # the normalised Gaussian keeps constants


def test_normalisation_removes_and_restores_detector_structure():
    """With an exact normalisation N = c / P the normalised finalize is
    P * G(F) * sens (the structure P passes through the smoothing untouched);
    with N computed from a structured reference object (a smooth field
    times the same P, heavily smoothed) the estimate keeps the structure far
    better than plain smoothing does."""
    shape = (3, 7, 32, 63)
    F, P = _structured(shape, 3)
    sens = np.ones(shape)
    S = P * F
    exact = post.finalize_normalised(S, 1.0, 2.0 / P, FWHM_PAPER, sens)
    assert np.allclose(exact, P * post.gaussian_smooth(F, FWHM_PAPER), rtol=1e-12)
    Fref, _ = _structured(shape, 4)
    Fref = np.ones(shape) * (1.0 + 0.1 * Fref)   # broad reference object
    N = post.smoothing_normalisation(P * Fref, 1.0, 3 * FWHM_PAPER)
    norm_est = post.finalize_normalised(S, 1.0, N, FWHM_PAPER, sens)
    plain_est = post.gaussian_smooth(S, FWHM_PAPER)
    target = P * post.gaussian_smooth(F, FWHM_PAPER)
    err_norm = np.abs(norm_est / target - 1).max()
    err_plain = np.abs(plain_est / target - 1).max()
    assert err_norm < 0.2 * err_plain, (err_norm, err_plain)


def test_total_scatter_is_the_exact_sum_of_the_products():
    """Integer-valued products sum exactly; a sum whose naive order loses
    the small terms keeps them; the TOF broadcast of a sensitivity without
    TOF axis equals the full-shape sensitivity."""
    rng = np.random.default_rng(4)
    w = rng.integers(0, 1000, (3, 2, 4, 5)).astype(np.float64)
    sens = rng.integers(1, 4, (2, 4, 5)).astype(np.float64)
    assert post.total_scatter(w, 2.0, sens) == float((2 * w * sens[None]).sum())
    big = np.zeros((1, 1, 1, 4))
    big[0, 0, 0] = [1e16, 1.0, -1e16, 1.0]
    assert post.total_scatter(big, 1.0, np.ones((1, 1, 4))) == 2.0
    full = np.broadcast_to(sens[None], w.shape)
    assert post.total_scatter(w, 0.37, sens) == post.total_scatter(w, 0.37, full)
