"""Smoothing parity on sinogram shapes other than the workloads': the whole
sinogram against the oracle's separable Gaussian (Methods, smoothing of the
scatter estimate along the radial, angular and planar axes).  One shape has
several radial tiles of the fused radial-and-plane pass with a ragged last
tile; the other has so many planes that a tile of all of them does not fit
in LDS and the library takes one pass per axis."""
import numpy as np
import pytest

import oracle.post as post
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PAPER_SIGMA = tuple(f / 2.35482 for f in (9.0, 6.0, 10.5))
HEAVY = tuple(3 * s for s in PAPER_SIGMA)

SHAPES = {
    # n_rad 257 over tiles of 86, 86, 85 radial positions; 23 planes
    "wide": (W.Scanner(n_crystals=320, n_rings=12, radius_mm=300.0, length_mm=150.0, crystals_per_module=8,
                       rings_per_block=4),
             W.Sinogram(n_rad=257, n_view=160, n_plane=23, n_tof=3, tof_bin_mm=200.0, tof_sigma_mm=0.0)),
    # 335 planes: the fused tile exceeds its LDS budget at these radii
    "tall": (W.Scanner(n_crystals=64, n_rings=168, radius_mm=150.0, length_mm=600.0, crystals_per_module=4,
                       rings_per_block=8),
             W.Sinogram(n_rad=63, n_view=32, n_plane=335, n_tof=2, tof_bin_mm=150.0, tof_sigma_mm=0.0)),
}


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("sigma", [PAPER_SIGMA, HEAVY, (2.0, 0.0, 3.0)], ids=["paper", "heavy", "no_view"])
def test_smoothing_matches_oracle_on_whole_sinogram(shape, sigma):
    import paper_2509_05047_amd as sse
    scanner, sino = SHAPES[shape]
    x = np.random.default_rng(11).uniform(0.1, 1.0, sino.shape).astype(np.float32)
    ref = post.gaussian_smooth(x, sigma).reshape(sino.shape)
    ctx = sse.Context(scanner, sino, dict(W.PHYSICS_DEFAULT))
    try:
        dx = torch.from_numpy(x.ravel()).cuda()
        out = torch.empty_like(dx)
        ctx.gaussian_smooth(dx, out, sigma)
        ctx.gaussian_smooth(dx, dx, sigma)  # in place
        torch.cuda.synchronize()
        got, inplace = out.cpu().numpy().reshape(sino.shape), dx.cpu().numpy().reshape(sino.shape)
    finally:
        ctx.close()
    assert np.array_equal(got, inplace)
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() < 1e-5, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))


# Which pass applies the ratio G / S of the smoothing normalisation depends on
# the axes smoothed: the view pass, the fused radial-and-plane pass, the
# radial or plane pass of the one-axis route, or the pointwise pass.
NORM_SIGMAS = {
    "all": HEAVY,
    "rad_plane": (HEAVY[0], 0.0, HEAVY[2]),
    "rad": (HEAVY[0], 0.0, 0.0),
    "view": (0.0, HEAVY[1], 0.0),
    "plane": (0.0, 0.0, HEAVY[2]),
    "none": (0.0, 0.0, 0.0),
}


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("which", sorted(NORM_SIGMAS))
def test_smoothing_normalisation_matches_oracle_in_every_route(shape, which):
    """The smoothing normalisation N = G_heavy(S) / S (1 where S or G is not
    positive) on the whole sinogram, whichever pass takes the ratio; empty
    bins of the reference give exactly 1."""
    import paper_2509_05047_amd as sse
    scanner, sino = SHAPES[shape]
    sigma = NORM_SIGMAS[which]
    rng = np.random.default_rng(12)
    Wd = rng.uniform(0.2, 2.0, sino.shape)
    Wd[0, 0, 0, :5] = 0.0
    Wd[-1, -1, -1, -3:] = 0.0
    ref = post.smoothing_normalisation(Wd, 0.75, sigma)
    ctx = sse.Context(scanner, sino, dict(W.PHYSICS_DEFAULT))
    try:
        dw = torch.from_numpy(Wd.ravel()).cuda()
        norm = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        ctx.smoothing_normalisation(dw, 0.75, norm, sigma)
        torch.cuda.synchronize()
        got = norm.cpu().numpy().reshape(sino.shape)
    finally:
        ctx.close()
    assert np.all(got[Wd == 0.0] == 1.0)
    if which == "none":
        assert np.all(got == 1.0)
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() < 1e-5, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))


# The clinical plane count (89) with 181 radial bins and one TOF bin: at
# three times the paper's FWHM the fused pass takes two radial tiles of 91
# positions, whose staged input and smoothed columns take 139 KB of LDS (the
# clinical shape: 141 KB), above 128 KB.
DEEP = (W.Scanner(n_crystals=182, n_rings=45, radius_mm=312.0, length_mm=250.0, crystals_per_module=7,
                  rings_per_block=5),
        W.Sinogram(n_rad=181, n_view=91, n_plane=89, n_tof=1, tof_bin_mm=624.0, tof_sigma_mm=0.0))


@pytest.mark.parametrize("which", ["all", "rad_plane"])
def test_fused_pass_with_large_lds_tiles_matches_oracle(which):
    """Smoothing and the smoothing normalisation at three times the paper's
    FWHM with the clinical plane count, against the oracle on the whole
    sinogram."""
    import paper_2509_05047_amd as sse
    scanner, sino = DEEP
    sigma = NORM_SIGMAS[which]
    rng = np.random.default_rng(13)
    Wd = rng.uniform(0.2, 2.0, sino.shape)
    Wd[0, 0, 0, :5] = 0.0
    ref_s = post.gaussian_smooth(Wd.astype(np.float32), sigma).reshape(sino.shape)
    ref_n = post.smoothing_normalisation(Wd, 0.75, sigma)
    ctx = sse.Context(scanner, sino, dict(W.PHYSICS_DEFAULT))
    try:
        x = torch.from_numpy(Wd.astype(np.float32).ravel()).cuda()
        out = torch.empty_like(x)
        ctx.gaussian_smooth(x, out, sigma)
        dw = torch.from_numpy(Wd.ravel()).cuda()
        norm = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        ctx.smoothing_normalisation(dw, 0.75, norm, sigma)
        torch.cuda.synchronize()
        got_s = out.cpu().numpy().reshape(sino.shape)
        got_n = norm.cpu().numpy().reshape(sino.shape)
    finally:
        ctx.close()
    rel = np.abs(got_s - ref_s) / np.abs(ref_s)
    assert rel.max() < 1e-5, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))
    assert np.all(got_n[Wd == 0.0] == 1.0)
    rel = np.abs(got_n - ref_n) / np.abs(ref_n)
    assert rel.max() < 1e-5, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))
