"""Pins of the reconstruction oracle of the joint estimation loop (TOF Joseph
projector and TOF-OSEM, binary64; Methods, "Unknown activity distribution,
very limited simulation time" and "Evaluation metrics").

What ties it to something other than itself:
  - the simulator oracle's own coincidences: a point source in air binned by
    the Monte Carlo lies on the projector's LOR of that bin, at the TOF
    coordinate the simulator measured (sign included);
  - adjointness <P x, y> = <x, P^T y> for the TOF and non-TOF projector and
    for subsets;
  - closed forms: line integrals of a Gaussian blob, and its TOF profile (a
    Gaussian of variance sigma_blob^2 + sigma_tof^2 along the LOR, integrated
    over each TOF bin);
  - OSEM: the true image is a fixed point of the update for noiseless data,
    and OSEM recovers a smooth phantom from noiseless data with attenuation
    and an additive background.
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O
import workloads as W


def tiny():
    w = W.WORKLOADS["tiny"]
    pd, mu, act = W.make_phantom(w)
    return w, pd, mu, act


def fine_grid(n=96, size=128.0):
    """A transaxial grid finer than the tiny phantom's, same extent."""
    v = size / n
    return W.PhantomDesc(n, n, 1, (v, v, v), (-size / 2, -size / 2, -size / 2))


def lor_geometry(scanner, n_rad):
    a, b = O.recon_lor_table(scanner.n_crystals, n_rad)
    R, n = scanner.radius_mm, scanner.n_crystals
    pa = 2 * np.pi * (a + 0.5) / n
    pb = 2 * np.pi * (b + 0.5) / n
    A = np.stack([R * np.cos(pa), R * np.sin(pa)], -1)
    B = np.stack([R * np.cos(pb), R * np.sin(pb)], -1)
    m = 0.5 * (A + B)
    u = (A - B) / np.linalg.norm(A - B, axis=-1, keepdims=True)
    return a, b, m, u


def test_lor_table_covers_every_bin_with_the_chord_distance_of_its_radial_index():
    w, *_ = tiny()
    a, b, m, u = lor_geometry(w.scanner, w.sino.n_rad)
    assert (a >= 0).all() and (b >= 0).all()
    pairs = {tuple(sorted(x)) for x in zip(a.ravel(), b.ravel())}
    assert len(pairs) == a.size == w.scanner.n_crystals * (w.scanner.n_crystals - 1) // 2
    rho = np.arange(w.sino.n_rad) - (w.sino.n_rad - 1) // 2
    d = np.abs(m[..., 0] * u[..., 1] - m[..., 1] * u[..., 0])  # distance of the LOR from the centre
    expect = w.scanner.radius_mm * np.abs(np.sin(np.pi * rho / w.scanner.n_crystals))
    np.testing.assert_allclose(d, np.broadcast_to(expect, d.shape), atol=1e-9)


def test_simulated_point_source_lies_on_the_projector_lor_at_its_tof_coordinate():
    """Trues of an off-centre point source in air, TOF jitter 0: for every
    counted coincidence the source lies within a crystal width of the LOR
    the projector assigns to its (view, rad), and the simulator's tau equals
    the source's signed distance from the LOR midpoint towards the
    TOF-positive end up to the crystal size (hit points are not crystal
    centres) -- which also fixes the end that is TOF-positive."""
    w, *_ = tiny()
    src = np.array([31.0, -17.0, 5.0])
    pd, mu, act = W.point_source(tuple(src))
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    r = O.simulate(w.scanner, w.sino, w.physics, pd, mu, activity=act, lut_desc=ld, lut=lut, seed=3, n=20000,
                   records=True, sinograms=False)
    rec = r["records"]
    rec = rec[(rec["outcome"] & 0xFF) == O.OUTCOME["true"]]
    assert rec.size > 1000
    bins = O.record_bins(rec)
    n_rad, n_view = w.sino.n_rad, w.sino.n_view
    rad = bins % n_rad
    view = (bins // n_rad) % n_view
    _, _, m, u = lor_geometry(w.scanner, n_rad)
    mm, uu = m[view, rad], u[view, rad]
    rel = src[None, :2] - mm
    dist = np.abs(rel[:, 0] * uu[:, 1] - rel[:, 1] * uu[:, 0])
    s = (rel * uu).sum(-1)
    pitch = 2 * np.pi * w.scanner.radius_mm / w.scanner.n_crystals
    assert dist.max() < pitch, dist.max()
    err = np.abs(s - rec["tau_mm"])
    assert err.max() < pitch and np.median(err) < 0.25 * pitch, (err.max(), np.median(err))
    far = np.abs(s) > pitch
    assert far.sum() > 1000 and np.all(np.sign(s[far]) == np.sign(rec["tau_mm"][far]))


@pytest.mark.parametrize("tof", [False, True])
@pytest.mark.parametrize("subsets", [(0, 1), (2, 5)])
def test_projector_and_backprojector_are_adjoint(tof, subsets):
    w, pd, *_ = tiny()
    sino = W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": 20.0})
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (sino.n_plane, pd.ny, pd.nx))
    shape = (sino.n_tof,) * tof + (sino.n_plane, sino.n_view, sino.n_rad)
    y = rng.uniform(0, 1, shape)
    s, n = subsets
    px = O.recon_project(w.scanner, sino, pd, x, tof=tof, subset=s, n_subsets=n)
    pty = O.recon_backproject(w.scanner, sino, pd, y, tof=tof, subset=s, n_subsets=n)
    lhs, rhs = float((px * y).sum()), float((x * pty).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs), (lhs, rhs)
    # only the subset's views are projected
    views = np.arange(sino.n_view)
    off = views % n != s
    assert np.all(px[..., off, :] == 0) and np.any(px[..., ~off, :] != 0)


def blob(pd, n_plane, c, sig, amp=1.0):
    x = pd.lo_mm[0] + (np.arange(pd.nx) + 0.5) * pd.voxel_mm[0]
    y = pd.lo_mm[1] + (np.arange(pd.ny) + 0.5) * pd.voxel_mm[1]
    g = amp * np.exp(-((x[None, :] - c[0]) ** 2 + (y[:, None] - c[1]) ** 2) / (2 * sig * sig))
    return np.broadcast_to(g, (n_plane, pd.ny, pd.nx)).copy()


def test_line_integrals_of_a_gaussian_blob():
    w, *_ = tiny()
    pd = fine_grid()
    c, sig = np.array([14.0, -9.0]), 8.0
    img = blob(pd, w.sino.n_plane, c, sig)
    y = O.recon_project(w.scanner, w.sino, pd, img, tof=False)[0]
    _, _, m, u = lor_geometry(w.scanner, w.sino.n_rad)
    rel = c[None, None, :] - m
    d = rel[..., 0] * u[..., 1] - rel[..., 1] * u[..., 0]
    expect = sig * math.sqrt(2 * math.pi) * np.exp(-d * d / (2 * sig * sig))
    # linear interpolation on pixels of h = 1.33 mm errs by about
    # h^2/8 |f''/f| = h^2 |d^2 - sig^2| / (8 sig^4): below 0.8 % where the
    # integral is above a fifth of its maximum (d < 1.8 sig)
    big = expect > 0.2 * expect.max()
    err = np.abs(y[big] - expect[big]) / expect[big]
    assert err.max() < 0.01, err.max()
    assert np.all(np.abs(y[~big] - expect[~big]) < 0.01 * expect.max())


def test_tof_bins_without_timing_error_split_the_line_integral():
    """With no timing error every sample goes to the bin holding its TOF
    coordinate: the TOF bins of an LOR sum to its line integral (inside the
    TOF range), and the blob's mass sits in the bins around the centre's
    projection."""
    w, *_ = tiny()
    pd = fine_grid()
    sino = W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": 0.0})
    c, sig = np.array([-22.0, 11.0]), 6.0
    img = blob(pd, sino.n_plane, c, sig)
    yt = O.recon_project(w.scanner, sino, pd, img, tof=True)
    y = O.recon_project(w.scanner, sino, pd, img, tof=False)
    np.testing.assert_allclose(yt.sum(0), y, rtol=1e-12, atol=1e-12)
    _, _, m, u = lor_geometry(w.scanner, sino.n_rad)
    s_c = ((c[None, None, :] - m) * u).sum(-1)
    wb = sino.tof_bin_mm
    big = y[0] > 0.2 * y[0].max()
    centres = (np.arange(sino.n_tof) - 0.5 * sino.n_tof + 0.5) * wb
    mean = (yt[:, 0][:, big] * centres[:, None]).sum(0) / yt[:, 0][:, big].sum(0)
    assert np.abs(mean - s_c[big]).max() < 0.5 * wb


@pytest.mark.parametrize("tof_sigma", [12.0, 24.19])
def test_tof_profile_of_a_gaussian_blob(tof_sigma):
    w, *_ = tiny()
    pd = fine_grid()
    sino = W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": tof_sigma})
    c, sig = np.array([-22.0, 11.0]), 6.0
    img = blob(pd, sino.n_plane, c, sig)
    y = O.recon_project(w.scanner, sino, pd, img, tof=True)[:, 0]  # [tof][view][rad] of plane 0
    _, _, m, u = lor_geometry(w.scanner, sino.n_rad)
    rel = c[None, None, :] - m
    d = rel[..., 0] * u[..., 1] - rel[..., 1] * u[..., 0]
    s_c = (rel * u).sum(-1)
    total = sig * math.sqrt(2 * math.pi) * np.exp(-d * d / (2 * sig * sig))
    se = math.sqrt(sig * sig + tof_sigma * tof_sigma)
    wb = sino.tof_bin_mm
    lo = (np.arange(sino.n_tof) - 0.5 * sino.n_tof) * wb
    cdf = lambda z: 0.5 * (1 + special.erf(z / math.sqrt(2)))  # noqa: E731
    frac = cdf((lo[:, None, None] + wb - s_c[None]) / se) - cdf((lo[:, None, None] - s_c[None]) / se)
    expect = total[None] * frac
    big = total > 0.2 * total.max()
    err = np.abs(y[:, big] - expect[:, big]).max(axis=0) / total[big]
    assert err.max() < 0.01, err.max()
    # the mean TOF coordinate is the blob centre's projection on the LOR
    centres = lo + 0.5 * wb
    mean = (y[:, big] * centres[:, None]).sum(0) / y[:, big].sum(0)
    inside = np.abs(s_c[big]) < 0.5 * sino.n_tof * wb - 4 * se
    assert np.abs(mean[inside] - s_c[big][inside]).max() < 0.05 * wb + 0.3


def smooth_phantom(pd, n_plane):
    img = blob(pd, n_plane, np.array([10.0, 5.0]), 14.0, 1.0)
    img += blob(pd, n_plane, np.array([-25.0, -15.0]), 7.0, 2.0)
    img += 0.3 * blob(pd, n_plane, np.array([0.0, 0.0]), 30.0, 1.0)
    img *= (1.0 + 0.2 * np.arange(n_plane) / n_plane)[:, None, None]
    return img


def loop_inputs(w, pd, img):
    sino = W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": 20.0})
    att = np.exp(-O.recon_project(w.scanner, sino, pd, 0.0096 * (img > 0.05).astype(float), tof=False))
    sens = W.make_sensitivity(sino, seed=3, tof_axis=False)
    mult = att * sens
    fwd = O.recon_project(w.scanner, sino, pd, img, tof=True)
    add = 0.3 * fwd.mean() * np.ones_like(fwd)
    return sino, mult, add, mult[None] * fwd + add


def test_true_image_is_a_fixed_point_of_the_osem_update():
    w, pd, *_ = tiny()
    x = smooth_phantom(pd, w.sino.n_plane)
    sino, mult, add, prompts = loop_inputs(w, pd, x)
    x1 = O.recon_osem(w.scanner, sino, pd, prompts, mult, add, x, n_iter=1, n_subsets=4)
    nz = x > 1e-9
    np.testing.assert_allclose(x1[nz], x[nz], rtol=1e-10)


def test_osem_recovers_a_smooth_phantom_from_noiseless_data():
    """TOF-OSEM with attenuation, a detector pattern and an additive
    background, from a uniform image: the error to the true image falls with
    the iterations and ends below 5 % (relative L2 over the object)."""
    w, pd, *_ = tiny()
    x_true = smooth_phantom(pd, w.sino.n_plane)
    sino, mult, add, prompts = loop_inputs(w, pd, x_true)
    x = np.ones_like(x_true) * x_true.mean()
    errs = []
    for _ in range(6):
        x = O.recon_osem(w.scanner, sino, pd, prompts, mult, add, x, n_iter=4, n_subsets=4)
        errs.append(float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true)))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.05, errs
