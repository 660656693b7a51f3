"""Pins of the oracle's scattered photon: the change of direction at an
interaction and the free path of a photon below 511 keV.

The paper leaves the transport physics to its simulator (Methods, "Scatter
simulator description"); the oracle's readings are a rotation of the
direction by the sampled polar angle and a uniform azimuth, and Woodcock
steps against the majorant mu_max g(E) with attenuation mu511(x) g(E) at the
photon's current energy.  These tests tie both to the mathematics, not to a
second copy of the same formula:
  - rotate: unit length, the polar angle to the old direction, and an
    azimuth that advances with phi about the old direction (right-handed,
    uniform) in a frame the test builds for itself, near and on the axis too;
  - free path at E < 511 keV: interaction-free escapes from a uniform water
    box equal exp(-mu511 g(E) l) with exact chords and g(E) from the
    closed-form Klein-Nishina model, with the natural and a 3x majorant.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
import workloads as W
from tests import refgeom as G

VARIANTS = [("f32", 1e-6), ("f64", 1e-12)]


def _frame(u):
    """An orthonormal pair perpendicular to u (Gram-Schmidt from the axis u is
    least aligned with), in binary64."""
    u = u / np.linalg.norm(u)
    a = np.zeros(3)
    a[np.argmin(np.abs(u))] = 1.0
    f1 = a - u * (a @ u)
    f1 /= np.linalg.norm(f1)
    f2 = np.cross(u, f1)
    return u, f1, f2


def _stored(u, variant):
    """u as the build holds it (rounded to binary32 in the binary32 build)."""
    u = np.asarray(u, np.float64)
    return u.astype(np.float32).astype(np.float64) if variant == "f32" else u


def _directions(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    near = []
    for eps in (4e-3, 1e-3, 1e-5, 1e-8, 1e-12, 0.0):
        for sgn in (1.0, -1.0):
            a = rng.uniform(0, 2 * np.pi)
            near.append([eps * math.cos(a), eps * math.sin(a), sgn * math.sqrt(1.0 - eps * eps)])
    return np.vstack([v, np.array(near)])


@pytest.mark.parametrize("variant,tol", VARIANTS)
def test_rotate_keeps_unit_length_and_turns_by_the_polar_angle(variant, tol):
    rng = np.random.default_rng(11)
    us = _directions(rng, 400)
    worst_norm = worst_cos = 0.0
    for u in us:
        for ct in (-1.0, -0.7, -1e-3, 0.0, 0.3, 0.8, 0.999, 1.0 - 2.0 ** -20, 1.0, rng.uniform(-1, 1)):
            phi = rng.uniform(0, 2 * np.pi)
            d = O.rotate(u, ct, math.cos(phi), math.sin(phi), variant)
            ur = _stored(u, variant)
            worst_norm = max(worst_norm, abs(np.linalg.norm(d) - 1.0))
            worst_cos = max(worst_cos, abs(d @ (ur / np.linalg.norm(ur)) - ct))
    assert worst_norm < tol, worst_norm
    # the binary32 polar cosine of the new direction is the sampled one up to
    # a few roundings of unit quantities (sqrt(1 - ct^2) amplifies none)
    assert worst_cos < (2e-6 if variant == "f32" else 1e-12), worst_cos


@pytest.mark.parametrize("variant", ["f32", "f64"])
def test_rotate_azimuth_advances_with_phi_about_the_old_direction(variant):
    """In a frame (f1, f2, u) the test builds itself, the new direction's
    azimuth psi = atan2(d.f2, d.f1) is phi plus a constant for each u: the
    rotation is right-handed about u (phi and psi increase together) and
    maps a uniform phi to a uniform psi."""
    rng = np.random.default_rng(12)
    us = _directions(rng, 60)
    tol = 2e-5 if variant == "f32" else 1e-10
    for u in us:
        _, f1, f2 = _frame(_stored(u, variant))
        ct = rng.uniform(-0.9, 0.9)
        phis = np.sort(rng.uniform(0, 2 * np.pi, 24))
        off = []
        for phi in phis:
            d = O.rotate(u, ct, math.cos(phi), math.sin(phi), variant)
            psi = math.atan2(d @ f2, d @ f1)
            off.append(math.remainder(psi - phi, 2 * math.pi))
        off = np.array(off)
        spread = np.abs(np.remainder(off - off[0] + math.pi, 2 * math.pi) - math.pi)
        assert spread.max() < tol / math.sqrt(1 - ct * ct), (u, spread.max())


def test_rotate_orientation_at_the_axis():
    """On the axis the frame is fixed: (x, y) about +z, (x, -y) about -z."""
    st, ct = math.sqrt(1 - 0.36), 0.6
    for variant in ("f32", "f64"):
        d = O.rotate([0.0, 0.0, 1.0], ct, 1.0, 0.0, variant)
        np.testing.assert_allclose(d, [st, 0.0, ct], atol=1e-7)
        d = O.rotate([0.0, 0.0, 1.0], ct, 0.0, 1.0, variant)
        np.testing.assert_allclose(d, [0.0, st, ct], atol=1e-7)
        d = O.rotate([0.0, 0.0, -1.0], ct, 0.0, 1.0, variant)
        np.testing.assert_allclose(d, [0.0, -st, -ct], atol=1e-7)
        # off the axis: turning (1, 0, 0) by phi = 0 tilts it towards -z
        d = O.rotate([1.0, 0.0, 0.0], ct, 1.0, 0.0, variant)
        np.testing.assert_allclose(d, [ct, 0.0, -st], atol=1e-7)


def test_rotate_with_sampled_azimuths_is_uniform_about_the_direction():
    """Azimuths drawn the way the transport draws them (2 pi u through the
    binary32 sine and cosine) give a uniform azimuth about a fixed old
    direction (chi-square, 36 bins)."""
    rng = np.random.default_rng(13)
    u = np.array([0.3, -0.5, 0.8])
    u /= np.linalg.norm(u)
    _, f1, f2 = _frame(_stored(u, "f32"))
    n = 20_000
    uu = np.array([O.u01(int(x)) for x in rng.integers(0, 2 ** 32, n, dtype=np.uint64)], np.float32)
    sn, cs = O.sincos_2pi(uu)
    psi = np.empty(n)
    for i in range(n):
        d = O.rotate(u, 0.25, float(cs[i]), float(sn[i]))
        psi[i] = math.atan2(d @ f2, d @ f1)
    hist, _ = np.histogram(np.mod(psi, 2 * np.pi), bins=36, range=(0, 2 * np.pi))
    chi2 = ((hist - n / 36) ** 2 / (n / 36)).sum()
    assert stats.chi2.sf(chi2, 35) > 1e-5, chi2


@pytest.mark.parametrize("e_kev", [300.0, 450.0])
@pytest.mark.parametrize("majorant_factor", [0.0, 3.0])
def test_free_path_below_511_kev_follows_beer_lambert(e_kev, majorant_factor):
    """Photons of energy E started uniformly inside a uniform water box in
    isotropic directions leave it without a real interaction with
    probability exp(-mu511 g(E) l), l the exact chord to the box's face and
    g(E) the attenuation model's closed form; a z-test on the count, with the
    phantom maximum and with three times it as the Woodcock majorant."""
    w = W.WORKLOADS["tiny"]
    mu_w = np.float32(W.MU_WATER)
    pd, mu, _ = W.uniform_box(n=(6, 5, 4), voxel_mm=(16.0, 18.0, 20.0), mu=float(mu_w))
    phys = dict(w.physics, mu_majorant=float(mu_w) * majorant_factor, e_kill_kev=100.0)
    n = 60_000
    rng = np.random.default_rng(int(e_kev) + int(10 * majorant_factor))
    lo = np.array(pd.lo_mm, np.float64)
    hi = lo + np.array([pd.nx, pd.ny, pd.nz]) * np.array(pd.voxel_mm)
    p0 = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32).astype(np.float64)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = d.astype(np.float32).astype(np.float64)
    rec = O.transport_photons(w.scanner, phys, pd, mu, p0, d, e_kev, seed=31)
    g = O.energy_model(phys, e_kev)[0]
    chord = G.box_chord(p0, d, lo, hi) * np.linalg.norm(d, axis=1)
    p = np.exp(-float(mu_w) * g * chord)
    fate = rec["inter"] >> 16
    clean = ((rec["inter"] & 0xFFFF) == 0) & ((fate == O.FATE["detected"]) | (fate == O.FATE["axial"]))
    obs = int(clean.sum())
    z = (obs - p.sum()) / math.sqrt((p * (1 - p)).sum())
    assert abs(z) < 4.5, (obs, p.sum(), z)
    # the same test with the 511 keV attenuation must fail: the energy
    # dependence is visible at this sample size
    p511 = np.exp(-float(mu_w) * O.energy_model(phys, 510.99895)[0] * chord)
    z511 = (obs - p511.sum()) / math.sqrt((p511 * (1 - p511)).sum())
    assert abs(z511) > 6.0, z511
    # energies are unchanged on interaction-free paths
    assert np.all(rec["e_kev"][clean] == np.float32(e_kev))
