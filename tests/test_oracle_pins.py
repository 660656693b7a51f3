"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself:
published known answers (Philox), closed forms (Beer-Lambert survival with
exact chords, point-source geometric efficiency, Klein-Nishina total cross
section vs its differential form), distributions (chi-square of the Compton
and emission samplers), exact invariants (alias-table masses, all-ones LUT,
mu = 0 => no scatter, weight-or-discard), and brute-force recomputation of
crystal / ring / LUT / sinogram / TOF indices from raw hit data.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
import workloads as W
from tests import refgeom as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run(scanner, sino, physics, pd, mu, act, lut_desc, lut, n, seed=7, **kw):
    return O.simulate(scanner, sino, physics, pd, mu, activity=act, lut_desc=lut_desc, lut=lut,
                      seed=seed, n=n, **kw)


def tiny_setup():
    w = W.WORKLOADS["tiny"]
    pd, mu, act = W.make_phantom(w)
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    return w, pd, mu, act, ld, lut


def ztest(observed, expected, var, limit=4.5):
    z = (observed - expected) / math.sqrt(var)
    assert abs(z) < limit, (observed, expected, z)
    return z


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    n = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            vals = [int(x, 16) for x in parts[2:]]
            out = O.philox(vals[0:4], vals[4:6])
            assert list(out) == vals[6:10]
            n += 1
    assert n == 3


def test_uniform_conversion_is_open_and_symmetric():
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 2**32, size=2000, dtype=np.uint64)
    assert O.u01(0) == 2.0**-24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0**-24
    for x in xs:
        u = O.u01(int(x))
        assert 0.0 < u < 1.0
        assert u + O.u01(int(x) ^ 0xFFFFFFFF) == 1.0


def test_free_path_logarithm_is_faithful_for_every_uniform():
    """The binary32 -ln(u) of the Woodcock step, over all 2^23 values the
    uniform conversion can produce, against binary64 log: error below one
    unit in the last place everywhere, correctly rounded for most, exact at
    the ends; the binary64 oracle uses the library log itself."""
    m = np.arange(1 << 23, dtype=np.float64) * 2.0 + 1.0
    u = (m * 2.0**-24).astype(np.float32)
    got = O.neg_log(u)
    ref = -np.log(u.astype(np.float64))
    ref32 = ref.astype(np.float32)
    err = np.abs(got.astype(np.float64) - ref) / np.spacing(ref32).astype(np.float64)
    assert err.max() < 0.85, err.max()
    assert np.mean(got == ref32) > 0.99
    assert got[0] == np.float32(24.0 * math.log(2.0))      # u = 2^-24
    assert got[-1] == ref32[-1] and got[-1] > 0.0           # u = 1 - 2^-24
    assert np.all(np.diff(got) <= 0.0)                      # decreasing in u
    assert np.array_equal(O.neg_log(u, "f64"), ref32)


def test_free_path_log_table_is_correctly_rounded():
    """The free-path logarithm's table, recomputed in 50-digit decimal
    arithmetic from its definition: c_i the binary32 nearest 1 / mid_i (1 for
    the five entries around F = 1), hi_i = -ln(c_i) rounded to a multiple of
    2^-16, lo_i the binary32 nearest -ln(c_i) - hi_i.  Equality shows that
    the table does not depend on the platform's binary64 log."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    tab = O.log_table()
    base = 0x3F348000
    as_f32 = lambda b: float(np.array([b], np.uint32).view(np.float32)[0])
    for i in range(129):
        a, b = as_f32(base + (i << 16)), as_f32(base + ((i + 1) << 16))
        mid = (Decimal(a) + Decimal(b)) / 2
        c = np.float32(1.0) if 73 <= i <= 77 else np.float32(float(1 / mid))
        # the binary32 nearest 1/mid: the double rounding above is checked
        # against the neighbours of c
        if not 73 <= i <= 77:
            exact = 1 / mid
            for nb in (np.nextafter(c, np.float32(0)), np.nextafter(c, np.float32(2))):
                assert abs(Decimal(float(c)) - exact) <= abs(Decimal(float(nb)) - exact), i
        t = -Decimal(float(c)).ln()
        hi = (t * 65536).to_integral_value() / 65536
        lo = np.float32(float(t - hi))
        assert tab[i, 0] == c and tab[i, 1] == np.float32(float(hi)) and tab[i, 2] == lo, (i, tab[i], c, hi, lo)
    assert np.all(tab[73:78, 0] == 1.0) and np.all(tab[73:78, 1:] == 0.0)


def test_azimuth_sincos_is_accurate_for_every_uniform():
    """The binary32 (sin 2 pi u, cos 2 pi u) of the azimuth and emission
    direction, over all 2^23 uniforms, against binary64 sin and cos: error
    below 2^-23 absolute, on the unit circle to 3e-7, exact at the quadrant
    points; the binary64 oracle uses the library functions."""
    m = np.arange(1 << 23, dtype=np.float64) * 2.0 + 1.0
    u = (m * 2.0**-24).astype(np.float32)
    sn, cs = O.sincos_2pi(u)
    ph = 2.0 * np.pi * u.astype(np.float64)
    assert np.abs(sn - np.sin(ph)).max() < 2.0**-23
    assert np.abs(cs - np.cos(ph)).max() < 2.0**-23
    assert np.abs(sn.astype(np.float64) ** 2 + cs.astype(np.float64) ** 2 - 1.0).max() < 3e-7
    q_s, q_c = O.sincos_2pi(np.array([0.0, 0.25, 0.5, 0.75], np.float32))
    assert np.array_equal(q_s, [0.0, 1.0, 0.0, -1.0]) and np.array_equal(q_c, [1.0, 0.0, -1.0, 0.0])
    s64, c64 = O.sincos_2pi(u, "f64")
    assert np.array_equal(s64, np.sin(ph).astype(np.float32)) and np.array_equal(c64, np.cos(ph).astype(np.float32))


def test_binary32_energy_model_tracks_the_binary64_model():
    """The binary32 transport's g, fC and fC + fR against the binary64 model
    (itself pinned to the integrated Klein-Nishina differential) from the
    lowest accepted kill energy, 100 keV, to 511 keV."""
    phys = W.PHYSICS_DEFAULT
    for e in np.linspace(100.0, 510.99895, 1500):
        got = O.transport_coefs(phys, e)
        g, c, r = O.energy_model(phys, e)
        ref = np.array([g, c, c + r])
        assert np.all(np.abs(got - ref) / ref < 2e-5), (e, got, ref)
    g511 = O.transport_coefs(phys, 510.99895)
    assert abs(g511[0] - 1.0) < 3e-7
    assert np.allclose(O.transport_coefs(phys, 300.0, "f64"), np.array(O.energy_model(phys, 300.0))[[0, 1, 1]]
                       + np.array([0.0, 0.0, O.energy_model(phys, 300.0)[2]]), rtol=1e-7)


# ---------------------------------------------------------------------------
# emission
# ---------------------------------------------------------------------------

def alias_masses(th, al):
    th = th.astype(np.int64)
    mass = np.zeros(th.size, np.int64)
    np.add.at(mass, np.arange(th.size), th)
    np.add.at(mass, al.astype(np.int64), (1 << 32) - th)
    return mass


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_alias_table_masses_match_activity(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 500))
    act = rng.uniform(0, 5, n).astype(np.float32)
    act[rng.random(n) < 0.3] = 0.0
    if act.sum() == 0:
        act[0] = 1.0
    th, al = O.build_alias(act)
    mass = alias_masses(th, al)
    assert mass.sum() == n * (1 << 32)
    assert np.all(mass[act == 0] == 0)
    expected = act.astype(np.float64) / act.astype(np.float64).sum() * n * 2.0**32
    assert np.max(np.abs(mass - expected)) <= n + 2


def test_alias_rejects_bad_activity():
    with pytest.raises(ValueError):
        O.build_alias(np.zeros(10, np.float32))
    with pytest.raises(ValueError):
        O.build_alias(np.array([1.0, -1.0], np.float32))


def test_emitted_voxels_follow_activity():
    rng = np.random.default_rng(5)
    pd = W.centred_desc((4, 4, 4), (10.0, 10.0, 10.0))
    act = rng.uniform(0, 1, pd.shape).astype(np.float32)
    act[0, 0, :2] = 0.0
    mu = np.zeros(pd.shape, np.float32)
    w, _, _, _, ld, lut = tiny_setup()
    n = 200_000
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, records=True, sinograms=False)
    counts = np.bincount(r["records"]["voxel"], minlength=act.size)
    p = act.ravel().astype(np.float64) / act.sum()
    assert np.all(counts[p == 0] == 0)
    nz = p > 0
    chi2 = ((counts[nz] - n * p[nz]) ** 2 / (n * p[nz])).sum()
    assert stats.chi2.sf(chi2, nz.sum() - 1) > 1e-5


def test_emission_position_and_direction_distribution():
    pd = W.centred_desc((3, 2, 5), (7.0, 3.0, 5.0))
    act = np.ones(pd.shape, np.float32)
    th, al = O.build_alias(act)
    n = 40_000
    frac, cos_t, phi, norm = [], [], [], []
    for h in range(n):
        v, pos, d = O.emit(pd, th, al, 99, h)
        ix, iy, iz = v % pd.nx, (v // pd.nx) % pd.ny, v // (pd.nx * pd.ny)
        frac.append((pos[0] - pd.lo_mm[0]) / pd.voxel_mm[0] - ix)
        frac.append((pos[1] - pd.lo_mm[1]) / pd.voxel_mm[1] - iy)
        frac.append((pos[2] - pd.lo_mm[2]) / pd.voxel_mm[2] - iz)
        nd = np.linalg.norm(d)
        norm.append(nd)
        cos_t.append(d[2] / nd)
        phi.append(math.atan2(d[1], d[0]))
    assert stats.kstest(np.clip(frac, 0, 1), "uniform").pvalue > 1e-4
    assert stats.kstest(np.array(cos_t), "uniform", args=(-1, 2)).pvalue > 1e-4
    assert stats.kstest(np.array(phi), "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-4
    assert np.max(np.abs(np.array(norm) - 1)) < 1e-6


# ---------------------------------------------------------------------------
# interaction physics
# ---------------------------------------------------------------------------

R_E2 = 1.0  # units of r_e^2


def kn_dsigma_dcos(c, alpha):
    """Klein-Nishina: dsigma/dOmega = r_e^2/2 eps^2 (eps + 1/eps - sin^2),
    eps = E'/E = 1 / (1 + alpha (1 - cos)); times 2 pi for d cos."""
    eps = 1.0 / (1.0 + alpha * (1.0 - c))
    return 2 * math.pi * 0.5 * R_E2 * eps * eps * (eps + 1.0 / eps - (1.0 - c * c))


@pytest.mark.parametrize("e_kev", [510.99895, 425.0, 300.0])
def test_compton_angles_follow_klein_nishina(e_kev):
    n = 300_000
    ct, e_out = O.sample_compton(11, e_kev, n)
    alpha = np.float32(e_kev) / np.float32(510.99895)
    edges = np.linspace(-1, 1, 101)
    hist, _ = np.histogram(ct, edges)
    probs = np.array([integrate.quad(kn_dsigma_dcos, a, b, args=(float(alpha),))[0]
                      for a, b in zip(edges[:-1], edges[1:])])
    probs /= probs.sum()
    chi2 = ((hist - n * probs) ** 2 / (n * probs)).sum()
    assert stats.chi2.sf(chi2, len(hist) - 1) > 1e-5, chi2
    # Compton kinematics E' = E / (1 + alpha (1 - cos))
    expect = e_kev / (1.0 + float(alpha) * (1.0 - ct))
    assert np.max(np.abs(e_out - expect) / expect) < 2e-6


def test_klein_nishina_total_matches_integrated_differential():
    phys = dict(W.PHYSICS_DEFAULT, f_compton=1.0, f_rayleigh=0.0, f_photo=0.0)
    total = lambda a: integrate.quad(kn_dsigma_dcos, -1, 1, args=(a,), epsabs=0, epsrel=1e-13)[0]
    ref511 = total(1.0)
    for e in [150.0, 300.0, 425.0, 510.99895, 600.0]:
        g, c, r = O.energy_model(phys, e)
        assert r == 0.0 and g == c
        assert abs(c - total(e / 510.99895) / ref511) < 1e-10, e


def test_energy_model_split_at_511():
    g, c, r = O.energy_model(W.PHYSICS_DEFAULT, 510.99895)
    p = W.PHYSICS_DEFAULT
    assert abs(g - 1.0) < 1e-7
    assert abs(c - np.float32(p["f_compton"])) < 1e-12
    assert abs(r - np.float32(p["f_rayleigh"])) < 1e-12


def test_rayleigh_angles_follow_model_pdf():
    """Self-consistency of the Rayleigh sampler with its analytic model
    (Thomson factor times (1 + beta' t)^-2, t = 1 - cos); the model itself
    is a reading, not a paper value."""
    n = 200_000
    beta = 1000.0
    e = 460.0
    ct = O.sample_rayleigh(13, e, beta, n)
    a = np.float32(e) / np.float32(510.99895)
    bp = beta * a * a
    pdf = lambda t: (1.0 + (1.0 - t) ** 2) / (1.0 + bp * t) ** 2
    edges = np.concatenate([[0.0], np.geomspace(1e-6, 2.0, 60)])
    t = 1.0 - ct
    hist, _ = np.histogram(t, edges)
    probs = np.array([integrate.quad(pdf, lo, hi, epsrel=1e-10)[0] for lo, hi in zip(edges[:-1], edges[1:])])
    probs /= probs.sum()
    keep = n * probs > 5
    chi2 = ((hist[keep] - n * probs[keep]) ** 2 / (n * probs[keep])).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-5, chi2


@pytest.mark.parametrize("variant", ["f32", "f64"])
def test_rayleigh_sampler_reduces_to_thomson_without_form_factor(variant):
    """With the form factor switched off (beta -> 0) the Rayleigh sampler must
    draw the classical Thomson distribution, pdf (3/8)(1 + cos^2) on [-1, 1]
    (CDF (3c + c^3 + 4) / 8): a textbook law that the sampler's inversion and
    rejection steps only reach together, so a wrong rejection test, a wrong
    inversion or a lost sign fails it.  Pinned by Kolmogorov-Smirnov and by
    the first three moments (E c = 0, E c^2 = 2/5, E c^3 = 0)."""
    n = 200_000
    ct = O.sample_rayleigh(29, 480.0, 1e-6, n, variant=variant)
    assert np.all((ct >= -1.0) & (ct <= 1.0))
    cdf = lambda c: (3.0 * c + c ** 3 + 4.0) / 8.0
    assert stats.kstest(ct, cdf).pvalue > 1e-5
    se = 1.0 / math.sqrt(n)
    assert abs(ct.mean()) < 5 * se * math.sqrt(0.4)
    assert abs((ct ** 2).mean() - 0.4) < 5 * se * 0.35
    assert abs((ct ** 3).mean()) < 5 * se * 0.55


# ---------------------------------------------------------------------------
# Woodcock transport: Beer-Lambert survival
# ---------------------------------------------------------------------------

def unscattered_escapes(rec, k):
    inter = rec["ph"][:, k]["inter"]
    fate = inter >> 16
    return ((inter & 0xFFFF) == 0) & ((fate == O.FATE["detected"]) | (fate == O.FATE["axial"]))


@pytest.mark.parametrize("majorant_factor", [0.0, 3.0])
def test_beer_lambert_uniform_box_exact_chords(majorant_factor):
    w, _, _, _, ld, lut = tiny_setup()
    mu_w = np.float32(W.MU_WATER)
    pd, mu, act = W.uniform_box(n=(6, 5, 4), voxel_mm=(16.0, 18.0, 20.0), mu=float(mu_w))
    phys = dict(w.physics, mu_majorant=float(mu_w) * majorant_factor)
    n = 100_000
    r = run(w.scanner, w.sino, phys, pd, mu, act, ld, lut, n, records=True, sinograms=False, seed=21)
    th, al = O.build_alias(act)
    pos = np.zeros((n, 3))
    d = np.zeros((n, 3))
    for h in range(n):
        _, pos[h], d[h] = O.emit(pd, th, al, 21, h)
    lo = np.array(pd.lo_mm)
    hi = lo + np.array([pd.nx, pd.ny, pd.nz]) * np.array(pd.voxel_mm)
    g511 = O.energy_model(phys, 510.99895)[0]
    for k, sgn in ((0, 1.0), (1, -1.0)):
        chord = G.box_chord(pos, sgn * d, lo, hi) * np.linalg.norm(d, axis=1)
        p = np.exp(-float(mu_w) * g511 * chord)
        obs = unscattered_escapes(r["records"], k).sum()
        ztest(obs, p.sum(), (p * (1 - p)).sum())


def test_beer_lambert_voxelised_water_cylinder_siddon():
    w, pd, mu, act, ld, lut = tiny_setup()
    n = 100_000
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, records=True, sinograms=False, seed=5)
    th, al = O.build_alias(act)
    pos = np.zeros((n, 3))
    d = np.zeros((n, 3))
    for h in range(n):
        _, pos[h], d[h] = O.emit(pd, th, al, 5, h)
    nd = np.linalg.norm(d, axis=1)
    integral = G.siddon_line_integral(pos, d, mu, pd.lo_mm, pd.voxel_mm) * nd
    p = np.exp(-integral)
    obs = unscattered_escapes(r["records"], 0).sum()
    ztest(obs, p.sum(), (p * (1 - p)).sum())
    # sanity: the pencil survival through 50 mm of water
    assert abs(math.exp(-0.0096 * 50) - 0.6188) < 1e-4


# ---------------------------------------------------------------------------
# detection geometry
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("z0", [0.0, 30.0])
@pytest.mark.parametrize("which", ["tiny", "clinical"])
def test_point_source_in_air_geometric_efficiency(z0, which):
    """On-axis point source at height z0 in air: both photons reach the
    cylinder inside its length iff |cos theta| < h / sqrt(R^2 + h^2),
    h = L/2 - |z0|, and cos theta is uniform."""
    w = W.WORKLOADS[which]
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    pd, mu, act = W.point_source((0.0, 0.0, z0))
    n = 200_000
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, records=True, sinograms=False, seed=3)
    fate = r["records"]["ph"]["inter"] >> 16
    both = ((fate[:, 0] == 0) & (fate[:, 1] == 0)).sum()
    single = (fate[:, 0] == 0).sum()
    R = w.scanner.radius_mm
    h = w.scanner.length_mm / 2 - abs(z0)
    p = h / math.sqrt(R * R + h * h)
    ztest(both, n * p, n * p * (1 - p))
    hs = w.scanner.length_mm / 2
    ps = 0.5 * ((hs - z0) / math.hypot(R, hs - z0) + (hs + z0) / math.hypot(R, hs + z0))
    ztest(single, n * ps, n * ps * (1 - ps))


def test_centre_point_source_bins_to_central_radial_and_tof():
    for which in ("tiny", "clinical"):
        w = W.WORKLOADS[which]
        sino = W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": 0.0})
        ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
        pd, mu, act = W.point_source((0.0, 0.0, 0.0))
        r = run(w.scanner, sino, w.physics, pd, mu, act, ld, lut, 50_000, records=True, trues=True)
        rec = r["records"]
        counted = (rec["outcome"] & 0xFF) == O.OUTCOME["true"]
        assert counted.sum() > 10_000
        rc = rec[counted]
        b = O.record_bins(rc)
        rad = b % sino.n_rad
        tof = b // (sino.n_rad * sino.n_view * sino.n_plane)
        # the source is within 1 um of the centre: a hit on a crystal
        # boundary may land one crystal over; nothing else may
        near = np.zeros(len(rc), bool)
        for k in range(2):
            _, f = G.crystal_of(rc["ph"][:, k]["hx"].astype(np.float64), rc["ph"][:, k]["hy"].astype(np.float64),
                                w.scanner.n_crystals)
            near |= np.abs(f - np.rint(f)) < 1e-3
        assert np.all((rad == (sino.n_rad - 1) // 2) | near)
        assert (rad != (sino.n_rad - 1) // 2).sum() <= 5
        assert np.all(tof == sino.n_tof // 2)
        assert r["scatter_counts"].sum() == 0


def test_no_attenuation_means_no_scatter():
    w, pd, mu, act, ld, lut = tiny_setup()
    r = run(w.scanner, w.sino, w.physics, pd, np.zeros_like(mu), act, ld, lut, 50_000, trues=True)
    assert r["scatter_counts"].sum() == 0 and r["scatter_weights"].sum() == 0.0
    assert r["stats"]["compton"] == 0 and r["stats"]["real"] == 0
    assert r["true_counts"].sum() > 0


# ---------------------------------------------------------------------------
# LUT weighting and list-mode invariants
# ---------------------------------------------------------------------------

def test_all_ones_lut_reproduces_unweighted_counts():
    w, pd, mu, act, ld, _ = tiny_setup()
    ones = np.ones(ld.dims, np.float32)
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, ones, 100_000, trues=True)
    assert r["scatter_counts"].sum() > 0
    assert np.array_equal(r["scatter_weights"], r["scatter_counts"].astype(np.float64))
    assert np.array_equal(r["true_weights"], r["true_counts"].astype(np.float64))


def test_weight_or_discard_invariant():
    w, pd, mu, act, ld, lut = tiny_setup()
    n = 100_000
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, trues=True)
    total = int(r["scatter_counts"].sum()) + int(r["true_counts"].sum())
    assert total == r["stats"]["scatter"] + r["stats"]["true"] <= n
    for cnt, wt in ((r["scatter_counts"], r["scatter_weights"]), (r["true_counts"], r["true_weights"])):
        c = cnt.astype(np.float64)
        assert np.all(wt <= c * (1 + 1e-12))
        lo = float(lut.min()) ** 2
        assert np.all(wt >= c * lo * (1 - 1e-6))


def test_one_hot_lut_selects_exactly_that_entry():
    w, pd, mu, act, ld, _ = tiny_setup()
    n = 60_000
    base = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, np.ones(ld.dims, np.float32), n,
               records=True, trues=True)
    rec = base["records"]
    counted = (rec["outcome"] & 0xFF) <= 1
    idx = rec["ph"]["lut_index"][counted]
    target = np.bincount(idx.ravel()).argmax()
    hot = np.zeros(int(np.prod(ld.dims)), np.float32)
    hot[target] = 1.0
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, hot, n, trues=True)
    both = (idx[:, 0] == target) & (idx[:, 1] == target)
    assert np.isclose(r["scatter_weights"].sum() + r["true_weights"].sum(), both.sum())


@pytest.mark.parametrize("which", ["tiny", "clinical_scanner"])
def test_indices_match_brute_force_geometry(which):
    """Crystal, ring, LUT and sinogram indices and the TOF offset of every
    counted coincidence, recomputed from the raw hit data in binary64."""
    w, pd, mu, act, ld, lut = tiny_setup()
    scanner, sino = w.scanner, w.sino
    if which == "clinical_scanner":
        wc = W.WORKLOADS["clinical"]
        scanner = wc.scanner
        sino = W.Sinogram(**{**wc.sino.__dict__, "tof_sigma_mm": 0.0})
        ld, lut = W.make_lut(wc.lut_dims, wc.lut_seed)
    n = 100_000
    r = run(scanner, sino, w.physics, pd, mu, act, ld, lut, n, records=True, trues=True, seed=17)
    rec = r["records"]
    counted = (rec["outcome"] & 0xFF) <= 1
    rc = rec[counted]
    assert len(rc) > 1000
    ph = rc["ph"]
    nE, nt, na, nct, nca = ld.dims
    ok_lut = 0
    cr = {}
    for k in range(2):
        p = ph[:, k]
        h = np.stack([p["hx"], p["hy"], p["hz"]], 1).astype(np.float64)
        d = np.stack([p["dx"], p["dy"], p["dz"]], 1).astype(np.float64)
        # hit point on the cylinder
        assert np.max(np.abs(np.hypot(h[:, 0], h[:, 1]) - scanner.radius_mm)) < 1e-3
        c, fc = G.crystal_of(h[:, 0], h[:, 1], scanner.n_crystals)
        rg, fr = G.ring_of(h[:, 2], scanner.length_mm, scanner.n_rings)
        rec_c = p["crystal_ring"] & 0xFFFF
        rec_r = p["crystal_ring"] >> 16
        near_c = np.abs(fc - np.rint(fc)) < 1e-5
        near_r = np.abs(fr - np.rint(fr)) < 1e-5
        assert np.all((rec_c == c) | near_c)
        assert np.all((rec_r == rg) | near_r)
        cr[k] = (rec_c.astype(np.int64), rec_r.astype(np.int64))
        fe = (p["e_kev"].astype(np.float64) - ld.e_min_kev) * nE / (ld.e_max_kev - ld.e_min_kev)
        ie = np.clip(np.floor(fe).astype(np.int64), 0, nE - 1)
        it, ft, ia, fa = G.angle_bins(h, d, nt, na)
        ct = (rec_c % scanner.crystals_per_module) * nct // scanner.crystals_per_module
        ca = (rec_r % scanner.rings_per_block) * nca // scanner.rings_per_block
        flat = (((ie * nt + it) * na + ia) * nct + ct) * nca + ca
        near = ((np.abs(fe - np.rint(fe)) < 1e-4) | (np.abs(ft - np.rint(ft)) < 1e-5)
                | (np.abs(fa - np.rint(fa)) < 1e-5))
        assert np.all((p["lut_index"] == flat) | near)
        ok_lut += int((p["lut_index"] == flat).sum())
        # weight factor is the LUT entry
    assert ok_lut > 0.999 * 2 * len(rc)
    w_expect = lut.ravel()[ph[:, 0]["lut_index"]] * lut.ravel()[ph[:, 1]["lut_index"]]
    assert np.array_equal(rc["weight"], w_expect.astype(np.float32))
    # sinogram coordinates from crystal-centre geometry
    view, rho, a_pos, _ = G.lor_geometry(cr[0][0], cr[1][0], scanner.n_crystals, scanner.radius_mm)
    b = O.record_bins(rc)
    nr, nv, npl = sino.n_rad, sino.n_view, sino.n_plane
    assert np.array_equal(b % nr, rho + (nr - 1) // 2)
    assert np.array_equal((b // nr) % nv, view)
    assert np.array_equal((b // (nr * nv)) % npl, cr[0][1] + cr[1][1])
    # TOF offset: half the path difference toward the TOF-positive end
    pa, pb = ph[:, 0]["path_mm"].astype(np.float64), ph[:, 1]["path_mm"].astype(np.float64)
    tau = np.where(a_pos, (pb - pa) / 2, (pa - pb) / 2)
    assert np.max(np.abs(tau - rc["tau_mm"])) < 1e-3
    ft = tau / sino.tof_bin_mm + sino.n_tof / 2
    tof = np.floor(ft).astype(np.int64)
    near = np.abs(ft - np.rint(ft)) < 1e-4
    assert np.all((b // (nr * nv * npl) == tof) | near)


def test_lor_mapping_is_a_bijection_with_geometric_meaning():
    for n in (64, 448):
        seen = set()
        c1, c2 = np.triu_indices(n, 1)
        views = np.zeros(len(c1), np.int64)
        rhos = np.zeros(len(c1), np.int64)
        apos = np.zeros(len(c1), bool)
        for i, (a, b) in enumerate(zip(c1, c2)):
            v, r, p = O.lor(n, int(a), int(b))
            views[i], rhos[i], apos[i] = v, r, p
            # symmetric in the crystal order except for the TOF end
            v2, r2, p2 = O.lor(n, int(b), int(a))
            assert (v2, r2) == (v, r) and p2 == 1 - p
            seen.add((v, r))
        assert len(seen) == n * (n - 1) // 2
        assert views.min() == 0 and views.max() == n // 2 - 1
        assert rhos.min() == -(n // 2 - 1) and rhos.max() == n // 2 - 1
        gv, gr, ga, _ = G.lor_geometry(c1, c2, n, 1.0)
        assert np.array_equal(gv, views) and np.array_equal(gr, rhos) and np.array_equal(ga, apos)


def test_off_centre_source_tof_offsets():
    """Source at (60, 0, 0) in air: each photon's path is its straight
    distance to the hit, and the TOF offset is the source's displacement
    from the LOR midpoint toward the TOF-positive end."""
    w = W.WORKLOADS["tiny"]
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    src = np.array([60.0, 0.0, 0.0])
    pd, mu, act = W.point_source(tuple(src))
    r = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, 30_000, records=True, trues=True)
    rec = r["records"]
    rc = rec[(rec["outcome"] & 0xFF) == O.OUTCOME["true"]]
    assert len(rc) > 5000
    h = [np.stack([rc["ph"][:, k][a] for a in ("hx", "hy", "hz")], 1).astype(np.float64) for k in range(2)]
    dist = [np.linalg.norm(h[k] - src, axis=1) for k in range(2)]
    for k in range(2):
        assert np.max(np.abs(dist[k] - rc["ph"][:, k]["path_mm"])) < 2e-3
    mid = (h[0] + h[1]) / 2
    u = (h[0] - h[1]) / np.linalg.norm(h[0] - h[1], axis=1)[:, None]
    offset_toward_a = ((src - mid) * u).sum(1)
    c1 = rc["ph"][:, 0]["crystal_ring"] & 0xFFFF
    c2 = rc["ph"][:, 1]["crystal_ring"] & 0xFFFF
    _, _, a_pos, _ = G.lor_geometry(c1.astype(np.int64), c2.astype(np.int64), w.scanner.n_crystals, w.scanner.radius_mm)
    expect = np.where(a_pos, offset_toward_a, -offset_toward_a)
    assert np.max(np.abs(expect - rc["tau_mm"])) < 2e-3


def test_binary64_transport_agrees_with_binary32():
    """The binary32 oracle takes the same decisions as the binary64 one for
    almost every history (rounding flips are rare)."""
    w, pd, mu, act, ld, lut = tiny_setup()
    n = 50_000
    a = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, records=True)["records"]
    b = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, records=True, variant="f64")["records"]
    assert O.real_size("f32") == 4 and O.real_size("f64") == 8
    same = (a["outcome"] == b["outcome"]) & (O.record_bins(a) == O.record_bins(b))
    assert same.mean() > 0.999


def test_binary32_oracle_tracks_binary64_on_the_clinical_workload():
    """One million clinical histories through both oracle builds, history by
    history: the binary32 transport takes the binary64 transport's decisions
    (interactions, steps, outcome, sinogram bin, LUT entry) for all but a
    handful of histories, its detected photons land within a few hundredths
    of a millimetre at the same energy to a few binary32 ulps, and the
    difference of the scatter totals is exactly that of the few histories
    that went another way.  This ties the binary32 arithmetic the kernel
    reproduces to the binary64 reading of the method on the workload's own
    geometry (128 x 128 x 89 phantom, 448 x 45 scanner)."""
    w = W.WORKLOADS["clinical"]
    pd, mu, act = W.make_phantom(w)
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    n = 1_000_000
    kw = dict(records=True, sinograms=False)
    a = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, **kw)["records"]
    b = run(w.scanner, w.sino, w.physics, pd, mu, act, ld, lut, n, variant="f64", **kw)["records"]
    pa, pb = a["ph"], b["ph"]
    assert np.count_nonzero(pa["inter"] != pb["inter"]) <= 10
    assert np.count_nonzero(a["n_steps"] != b["n_steps"]) <= 5
    same = (a["outcome"] == b["outcome"]) & (O.record_bins(a) == O.record_bins(b))
    assert np.count_nonzero(~same) <= 5
    det = ((pa["inter"] >> 16) == O.FATE["detected"]) & ((pb["inter"] >> 16) == O.FATE["detected"])
    assert det.sum() > 300_000
    for f, tol in (("hx", 0.05), ("hy", 0.05), ("hz", 0.05), ("path_mm", 0.05), ("e_kev", 1e-3)):
        d = np.abs(pa[f].astype(np.float64) - pb[f].astype(np.float64))[det]
        assert d.max() < tol, (f, d.max())
    counted = same & ((a["outcome"] & 0xFF) == 0)
    assert counted.sum() > 10_000
    assert np.count_nonzero(counted & (pa["lut_index"] != pb["lut_index"]).any(axis=1)) <= 5
    wa, wb = a["weight"].astype(np.float64), b["weight"].astype(np.float64)
    same_entry = counted & (pa["lut_index"] == pb["lut_index"]).all(axis=1)
    assert np.array_equal(wa[same_entry], wb[same_entry])
    other = ~same_entry
    assert abs((wa.sum() - wb.sum()) - (wa[other].sum() - wb[other].sum())) < 1e-9 * wb.sum()
    assert abs(wa.sum() - wb.sum()) < 2e-4 * wb.sum()


# ---------------------------------------------------------------------------
# LUT variants and energy configurations (Methods, "Scatter simulator
# description"; "Photon detection probability LUT")
# ---------------------------------------------------------------------------

def test_energy_blur_is_gaussian_with_the_stated_resolution():
    """Point source in air: every photon arrives at 511 keV, so the detected
    energies are 511 (1 + sigma n) with sigma = FWHM / 2.35482 (11.2 %, the
    no-LUT configuration), n standard normal."""
    w = W.WORKLOADS["tiny"]
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    pd, mu, act = W.point_source((0.0, 0.0, 0.0))
    phys = dict(W.PHYSICS_NO_LUT, e_lo_kev=0.0, e_hi_kev=2000.0)
    r = run(w.scanner, w.sino, phys, pd, mu, act, ld, lut, 40_000, records=True, sinograms=False, seed=11)
    ph = r["records"]["ph"]
    det = (ph["inter"] >> 16) == 0
    assert np.all(ph["e_kev"][det] == np.float32(510.99895))
    z = (ph["e_det_kev"][det].astype(np.float64) / 510.99895 - 1.0) / (0.112 / 2.35482)
    assert det.sum() > 20_000
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.std() - 1.0) < 0.02


def test_no_lut_mode_counts_in_window_coincidences_with_weight_one():
    """No-LUT mode: a one-entry LUT of 1 makes the weighted sinogram the
    count sinogram, and every counted single lies in the 425-650 keV window
    after the 11.2 % blur."""
    w = W.WORKLOADS["tiny"]
    phys, ld, lut = W.lut_mode(w, "nolut")
    pd, mu, act = W.make_phantom(w)
    r = run(w.scanner, w.sino, phys, pd, mu, act, ld, lut, 60_000, records=True, trues=True)
    assert r["scatter_counts"].sum() > 0
    assert np.array_equal(r["scatter_weights"], r["scatter_counts"].astype(np.float64))
    rec = r["records"]
    counted = (rec["outcome"] & 0xFF) <= 1
    e = rec["ph"]["e_det_kev"][counted]
    assert np.all((e >= 425.0) & (e <= 650.0))
    blurred = rec["ph"]["e_det_kev"] != rec["ph"]["e_kev"]
    assert blurred[counted].all()


@pytest.mark.parametrize("mode", ["lut1d", "lut3d_angles", "lut3d_crystals"])
def test_reduced_lut_equals_the_5d_lut_constant_along_the_other_axes(mode):
    """A LUT with unit dimensions gives exactly the sinograms of the 5D LUT
    that repeats its values along the missing axes (same energy axis)."""
    w = W.WORKLOADS["tiny"]
    phys, ld, lut = W.lut_mode(w, mode)
    full = np.broadcast_to(lut, tuple(max(a, b) for a, b in zip(lut.shape, w.lut_dims))).copy()
    assert full.shape == tuple(w.lut_dims)
    ld5 = W.LutDesc(tuple(w.lut_dims), ld.e_min_kev, ld.e_max_kev)
    pd, mu, act = W.make_phantom(w)
    a = run(w.scanner, w.sino, phys, pd, mu, act, ld, lut, 50_000)
    b = run(w.scanner, w.sino, phys, pd, mu, act, ld5, full, 50_000)
    assert np.array_equal(a["scatter_counts"], b["scatter_counts"])
    assert np.array_equal(a["scatter_weights"], b["scatter_weights"])
