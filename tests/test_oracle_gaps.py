"""Pins of the oracle's gap model and edge-crystal assignment (Methods,
"Scatter simulator description", "Photon detection probability LUT", "Edge
crystal assignment LUT", Eq. (1)-(3)).

Each pin checks the oracle against something fixed outside its code: path
lengths by ray marching, detection probabilities by integrating the
interaction density along the ray (no chord formula, no case split on the
sign of the angle), crystal centres and gap measures of the stated geometry,
and the observable effect of each gap policy on whole runs."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.harness import case_from, run_oracle, with_gaps

GEOM = dict(gap_mm=2.0, depth_mm=25.0, doi_mm=8.0, mu_per_mm=0.087, n_angle=36, n_pos=16)
THETAS_DEG = [-85.0, -60.0, -30.0, -10.0, -3.0, 3.0, 10.0, 30.0, 60.0, 85.0]
X_FRACS = [-0.95, -0.5, -0.1, 0.0, 0.3, 0.9]


def _march(geom, theta, x0, n=400_000):
    """Block membership (1, 2 or 0) at n equally spaced depths along the ray
    through the blocks' depth range, in the order the photon travels them,
    and the path length per sample."""
    D, d, hw = geom["depth_mm"], geom["doi_mm"], 0.5 * geom["gap_mm"]
    y = (np.arange(n) + 0.5) * D / n
    x = x0 + (y - d) * math.tan(theta)
    which = np.where(x <= -hw, 1, np.where(x >= hw, 2, 0))
    return which, D / n / math.cos(theta)


def _integrated_probs(geom, theta, x0):
    """P(first interaction in block 1), P(in block 2): the interaction density
    mu exp(-tau(s)) integrated along the ray, tau the optical depth
    accumulated in either block before s."""
    which, ds = _march(geom, theta, x0)
    mu = geom["mu_per_mm"]
    inside = (which > 0).astype(np.float64)
    tau_before = mu * ds * (np.cumsum(inside) - 0.5 * inside)
    dens = mu * ds * np.exp(-tau_before)
    return float(dens[which == 1].sum()), float(dens[which == 2].sum())


@pytest.mark.parametrize("theta_deg", THETAS_DEG)
def test_edge_paths_match_ray_marching(theta_deg):
    th = math.radians(theta_deg)
    hw = 0.5 * GEOM["gap_mm"]
    for f in X_FRACS:
        x0 = f * hw
        l1, l2 = O.edge_paths(GEOM, th, x0)
        which, ds = _march(GEOM, th, x0)
        assert abs(l1 - ds * np.count_nonzero(which == 1)) <= 2 * ds
        assert abs(l2 - ds * np.count_nonzero(which == 2)) <= 2 * ds


@pytest.mark.parametrize("theta_deg", THETAS_DEG)
def test_edge_probability_is_the_first_interaction_share(theta_deg):
    """Eq. (1)-(3) read as detection probabilities (the block met first
    absorbs with 1 - exp(-mu l), the second only what the first let through),
    normalised: the share of block 1 among first interactions in either
    block.  Where the ray misses both blocks the nearer edge is taken."""
    th = math.radians(theta_deg)
    hw = 0.5 * GEOM["gap_mm"]
    for f in X_FRACS:
        x0 = f * hw
        p1, p2 = _integrated_probs(GEOM, th, x0)
        got = O.edge_prob(GEOM, th, x0)
        if p1 + p2 > 0:
            assert abs(got - p1 / (p1 + p2)) < 1e-4, (theta_deg, f, got, p1, p2)
        else:
            assert got == (1.0 if x0 < 0 else 0.0 if x0 > 0 else 0.5)


def test_edge_probability_symmetry_and_limits():
    hw = 0.5 * GEOM["gap_mm"]
    for td in THETAS_DEG:
        th = math.radians(td)
        for f in X_FRACS:
            # mirror image: the roles of the blocks swap
            assert abs(O.edge_prob(GEOM, th, f * hw) + O.edge_prob(GEOM, -th, -f * hw) - 1.0) < 1e-12
    # a very dense crystal: the block met first takes the photon whenever the
    # ray passes through it
    dense = dict(GEOM, mu_per_mm=50.0)
    for td in (10.0, 30.0, 60.0):
        th = math.radians(td)
        l1, _ = O.edge_paths(dense, th, 0.0)
        assert l1 > 0.1
        assert O.edge_prob(dense, th, 0.0) > 1 - 1e-9
        assert O.edge_prob(dense, -th, 0.0) < 1e-9
    # a thin crystal: shares proportional to the path lengths
    thin = dict(GEOM, mu_per_mm=1e-7)
    for td in (10.0, 30.0, -60.0):
        th = math.radians(td)
        l1, l2 = O.edge_paths(thin, th, 0.2)
        assert abs(O.edge_prob(thin, th, 0.2) - l1 / (l1 + l2)) < 1e-5


def test_edge_lut_layout_and_monotone():
    lut = O.edge_lut(GEOM)
    assert lut.shape == (GEOM["n_angle"], GEOM["n_pos"]) and lut.dtype == np.float32
    w = GEOM["gap_mm"]
    for a in (0, 5, 17, 18, 30, 35):
        th = math.radians(-90.0 + (a + 0.5) * 180.0 / GEOM["n_angle"])
        for j in (0, 7, 15):
            x0 = -0.5 * w + (j + 0.5) * w / GEOM["n_pos"]
            assert lut[a, j] == np.float32(O.edge_prob(GEOM, th, x0))
    # for any angle, a photon further towards block 1 is at least as likely
    # to be assigned to it
    assert np.all(np.diff(lut.astype(np.float64), axis=1) <= 1e-7)
    assert np.all((lut >= 0) & (lut <= 1))


# --------------------------------------------------------------------------
# gap geometry
# --------------------------------------------------------------------------

def _signa():
    return W.signa_scanner()


def _hit(sc, phi, z):
    return (np.float32(sc.radius_mm * math.cos(phi)), np.float32(sc.radius_mm * math.sin(phi)), np.float32(z))


@pytest.mark.parametrize("which", ["signa", "tiny"])
def test_locate_crystal_and_ring_centres(which):
    sc = W.signa_scanner() if which == "signa" else W.tiny_scanner()
    gaps = W.gap_desc(W.SIGNA_GAPS if which == "signa" else W.TINY_GAPS, "nearest")
    cm, rb = sc.crystals_per_module, sc.rings_per_block
    nm, nb = sc.n_crystals // cm, sc.n_rings // rb
    g, w, L = gaps["transaxial_gap_rad"], gaps["axial_gap_mm"], sc.length_mm
    D = 2 * math.pi / nm
    pa = (L - (nb - 1) * w) / sc.n_rings
    for m in range(nm):
        for k in range(cm):
            phi = m * D + g / 2 + (k + 0.5) * (D - g) / cm
            r = O.locate(sc, gaps, *_hit(sc, phi, 0.0))
            assert (r["crystal"], r["ct"], r["tgap"]) == (m * cm + k, k + 1, 0)
    for b in range(nb):
        for k in range(rb):
            z = -L / 2 + b * (rb * pa + w) + (k + 0.5) * pa
            r = O.locate(sc, gaps, *_hit(sc, 0.3 * D + g, z))
            assert (r["ring"], r["ca"], r["agap"]) == (b * rb + k, b * (rb + 2) + 1 + k, 0)


@pytest.mark.parametrize("which", ["signa", "tiny"])
def test_locate_gap_halves(which):
    sc = W.signa_scanner() if which == "signa" else W.tiny_scanner()
    gaps = W.gap_desc(W.SIGNA_GAPS if which == "signa" else W.TINY_GAPS, "nearest")
    cm, rb = sc.crystals_per_module, sc.rings_per_block
    nm, nb = sc.n_crystals // cm, sc.n_rings // rb
    g, w, L = gaps["transaxial_gap_rad"], gaps["axial_gap_mm"], sc.length_mm
    D = 2 * math.pi / nm
    pa = (L - (nb - 1) * w) / sc.n_rings
    zc = -L / 2 + 0.5 * pa  # inside ring 0
    for m in range(nm):
        lo, hi = ((m - 1) % nm) * cm + cm - 1, m * cm
        # quarter of the gap on module m's side of the boundary m D
        r = O.locate(sc, gaps, *_hit(sc, (m * D + g / 4) % (2 * math.pi), zc))
        assert (r["tgap"], r["ct"], r["crystal"], r["c_lo"], r["c_hi"]) == (1, 0, hi, lo, hi)
        assert abs(r["tfrac"] - 0.75) < 1e-3
        # quarter of the gap on module m-1's side
        r = O.locate(sc, gaps, *_hit(sc, (m * D - g / 4) % (2 * math.pi), zc))
        assert (r["tgap"], r["ct"], r["crystal"], r["c_lo"], r["c_hi"]) == (1, cm + 1, lo, lo, hi)
        assert abs(r["tfrac"] - 0.25) < 1e-3
    phic = 0.5 * D  # middle of module 0
    for b in range(nb - 1):
        z0 = -L / 2 + b * (rb * pa + w) + rb * pa  # start of the gap above block b
        r = O.locate(sc, gaps, *_hit(sc, phic, z0 + 0.25 * w))
        assert (r["agap"], r["ca"], r["ring"], r["r_lo"], r["r_hi"]) == (
            1, b * (rb + 2) + rb + 1, b * rb + rb - 1, b * rb + rb - 1, (b + 1) * rb)
        assert abs(r["afrac"] - 0.25) < 1e-3
        r = O.locate(sc, gaps, *_hit(sc, phic, z0 + 0.75 * w))
        assert (r["agap"], r["ca"], r["ring"]) == (1, (b + 1) * (rb + 2), (b + 1) * rb)
        assert abs(r["afrac"] - 0.75) < 1e-3


def test_locate_measure_of_gaps_and_crystals():
    """On a dense regular grid the share of gap hits is the gaps' share of
    the circumference / length and every crystal and ring covers an equal
    share of the rest."""
    sc = W.signa_scanner()
    gaps = W.gap_desc(W.SIGNA_GAPS, "nearest")
    cm, rb = sc.crystals_per_module, sc.rings_per_block
    nm, nb = sc.n_crystals // cm, sc.n_rings // rb
    g, w, L = gaps["transaxial_gap_rad"], gaps["axial_gap_mm"], sc.length_mm
    N = 179_200
    counts = np.zeros(sc.n_crystals, np.int64)
    n_gap = 0
    for i in range(N):
        r = O.locate(sc, gaps, *_hit(sc, 2 * math.pi * (i + 0.5) / N, 0.0))
        if r["tgap"]:
            n_gap += 1
        else:
            counts[r["crystal"]] += 1
    assert abs(n_gap / N - nm * g / (2 * math.pi)) < 3.0 / N * nm
    per = N * (2 * math.pi / nm - g) / cm / (2 * math.pi)
    assert np.all(np.abs(counts - per) <= 2)
    Nz = 45_000
    rcounts = np.zeros(sc.n_rings, np.int64)
    z_gap = 0
    for i in range(Nz):
        r = O.locate(sc, gaps, *_hit(sc, 0.01, -L / 2 + L * (i + 0.5) / Nz))
        if r["agap"]:
            z_gap += 1
        else:
            rcounts[r["ring"]] += 1
    assert abs(z_gap / Nz - (nb - 1) * w / L) < 3.0 / Nz * nb
    pa = (L - (nb - 1) * w) / sc.n_rings
    assert np.all(np.abs(rcounts - Nz * pa / L) <= 2)


def test_locate_zero_gaps_is_the_plain_cylinder():
    sc = W.tiny_scanner()
    gaps = dict(transaxial_gap_rad=0.0, axial_gap_mm=0.0, policy="nearest")
    rng = np.random.default_rng(5)
    pitch = sc.length_mm / sc.n_rings
    for _ in range(5000):
        phi = rng.uniform(0, 2 * math.pi)
        z = rng.uniform(-sc.length_mm / 2, sc.length_mm / 2)
        hx, hy, hz = _hit(sc, phi, z)
        a = math.atan2(float(hy), float(hx)) % (2 * math.pi)
        fc = a * sc.n_crystals / (2 * math.pi)
        fr = (float(hz) + sc.length_mm / 2) / pitch
        if min(abs(fc - round(fc)), abs(fr - round(fr))) < 1e-6:
            continue
        r = O.locate(sc, gaps, hx, hy, hz)
        assert (r["crystal"], r["ring"], r["tgap"], r["agap"]) == (int(fc), int(fr), 0, 0)


# --------------------------------------------------------------------------
# policies on whole runs
# --------------------------------------------------------------------------
N_RUN = 200_000
SEED = 31


def _lut_coords(case, lut_index):
    d3, d4 = case.lut_desc.dims[3], case.lut_desc.dims[4]
    return (lut_index // d4) % d3, lut_index % d4


def _gap_single(case, rec_ph):
    ct, ca = _lut_coords(case, rec_ph["lut_index"].astype(np.int64))
    cm, rb = case.scanner.crystals_per_module, case.scanner.rings_per_block
    return (ct == 0) | (ct == cm + 1) | (ca % (rb + 2) == 0) | (ca % (rb + 2) == rb + 1)


def _evaluated(rec):
    """Coincidences that reached crystal assignment (both singles in the window)."""
    o = rec["outcome"] & 0xFF
    return (o == 0) | (o == 1) | (o >= 4)


def _bin_coords(case, b):
    s = case.sino
    rad = b % s.n_rad
    view = (b // s.n_rad) % s.n_view
    plane = (b // (s.n_rad * s.n_view)) % s.n_plane
    return plane, view, rad


def _lor_matches(case, b, cA, rA, cB, rB):
    plane, view, rad = _bin_coords(case, b)
    v, rho, _ = O.lor(case.scanner.n_crystals, cA, cB)
    return plane == rA + rB and view == v and rad == rho + (case.sino.n_rad - 1) // 2


def test_discard_policy_drops_exactly_the_gap_coincidences():
    case = with_gaps(case_from("tiny"), W.TINY_GAPS, "discard")
    r = run_oracle(case, N_RUN, SEED)
    rec, st = r["records"], r["stats"]
    ev = _evaluated(rec)
    gap = _gap_single(case, rec["ph"][:, 0]) | _gap_single(case, rec["ph"][:, 1])
    out8 = (rec["outcome"] & 0xFF) == O.OUTCOME["gap"]
    assert np.array_equal(out8, ev & gap)
    assert st["rej_gap"] == int(out8.sum()) > 0
    assert st["gap_assigned"] == 0


def _assignment_sides(case, rec, table_check=None):
    """For each binned coincidence, which edge crystal / ring each gap photon
    went to, read back from the sinogram bin: list of (kind, lower_side)."""
    sides = []
    sc = case.scanner
    binned = ((rec["outcome"] & 0xFF) <= 1)
    for i in np.nonzero(binned)[0]:
        b = int(rec["bin_lo"][i]) | (int(rec["bin_hi"][i]) << 32)
        locs = [O.locate(sc, case.gaps, rec["ph"][i, k]["hx"], rec["ph"][i, k]["hy"], rec["ph"][i, k]["hz"])
                for k in (0, 1)]
        if not any(l["tgap"] or l["agap"] for l in locs):
            continue
        opts = []
        for k, l in enumerate(locs):
            cs = [(l["c_lo"], True), (l["c_hi"], False)] if l["tgap"] else [(l["crystal"], None)]
            rs = [(l["r_lo"], True), (l["r_hi"], False)] if l["agap"] else [(l["ring"], None)]
            opts.append([(c, r, cl, rl) for c, cl in cs for r, rl in rs])
        found = [(a, bb) for a in opts[0] for bb in opts[1]
                 if _lor_matches(case, b, a[0], a[1], bb[0], bb[1])]
        assert found, i
        if len(found) > 1:
            # both photons in axial gaps: the plane r_A + r_B does not tell
            # (lower, upper) from (upper, lower)
            continue
        for k, (c, rg, cl, rl) in enumerate(found[0]):
            if cl is not None:
                sides.append(("t", cl))
            if rl is not None:
                sides.append(("a", rl))
    return sides


def test_nearest_policy_keeps_the_nearest_edge_crystal():
    case = with_gaps(case_from("tiny"), W.TINY_GAPS, "nearest")
    r = run_oracle(case, N_RUN // 4, SEED)
    rec, st = r["records"], r["stats"]
    assert not np.any((rec["outcome"] & 0xFF) == O.OUTCOME["gap"])
    binned = np.nonzero((rec["outcome"] & 0xFF) <= 1)[0]
    cr = rec["ph"]["crystal_ring"]
    for i in binned:
        b = int(rec["bin_lo"][i]) | (int(rec["bin_hi"][i]) << 32)
        assert _lor_matches(case, b, int(cr[i, 0] & 0xFFFF), int(cr[i, 0] >> 16),
                            int(cr[i, 1] & 0xFFFF), int(cr[i, 1] >> 16))
    assert st["gap_assigned"] > 0


@pytest.mark.parametrize("p,expect_lower", [(1.0, True), (0.0, False)])
def test_edge_policy_with_certain_tables(p, expect_lower):
    base = case_from("tiny")
    nt = W.EDGE_N_ANGLE * W.EDGE_N_POS
    tab = np.full((W.EDGE_N_ANGLE, W.EDGE_N_POS), p, np.float32)
    case = with_gaps(base, W.TINY_GAPS, "edge_lut", edge=(tab, tab))
    r = run_oracle(case, N_RUN // 4, SEED)
    sides = _assignment_sides(case, r["records"])
    assert len(sides) > 100 and nt > 0
    assert all(s == expect_lower for _, s in sides)


def test_edge_policy_assigns_with_the_table_probability():
    base = case_from("tiny")
    tt = np.full((W.EDGE_N_ANGLE, W.EDGE_N_POS), 0.3, np.float32)
    ta = np.full((W.EDGE_N_ANGLE, W.EDGE_N_POS), 0.8, np.float32)
    case = with_gaps(base, W.TINY_GAPS, "edge_lut", edge=(tt, ta))
    r = run_oracle(case, N_RUN, SEED)
    sides = _assignment_sides(case, r["records"])
    for kind, p in (("t", 0.3), ("a", 0.8)):
        s = np.array([lo for k, lo in sides if k == kind], float)
        assert s.size > 300
        assert abs(s.mean() - p) < 4 * math.sqrt(p * (1 - p) / s.size), (kind, s.mean(), s.size)


def test_edge_policy_with_the_physical_tables_prefers_the_block_met_first():
    """With the Eq. (1)-(3) tables, photons crossing a transaxial gap towards
    the upper module (positive transaxial angle) land in the lower module's
    edge crystal more often than photons crossing it the other way."""
    case = with_gaps(case_from("tiny"), W.TINY_GAPS, "edge_lut")
    r = run_oracle(case, N_RUN, SEED)
    assert r["stats"]["gap_assigned"] > 0
    assert r["stats"]["rej_gap"] == 0
    rec = r["records"]
    sides = _assignment_sides(case, rec)
    t = np.array([lo for k, lo in sides if k == "t"], float)
    assert 0.05 < t.mean() < 0.95


def test_gap_share_of_coincidences_on_the_signa_geometry():
    """Sanity range, not a pin: the paper reports about 20 % of coincidences
    with a gap photon on the Signa (Discussion)."""
    base = case_from("tiny")
    sc = W.signa_scanner()
    from workloads import Sinogram
    sino = W.signa_sinogram(0.0)
    plain = type(base)(sc, sino, base.physics, base.pdesc, base.mu, base.act,
                       *W.make_lut((8, 4, 4, 8, 4), 1), None)
    plain.lut_store = plain.lut
    case = with_gaps(plain, W.SIGNA_GAPS, "discard")
    r = run_oracle(case, 100_000, SEED)
    st = r["stats"]
    ev = st["scatter"] + st["true"] + st["rej_gap"] + st["rej_same"] + st["rej_ring"] + st["rej_radial"] + st["rej_tof"]
    share = st["rej_gap"] / ev
    assert 0.12 < share < 0.35, share


def test_zero_width_gaps_reproduce_the_plain_run():
    base = case_from("tiny")
    d = base.lut_desc.dims
    ld, vals = W.make_lut((d[0], d[1], d[2], 1, 1), 3)
    plain = case_from("tiny", lut=(ld, vals))
    zero = with_gaps(plain, dict(transaxial_gap_rad=0.0, axial_gap_mm=0.0), "nearest")
    zero.lut_desc, zero.lut, zero.lut_store = ld, vals, vals
    a = run_oracle(plain, 50_000, SEED)
    b = run_oracle(zero, 50_000, SEED)
    assert np.array_equal(a["scatter_counts"], b["scatter_counts"])
    assert np.array_equal(a["scatter_weights"], b["scatter_weights"])
    wa = a["records"].view(np.uint32).reshape(-1, 32)
    wb = b["records"].view(np.uint32).reshape(-1, 32)
    assert np.array_equal(wa, wb)
    assert b["stats"]["gap_assigned"] == 0
