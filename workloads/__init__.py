"""Seeded synthetic inputs for the scatter-estimation path.

This module builds the inputs that both the CPU oracle and the HIP library
consume: voxel phantoms (attenuation at 511 keV and activity), detection
probability LUTs, scatter-sensitivity sinograms and the scanner / sinogram /
physics parameter sets of the five workloads.  It holds none of the method's
arithmetic: no transport, no sampling, no binning.  Every array is produced
from a fixed numpy seed or a closed-form pattern, so the oracle and the GPU
path see the same bytes.

The paper's own phantoms, LUT and sensitivity sinograms come from GATE runs
that are not available; these stand in with the paper's shapes:
  * scanner: Signa PET/MR, 28 modules x 16 crystals = 448 crystals per ring,
    45 rings in 5 blocks of 9, radius 311.8 mm to the module face (plus an
    average depth of interaction), length 250.4 mm (Methods, "Signa PET/MR
    description" and "Scatter simulator description");
  * energy window 425-650 keV and 380 ps FWHM TOF (Methods, "Simulated scans
    in GATE");
  * 5D LUT axes energy x transaxial angle x axial angle x transaxial crystal
    x axial crystal, values in [0, 1] (Methods, "Photon detection probability
    LUT").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# parameter sets
# --------------------------------------------------------------------------

# Photon physics model parameters (builder's choice; the paper delegates the
# transport physics to its simulator).  The fractions split the total
# attenuation at 511 keV into Compton, Rayleigh and photoabsorption, roughly as
# for water; the Rayleigh form-factor parameter sets a characteristic angle of
# about 2.6 degrees at 511 keV.
PHYSICS_DEFAULT = dict(
    e_lo_kev=425.0,
    e_hi_kev=650.0,
    e_kill_kev=425.0,
    e_fwhm_frac=0.0,
    f_compton=0.9955,
    f_rayleigh=0.0040,
    f_photo=0.0005,
    rayleigh_beta=1000.0,
    mu_majorant=0.0,  # 0: use the phantom maximum
    max_interactions=1000,
)

C_LIGHT_MM_PER_PS = 0.299792458


def tof_sigma_mm(fwhm_ps: float) -> float:
    """Standard deviation of the TOF offset along the LOR, in mm, for a
    coincidence timing resolution given as FWHM in ps (offset = c * dt / 2)."""
    return fwhm_ps * C_LIGHT_MM_PER_PS / 2.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclass
class Scanner:
    n_crystals: int
    n_rings: int
    radius_mm: float
    length_mm: float
    crystals_per_module: int
    rings_per_block: int
    max_ring_diff: int = -1


@dataclass
class Sinogram:
    n_rad: int
    n_view: int
    n_plane: int
    n_tof: int
    tof_bin_mm: float
    tof_sigma_mm: float

    @property
    def shape(self):
        """C-order array shape [tof][plane][view][rad]."""
        return (self.n_tof, self.n_plane, self.n_view, self.n_rad)

    @property
    def n_bins(self) -> int:
        return self.n_tof * self.n_plane * self.n_view * self.n_rad


@dataclass
class PhantomDesc:
    nx: int
    ny: int
    nz: int
    voxel_mm: tuple
    lo_mm: tuple  # minimum corner of the voxel box

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


@dataclass
class LutDesc:
    dims: tuple  # (n_e, n_theta_t, n_theta_a, n_ct, n_ca)
    e_min_kev: float
    e_max_kev: float


@dataclass
class Workload:
    name: str
    scanner: Scanner
    sino: Sinogram
    physics: dict
    n_histories: int
    seed: int
    lut_dims: tuple
    lut_seed: int
    phantom_kind: str
    extra: dict = field(default_factory=dict)


def signa_scanner() -> Scanner:
    return Scanner(n_crystals=448, n_rings=45, radius_mm=312.0, length_mm=250.4,
                   crystals_per_module=16, rings_per_block=9)


def signa_sinogram(tof_fwhm_ps: float = 380.0) -> Sinogram:
    n_tof = 29
    return Sinogram(n_rad=357, n_view=224, n_plane=89, n_tof=n_tof,
                    tof_bin_mm=2.0 * 312.0 / n_tof,
                    tof_sigma_mm=tof_sigma_mm(tof_fwhm_ps) if tof_fwhm_ps > 0 else 0.0)


def tiny_scanner() -> Scanner:
    return Scanner(n_crystals=64, n_rings=4, radius_mm=150.0, length_mm=128.0,
                   crystals_per_module=4, rings_per_block=2)


def tiny_sinogram() -> Sinogram:
    n_tof = 11
    return Sinogram(n_rad=63, n_view=32, n_plane=7, n_tof=n_tof,
                    tof_bin_mm=2.0 * 150.0 / n_tof, tof_sigma_mm=0.0)


WORKLOADS = {
    "tiny": Workload("tiny", tiny_scanner(), tiny_sinogram(), dict(PHYSICS_DEFAULT),
                     n_histories=100_000, seed=1234, lut_dims=(16, 8, 8, 4, 2), lut_seed=1,
                     phantom_kind="tiny_cylinder"),
    "clinical": Workload("clinical", signa_scanner(), signa_sinogram(), dict(PHYSICS_DEFAULT),
                         n_histories=1_000_000_000, seed=5678, lut_dims=(32, 16, 16, 8, 4), lut_seed=2,
                         phantom_kind="clinical_body"),
    "large": Workload("large", signa_scanner(), signa_sinogram(), dict(PHYSICS_DEFAULT),
                      n_histories=2_000_000_000, seed=9012, lut_dims=(32, 16, 16, 8, 4), lut_seed=2,
                      phantom_kind="large_body", extra=dict(n_requests=5, smooth_sigma_bins=2.0)),
}


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------

MU_WATER = 0.0096   # 1/mm at 511 keV (0.096 / cm)
MU_LUNG = 0.0030
MU_BONE = 0.0170


def centred_desc(n, voxel_mm, offset_mm=(0.0, 0.0, 0.0)) -> PhantomDesc:
    nx, ny, nz = n
    lo = tuple(float(np.float32(-0.5 * ni * vi + oi)) for ni, vi, oi in zip(n, voxel_mm, offset_mm))
    return PhantomDesc(nx, ny, nz, tuple(float(np.float32(v)) for v in voxel_mm), lo)


def voxel_centres(desc: PhantomDesc):
    """Voxel-centre coordinates (z, y, x) in mm as broadcastable float64 arrays."""
    z = desc.lo_mm[2] + (np.arange(desc.nz) + 0.5) * desc.voxel_mm[2]
    y = desc.lo_mm[1] + (np.arange(desc.ny) + 0.5) * desc.voxel_mm[1]
    x = desc.lo_mm[0] + (np.arange(desc.nx) + 0.5) * desc.voxel_mm[0]
    return z[:, None, None], y[None, :, None], x[None, None, :]


def tiny_cylinder():
    """32^3 voxels of 4 mm; water cylinder r = 50 mm along z, full length,
    uniform activity (voxel centres inside the radius are filled)."""
    desc = centred_desc((32, 32, 32), (4.0, 4.0, 4.0))
    z, y, x = voxel_centres(desc)
    inside = (x * x + y * y <= 50.0 ** 2) & (z == z)
    mu = np.where(inside, MU_WATER, 0.0).astype(np.float32)
    act = np.where(inside, 1.0, 0.0).astype(np.float32)
    return desc, mu, act


def _paint_body(desc, body_ax=150.0, body_ay=100.0, scale=1.0, sphere_z=-70.0):
    z, y, x = voxel_centres(desc)
    shape = desc.shape
    mu = np.zeros(shape, np.float64)
    act = np.zeros(shape, np.float64)
    body = ((x / (body_ax * scale)) ** 2 + (y / (body_ay * scale)) ** 2 <= 1.0) & (z == z)
    mu[body] = MU_WATER
    act[body] = 1.0
    for sx in (-65.0, 65.0):
        lung = (((x - sx * scale) / (40.0 * scale)) ** 2 + ((y + 10.0 * scale) / (55.0 * scale)) ** 2
                + ((z - 40.0) / 70.0) ** 2 <= 1.0)
        lung = np.broadcast_to(lung, shape)
        mu[lung] = MU_LUNG
        act[lung] = 0.25
    spine = np.broadcast_to((x ** 2 + (y - 70.0 * scale) ** 2 <= (15.0 * scale) ** 2) & (z == z), shape)
    mu[spine] = MU_BONE
    act[spine] = 1.0
    for i in range(6):
        d = 10.0 * 3.7 ** (i / 5.0)
        ang = 2.0 * math.pi * i / 6.0
        cx, cy = 55.0 * scale * math.cos(ang), 55.0 * scale * math.sin(ang)
        sph = np.broadcast_to((x - cx) ** 2 + (y - cy) ** 2 + (z - sphere_z) ** 2 <= (d / 2.0) ** 2, shape)
        mu[sph] = MU_WATER
        act[sph] = 4.0
    return mu.astype(np.float32), act.astype(np.float32)


def clinical_body():
    """128 x 128 x 89 voxels of 2.34 x 2.34 x 2.78 mm: elliptical water body
    300 x 200 mm, two lungs (mu 0.03/cm, activity 0.25), a bone spine
    (0.17/cm) and six hot spheres of 10-37 mm diameter at 4:1 activity."""
    desc = centred_desc((128, 128, 89), (2.34, 2.34, 2.78))
    mu, act = _paint_body(desc)
    return desc, mu, act


def large_body():
    """256 x 256 x 89 voxels of 1.17 x 1.17 x 2.78 mm, same body as the
    clinical phantom."""
    desc = centred_desc((256, 256, 89), (1.17, 1.17, 2.78))
    mu, act = _paint_body(desc)
    return desc, mu, act


def point_source(pos_mm=(0.0, 0.0, 0.0), mu=0.0, size_mm=1e-3):
    """A single tiny voxel centred at pos_mm (one-voxel phantom)."""
    desc = PhantomDesc(1, 1, 1, (size_mm, size_mm, size_mm),
                       tuple(float(np.float32(p - 0.5 * size_mm)) for p in pos_mm))
    return desc, np.full((1, 1, 1), mu, np.float32), np.ones((1, 1, 1), np.float32)


def uniform_box(n=(16, 16, 16), voxel_mm=(8.0, 8.0, 8.0), mu=MU_WATER, source_voxel=None):
    """Uniform attenuating box; activity in one voxel (default: none given ->
    all voxels active)."""
    desc = centred_desc(n, voxel_mm)
    mu_a = np.full(desc.shape, mu, np.float32)
    act = np.zeros(desc.shape, np.float32)
    if source_voxel is None:
        act[:] = 1.0
    else:
        act[source_voxel] = 1.0
    return desc, mu_a, act


def serving_phantom(seed: int):
    """Body-like ellipsoid phantom for a serving request: grid kind, body
    semi-axes and 3-6 organ ellipsoids drawn from the request seed."""
    rng = np.random.default_rng(seed)
    kind = int(rng.integers(0, 3))
    if kind == 0:
        desc = centred_desc((64, 64, 64), (4.68, 4.68, 4.68))
    elif kind == 1:
        desc = centred_desc((128, 128, 128), (2.34, 2.34, 2.34))
    else:
        desc = centred_desc((192, 192, 89), (1.56, 1.56, 2.78))
    z, y, x = voxel_centres(desc)
    shape = desc.shape
    ax, ay = rng.uniform(120.0, 160.0), rng.uniform(80.0, 120.0)
    half_z = 0.5 * desc.nz * desc.voxel_mm[2]
    mu = np.zeros(shape, np.float64)
    act = np.zeros(shape, np.float64)
    body = np.broadcast_to((x / ax) ** 2 + (y / ay) ** 2 <= 1.0, shape)
    mu[body] = MU_WATER
    act[body] = 1.0
    for _ in range(int(rng.integers(3, 7))):
        cx, cy = rng.uniform(-0.5, 0.5) * ax, rng.uniform(-0.5, 0.5) * ay
        cz = rng.uniform(-0.5, 0.5) * half_z
        rx, ry, rz = rng.uniform(10.0, 40.0, size=3)
        m = (MU_LUNG, MU_WATER, MU_BONE)[int(rng.integers(0, 3))]
        a = rng.uniform(0.5, 4.0)
        org = np.broadcast_to(((x - cx) / rx) ** 2 + ((y - cy) / ry) ** 2 + ((z - cz) / rz) ** 2 <= 1.0, shape) & body
        mu[org] = m
        act[org] = a
    return desc, mu.astype(np.float32), act.astype(np.float32)


def reference_cylinder(desc: PhantomDesc, radius_mm: float):
    """Uniform water cylinder of the given radius along z, full length, on a
    phantom grid: the reference object of the smoothing normalisation (the
    paper uses a 40 cm cylinder)."""
    z, y, x = voxel_centres(desc)
    inside = np.broadcast_to(x * x + y * y <= radius_mm ** 2, desc.shape)
    return (np.where(inside, MU_WATER, 0.0).astype(np.float32), np.where(inside, 1.0, 0.0).astype(np.float32))


def plane_image(desc: PhantomDesc, vol: np.ndarray, scanner: Scanner) -> np.ndarray:
    """A voxel volume on the reconstruction image grid: the phantom's
    transaxial grid with one slice per sinogram plane, plane p (at z = -L/2 +
    (p + 1) pitch / 2) taking the voxel slice that holds its z."""
    n_plane = 2 * scanner.n_rings - 1
    half_pitch = 0.5 * scanner.length_mm / scanner.n_rings
    z = -0.5 * scanner.length_mm + (np.arange(n_plane) + 1) * half_pitch
    iz = np.clip(np.floor((z - desc.lo_mm[2]) / desc.voxel_mm[2]), 0, desc.nz - 1).astype(int)
    return np.ascontiguousarray(np.asarray(vol).reshape(desc.shape)[iz], np.float32)


def scaled_activity(act: np.ndarray, k: int, sigma_vox: float = 15.0) -> np.ndarray:
    """activity_k = activity_0 * max(0, 1 + 0.3 g_k), with g_k a Gaussian-filtered
    N(0, 1) field (sigma in voxels) normalised to max |g| = 1, seed k."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(k)
    g = gaussian_filter(rng.standard_normal(act.shape), sigma=sigma_vox, mode="wrap")
    g /= np.abs(g).max()
    return (act * np.maximum(0.0, 1.0 + 0.3 * g)).astype(np.float32)


PHANTOMS = {
    "tiny_cylinder": tiny_cylinder,
    "clinical_body": clinical_body,
    "large_body": large_body,
}


def make_phantom(w: Workload):
    return PHANTOMS[w.phantom_kind]()


# --------------------------------------------------------------------------
# LUT and sensitivity
# --------------------------------------------------------------------------

def make_lut(dims, seed: int, low: float = 0.2, high: float = 1.0, e_min=425.0, e_max=511.0):
    """Synthetic 5D detection-probability LUT, row-major [E][theta_t][theta_a][ct][ca],
    drawn uniform in [low, high] from the seed."""
    rng = np.random.default_rng(seed)
    vals = rng.uniform(low, high, size=tuple(dims)).astype(np.float32)
    return LutDesc(tuple(dims), float(e_min), float(e_max)), vals


# The paper's two simulator energy configurations (Methods, "Scatter
# simulator description"): with the LUT, a near-perfect 0.1 % energy
# resolution and a 300-650 keV window; without it, GATE's 11.2 % and
# 425-650 keV.  The kill energies are readings: at least six energy-resolution
# sigmas below the window, so that no killed photon could have blurred into
# it (11.2 % FWHM at 300 keV: sigma 18.6 keV, 125 keV below 425).
PHYSICS_LUT_PAPER = dict(PHYSICS_DEFAULT, e_fwhm_frac=0.001, e_lo_kev=300.0, e_hi_kev=650.0, e_kill_kev=290.0)
PHYSICS_NO_LUT = dict(PHYSICS_DEFAULT, e_fwhm_frac=0.112, e_lo_kev=425.0, e_hi_kev=650.0, e_kill_kev=300.0)

# LUT variants of the paper's comparison (Methods, "Photon detection
# probability LUT"; 1D over energy, 3D over energy and the two incidence
# angles, 3D over energy and the two in-block crystal coordinates, and the
# full 5D), expressed as unit dimensions of the 5D index, and the no-LUT
# mode (a single entry of 1: every coincidence counts 1).
LUT_MODES = ("lut5d", "lut5d_paper", "lut3d_angles", "lut3d_crystals", "lut1d", "nolut")


def lut_mode(w: "Workload", mode: str):
    """(physics, LutDesc, values) of a LUT mode for workload w.  'lut5d' is
    the workload's own setting (425-650 keV, no blur, LUT energy axis
    425-511 keV); the others use the paper's energy configurations, the LUT
    energy axis over 300-511 keV (the 300 keV window edge to the source
    line)."""
    d = tuple(w.lut_dims)
    if mode == "lut5d":
        ld, vals = make_lut(d, w.lut_seed)
        return dict(w.physics), ld, vals
    if mode == "nolut":
        return dict(PHYSICS_NO_LUT), LutDesc((1, 1, 1, 1, 1), 425.0, 511.0), np.ones((1, 1, 1, 1, 1), np.float32)
    dims = {"lut5d_paper": d, "lut3d_angles": (d[0], d[1], d[2], 1, 1),
            "lut3d_crystals": (d[0], 1, 1, d[3], d[4]), "lut1d": (d[0], 1, 1, 1, 1)}[mode]
    ld, vals = make_lut(dims, w.lut_seed, e_min=300.0, e_max=511.0)
    return dict(PHYSICS_LUT_PAPER), ld, vals


# --------------------------------------------------------------------------
# gaps between modules and blocks
# --------------------------------------------------------------------------
# Gap geometry (builder's choice; the paper gives the Signa's gaps only as
# "the real scanner's"): on the Signa-like scanner a module spans
# 2 pi 312 / 28 = 70.0 mm of arc, 16 crystals of about 4 mm leave a 6 mm
# transaxial gap; 45 rings of about 5.3 mm in 5 blocks over 250.4 mm leave
# 3 mm axial gaps.  About one in eight singles then lands in a gap, and about
# a quarter of coincidences contain one (the paper: about 20 % on the Signa,
# Discussion).  The tiny scanner's gaps are scaled to give a similar share.
SIGNA_GAPS = dict(transaxial_gap_rad=6.0 / 312.0, axial_gap_mm=3.0)
TINY_GAPS = dict(transaxial_gap_rad=0.06, axial_gap_mm=6.0)

# Crystal blocks for the edge-crystal LUT: 25 mm deep LYSO (Signa), the
# detection surface 8 mm below the front face (the mean interaction depth at
# normal incidence), LYSO attenuation 0.087 / mm at 511 keV; 5 degree angle
# bins as the 5D LUT, 16 position bins across a gap.
EDGE_BLOCKS = dict(depth_mm=25.0, doi_mm=8.0, mu_per_mm=0.087)
EDGE_N_ANGLE = 36
EDGE_N_POS = 16

# The paper's LUT shape (Methods, "Photon detection probability LUT"): 5 keV
# energy bins over the 0-511 keV source spectrum (103 bins, to 515 keV),
# 5 degree bins of both incidence angles, 18 transaxial (16 crystals and two
# gap halves) and 55 axial (5 blocks of 9 rings and two gap halves each)
# crystal indices: 132 M entries.
PAPER_LUT_DIMS = (103, 36, 36, 18, 55)
PAPER_LUT_E_RANGE = (0.0, 515.0)

# Gap policy of each LUT mode (Methods, "Photon detection probability LUT"):
# no crystal information (or no LUT): discard; 3D with crystals: nearest edge
# crystal; 5D: the edge-crystal LUT.
GAP_POLICY_OF_MODE = {"lut5d": "edge_lut", "lut5d_paper": "edge_lut", "lut3d_crystals": "nearest",
                      "lut3d_angles": "discard", "lut1d": "discard", "nolut": "discard"}


def gap_desc(gaps: dict, policy: str) -> dict:
    """Gap description as the oracle and the library take it."""
    d = dict(gaps, policy=policy)
    if policy == "edge_lut":
        d.update(edge_n_angle=EDGE_N_ANGLE, edge_n_pos=EDGE_N_POS)
    return d


def edge_geometries(scanner: Scanner, gaps: dict):
    """(transaxial, axial) edge-LUT geometries: the transaxial gap's width is
    its angle times the detection radius (the angle between the two modules'
    faces is neglected, as in the paper)."""
    t = dict(EDGE_BLOCKS, gap_mm=float(np.float32(scanner.radius_mm * gaps["transaxial_gap_rad"])),
             n_angle=EDGE_N_ANGLE, n_pos=EDGE_N_POS)
    a = dict(EDGE_BLOCKS, gap_mm=float(gaps["axial_gap_mm"]), n_angle=EDGE_N_ANGLE, n_pos=EDGE_N_POS)
    return t, a


def gap_lut_dims(scanner: Scanner, dims) -> tuple:
    """LUT dims with the virtual gap indices on the crystal axes (an axis of
    size 1 stays 1): crystals_per_module + 2 transaxial, n_blocks
    (rings_per_block + 2) axial."""
    nb = scanner.n_rings // scanner.rings_per_block
    d = list(dims)
    if d[3] != 1:
        d[3] = scanner.crystals_per_module + 2
    if d[4] != 1:
        d[4] = nb * (scanner.rings_per_block + 2)
    return tuple(d)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even); returns uint16 bits."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def make_sensitivity(sino: Sinogram, seed: int = 3, tof_axis: bool = True) -> np.ndarray:
    """Smooth positive synthetic scatter-sensitivity sinogram:
    1 + 0.2 cos(a view + b) cos(c rad + d) (1 + 0.05 cos(e plane)), phases from the seed."""
    rng = np.random.default_rng(seed)
    a, c, e = rng.uniform(1.0, 4.0, size=3)
    b, d = rng.uniform(0.0, 2.0 * math.pi, size=2)
    view = np.arange(sino.n_view)[:, None]
    rad = np.arange(sino.n_rad)[None, :]
    vr = (0.2 * np.cos(a * 2 * math.pi * view / sino.n_view + b)
          * np.cos(c * 2 * math.pi * rad / sino.n_rad + d)).astype(np.float32)
    pl = (1.0 + 0.05 * np.cos(e * 2 * math.pi * np.arange(sino.n_plane) / sino.n_plane)).astype(np.float32)
    s = ((1.0 + vr)[None, :, :] * pl[:, None, None]).astype(np.float32)
    if tof_axis:
        s = np.broadcast_to(s[None], sino.shape).copy()
    return s


def sens_at(sino: Sinogram, seed: int, tof, plane, view, rad) -> np.ndarray:
    """Values of make_sensitivity at given bin coordinates without building the
    whole array (same float32 rounding steps)."""
    rng = np.random.default_rng(seed)
    a, c, e = rng.uniform(1.0, 4.0, size=3)
    b, d = rng.uniform(0.0, 2.0 * math.pi, size=2)
    vr = (0.2 * np.cos(a * 2 * math.pi * np.asarray(view) / sino.n_view + b)
          * np.cos(c * 2 * math.pi * np.asarray(rad) / sino.n_rad + d)).astype(np.float32)
    pl = (1.0 + 0.05 * np.cos(e * 2 * math.pi * np.asarray(plane) / sino.n_plane)).astype(np.float32)
    return ((np.float32(1.0) + vr) * pl).astype(np.float32)
