"""Reconstruction of the joint estimation loop on the GPU (TOF Joseph
projector, its transpose, TOF-OSEM, activity from an image) against the
binary64 oracle (oracle/recon.c).

Tolerance: the kernels work in binary32.  A projected bin sums at most a few
hundred samples, each a product of rounded interpolation, path and TOF
weights (the TOF weight a difference of binary32 erfc values, within a few
ulp), so relative errors stay near 1e-6 of the LOR's total; the tests allow
1e-4 relative plus 2e-5 of the largest bin.  OSEM compounds such errors over
its subsets: 1e-3 relative on the image."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import harness as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_05047_amd as sse  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def close(got, ref, rtol=1e-4, atol_frac=2e-5):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    atol = atol_frac * np.abs(ref).max()
    bad = np.abs(got - ref) > rtol * np.abs(ref) + atol
    assert not bad.any(), (int(bad.sum()), float(np.abs(got - ref).max()), float(np.abs(ref).max()))


def setup(which, tof_sigma=None, n_tof=None):
    w = W.WORKLOADS[which]
    sino = w.sino if tof_sigma is None else W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": tof_sigma})
    if n_tof is not None:  # the same TOF range in n_tof bins
        span = sino.n_tof * sino.tof_bin_mm
        sino = W.Sinogram(**{**sino.__dict__, "n_tof": n_tof, "tof_bin_mm": span / n_tof})
    pd, mu, act = W.make_phantom(w)
    ctx = sse.Context(w.scanner, sino, w.physics)
    pid = ctx.load_phantom(pd, mu, act)
    return w, sino, pd, mu, act, ctx, pid


def smooth_image(pd, n_plane, seed):
    rng = np.random.default_rng(seed)
    x = pd.lo_mm[0] + (np.arange(pd.nx) + 0.5) * pd.voxel_mm[0]
    y = pd.lo_mm[1] + (np.arange(pd.ny) + 0.5) * pd.voxel_mm[1]
    img = np.zeros((n_plane, pd.ny, pd.nx))
    for _ in range(5):
        c = rng.uniform(-0.3, 0.3, 2) * np.array([pd.nx * pd.voxel_mm[0], pd.ny * pd.voxel_mm[1]])
        s = rng.uniform(5, 20)
        g = np.exp(-((x[None] - c[0]) ** 2 + (y[:, None] - c[1]) ** 2) / (2 * s * s))
        img += rng.uniform(0.5, 2.0) * g[None] * rng.uniform(0.5, 1.5, (n_plane, 1, 1))
    return img.astype(np.float32)


@pytest.mark.parametrize("tof_sigma", [0.0, 20.0])
@pytest.mark.parametrize("tof", [False, True])
@pytest.mark.parametrize("subsets", [(0, 1), (3, 7)])
def test_projector_matches_oracle_tiny(tof_sigma, tof, subsets):
    w, sino, pd, mu, act, ctx, pid = setup("tiny", tof_sigma)
    try:
        img = smooth_image(pd, sino.n_plane, 1)
        shape = (sino.n_tof,) * tof + (sino.n_plane, sino.n_view, sino.n_rad)
        out = torch.full(shape, -7.0, dtype=torch.float32, device="cuda")
        s, n = subsets
        ctx.project(pid, torch.from_numpy(img).cuda(), out, tof=tof, subset=s, n_subsets=n)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        ctx.close()
    ref = O.recon_project(w.scanner, sino, pd, img, tof=tof, subset=s, n_subsets=n)
    views = np.arange(sino.n_view) % n == s
    close(got[..., views, :], ref[..., views, :])
    assert np.all(got[..., ~views, :] == -7.0)   # other views untouched


@pytest.mark.parametrize("tof_sigma", [0.0, 20.0])
@pytest.mark.parametrize("tof", [False, True])
@pytest.mark.parametrize("subsets", [(0, 1), (3, 7)])
def test_backprojector_matches_oracle_tiny(tof_sigma, tof, subsets):
    w, sino, pd, mu, act, ctx, pid = setup("tiny", tof_sigma)
    try:
        rng = np.random.default_rng(2)
        shape = (sino.n_tof,) * tof + (sino.n_plane, sino.n_view, sino.n_rad)
        y = rng.uniform(0, 1, shape).astype(np.float32)
        img = torch.full((sino.n_plane, pd.ny, pd.nx), -7.0, dtype=torch.float32, device="cuda")
        s, n = subsets
        ctx.backproject(pid, torch.from_numpy(y).cuda(), img, tof=tof, subset=s, n_subsets=n)
        torch.cuda.synchronize()
        got = img.cpu().numpy()
    finally:
        ctx.close()
    ref = O.recon_backproject(w.scanner, sino, pd, y, tof=tof, subset=s, n_subsets=n)
    close(got, ref)


@pytest.mark.parametrize("view", [0, 37, 111, 223])
def test_clinical_single_view_matches_oracle(view):
    """The clinical geometry (448 crystals, 357 x 224 x 89 x 29 TOF sinogram,
    128 x 128 image), one view as a subset of 224: forward and back."""
    w, sino, pd, mu, act, ctx, pid = setup("clinical")
    try:
        img = smooth_image(pd, sino.n_plane, 3)
        fw = torch.zeros((sino.n_tof, sino.n_plane, sino.n_view, sino.n_rad), dtype=torch.float32, device="cuda")
        ctx.project(pid, torch.from_numpy(img).cuda(), fw, tof=True, subset=view, n_subsets=sino.n_view)
        rng = np.random.default_rng(4)
        y = np.zeros((sino.n_tof, sino.n_plane, sino.n_view, sino.n_rad), np.float32)
        y[:, :, view, :] = rng.uniform(0, 1, (sino.n_tof, sino.n_plane, sino.n_rad))
        bp = torch.empty((sino.n_plane, pd.ny, pd.nx), dtype=torch.float32, device="cuda")
        ctx.backproject(pid, torch.from_numpy(y).cuda(), bp, tof=True, subset=view, n_subsets=sino.n_view)
        torch.cuda.synchronize()
        got_f = fw.cpu().numpy()[:, :, view, :]
        got_b = bp.cpu().numpy()
    finally:
        ctx.close()
    ref_f = O.recon_project(w.scanner, sino, pd, img, tof=True, subset=view, n_subsets=sino.n_view)[:, :, view, :]
    close(got_f, ref_f)
    ref_b = O.recon_backproject(w.scanner, sino, pd, y, tof=True, subset=view, n_subsets=sino.n_view)
    close(got_b, ref_b)


@pytest.mark.parametrize("which", ["tiny", "clinical"])
def test_gpu_projector_pair_is_adjoint(which):
    """<P x, y> = <P^T y, x> for the GPU pair on the full sinogram, summed
    in binary64 from the binary32 results."""
    w, sino, pd, mu, act, ctx, pid = setup(which)
    try:
        g = torch.Generator(device="cuda").manual_seed(5)
        x = torch.rand((sino.n_plane, pd.ny, pd.nx), device="cuda", generator=g)
        y = torch.rand((sino.n_tof, sino.n_plane, sino.n_view, sino.n_rad), device="cuda", generator=g)
        px = torch.empty_like(y)
        pty = torch.empty_like(x)
        ctx.project(pid, x, px, tof=True)
        ctx.backproject(pid, y, pty, tof=True)
        lhs = float((px.double() * y.double()).sum())
        rhs = float((pty.double() * x.double()).sum())
    finally:
        ctx.close()
    say(f"[recon] {which}: <Px,y> {lhs:.9e} <x,P'y> {rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)


# TOF bins per LOR in the compact subset layout: 8 (5 bins), 16 (11, the tiny
# workload's own) and 32 (29, the clinical workload's count)
@pytest.mark.parametrize("n_tof", [5, 11, 29])
def test_osem_matches_oracle_tiny(n_tof):
    w, sino, pd, mu, act, ctx, pid = setup("tiny", 20.0, n_tof)
    try:
        x_true = smooth_image(pd, sino.n_plane, 6).astype(np.float64)
        att = np.exp(-O.recon_project(w.scanner, sino, pd, 0.0096 * (x_true > 0.05), tof=False))
        mult = (att * W.make_sensitivity(sino, seed=3, tof_axis=False)).astype(np.float32)
        fwd = O.recon_project(w.scanner, sino, pd, x_true, tof=True)
        add = (0.3 * fwd.mean() * np.ones_like(fwd)).astype(np.float32)
        prompts = (mult[None] * fwd + add).astype(np.float32)
        x0 = np.full_like(x_true, x_true.mean()).astype(np.float32)
        img = torch.from_numpy(x0).cuda()
        dp, dm, da = (torch.from_numpy(a).cuda() for a in (prompts, mult, add))
        ctx.osem(pid, dp, dm, da, img, n_iter=2, n_subsets=4)
        # with the subset sensitivity images computed beforehand: the same bits
        img2 = torch.from_numpy(x0).cuda()
        sens = ctx.osem_sensitivity(pid, dm, 4)
        ctx.osem(pid, dp, dm, da, img2, n_iter=2, n_subsets=4, sens=sens)
        torch.cuda.synchronize()
        got = img.cpu().numpy()
        assert torch.equal(img, img2)
    finally:
        ctx.close()
    ref = O.recon_osem(w.scanner, sino, pd, prompts, mult, add, x0, n_iter=2, n_subsets=4)
    close(got, ref, rtol=1e-3, atol_frac=1e-4)


def test_image_to_activity_feeds_the_simulation():
    """An image turned into the phantom's activity (nearest plane per voxel
    slice, negatives to 0) gives the histories the oracle gives for that
    activity."""
    case = H.case_from("tiny")
    w = W.WORKLOADS["tiny"]
    sino = w.sino
    pd = case.pdesc
    img = smooth_image(pd, sino.n_plane, 8)
    img[0, :4, :4] = -1.0
    half_pitch = 0.5 * w.scanner.length_mm / w.scanner.n_rings
    z = pd.lo_mm[2] + (np.arange(pd.nz) + 0.5) * pd.voxel_mm[2]
    p = np.clip(np.rint((z + 0.5 * w.scanner.length_mm) / half_pitch - 1.0), 0, sino.n_plane - 1).astype(int)
    act = np.maximum(img[p], 0.0).astype(np.float32)
    ctx, pid = H.open_context(case)
    try:
        ctx.image_to_activity(pid, torch.from_numpy(img).cuda())
        g = H.run_gpu(ctx, pid, 20_000, 77, record_stride=1)
    finally:
        ctx.close()
    c2 = H.Case(case.scanner, case.sino, case.physics, case.pdesc, case.mu, act, case.lut_desc, case.lut,
                case.lut_store, case.lut_dtype)
    o = H.run_oracle(c2, 20_000, 77)
    same = H.identical_mask(g["records"], o["records"])
    assert same.mean() >= 0.999, H.describe_mismatch(g["records"], o["records"])


@pytest.mark.parametrize("which", ["tiny", "clinical"])
def test_attenuation_factors_match_oracle(which):
    """exp(-line integral) of the phantom's own attenuation map, each plane
    reading the voxel slice that holds its z, against the oracle projector on
    the same plane image."""
    w, sino, pd, mu, act, ctx, pid = setup(which)
    try:
        out = torch.empty((sino.n_plane, sino.n_view, sino.n_rad), dtype=torch.float32, device="cuda")
        ctx.attenuation_factors(pid, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        ctx.close()
    mu_img = W.plane_image(pd, mu, w.scanner)
    ref = np.exp(-O.recon_project(w.scanner, sino, pd, mu_img, tof=False))
    close(got, ref, rtol=1e-4, atol_frac=1e-6)
    assert got.min() > 0 and got.max() <= 1.0
