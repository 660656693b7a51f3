"""Independent binary64 geometry used by the tests to pin the oracle and the
HIP path: crystal / ring / LUT bins recomputed from raw hit data with numpy's
arctan2 in degrees, sinogram coordinates from crystal-centre geometry, exact
ray chords through voxel grids (Siddon's parametric method)."""
from __future__ import annotations

import numpy as np


def crystal_of(hx, hy, n_crystals):
    phi = np.mod(np.arctan2(hy, hx), 2 * np.pi)
    f = phi / (2 * np.pi / n_crystals)
    return np.minimum(np.floor(f).astype(np.int64), n_crystals - 1), f


def ring_of(hz, length, n_rings):
    f = (hz + length / 2) / (length / n_rings)
    return np.clip(np.floor(f).astype(np.int64), 0, n_rings - 1), f


def angle_bins(h, d, n_t, n_a):
    """Transaxial and axial incidence angles (degrees) between the path and
    the hit point's position vector, and their bins of width 180/n over
    [-90, 90]."""
    hx, hy = h[:, 0].astype(np.float64), h[:, 1].astype(np.float64)
    dx, dy, dz = (d[:, i].astype(np.float64) for i in range(3))
    rho = np.hypot(hx, hy)
    nrx, nry = hx / rho, hy / rho
    radial = nrx * dx + nry * dy
    tangential = -nry * dx + nrx * dy
    th_t = np.degrees(np.arctan2(tangential, radial))
    th_a = np.degrees(np.arctan2(dz, radial))
    ft = (th_t + 90.0) / (180.0 / n_t)
    fa = (th_a + 90.0) / (180.0 / n_a)
    return (np.clip(np.floor(ft).astype(np.int64), 0, n_t - 1), ft,
            np.clip(np.floor(fa).astype(np.int64), 0, n_a - 1), fa)


def crystal_centre_angle(c, n):
    return 2 * np.pi * (np.asarray(c, np.float64) + 0.5) / n


def lor_geometry(c1, c2, n, radius):
    """View index, signed radial index, and which crystal is the TOF-positive
    end, computed from the LOR between crystal centres: the view angle psi in
    [0, pi) is the direction of the LOR normal, the signed distance s along
    (cos psi, sin psi), the TOF-positive end has the larger projection on
    (-sin psi, cos psi).  Views pair neighbouring angle steps (pi / n each)."""
    p1 = crystal_centre_angle(c1, n)
    p2 = crystal_centre_angle(c2, n)
    e1 = np.stack([np.cos(p1), np.sin(p1)], -1) * radius
    e2 = np.stack([np.cos(p2), np.sin(p2)], -1) * radius
    t = e2 - e1
    normal = np.stack([-t[..., 1], t[..., 0]], -1)
    psi = np.mod(np.arctan2(normal[..., 1], normal[..., 0]), np.pi)
    k = np.rint(psi / (np.pi / n)).astype(np.int64)
    k = np.where(k == n, 0, k)
    psi = k * (np.pi / n)
    nv = np.stack([np.cos(psi), np.sin(psi)], -1)
    s = (e1 * nv).sum(-1)
    rho = np.rint(np.arcsin(np.clip(s / radius, -1, 1)) / (np.pi / n)).astype(np.int64)
    tv = np.stack([-np.sin(psi), np.cos(psi)], -1)
    a_pos = (e1 * tv).sum(-1) > (e2 * tv).sum(-1)
    return k // 2, rho, a_pos, s


def box_chord(pos, d, lo, hi):
    """Distance from pos along d to the exit of the box [lo, hi] (binary64)."""
    t = np.full(len(pos), np.inf)
    for i in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            tp = np.where(d[:, i] > 0, (hi[i] - pos[:, i]) / d[:, i],
                          np.where(d[:, i] < 0, (lo[i] - pos[:, i]) / d[:, i], np.inf))
        t = np.minimum(t, tp)
    return t


def siddon_line_integral(pos, d, mu, lo, vox):
    """Exact sum of mu_v * length_v along rays from pos in direction d to the
    exit of the voxel grid (Siddon 1985, parametric form), binary64.
    mu is [nz][ny][nx]."""
    nz, ny, nx = mu.shape
    n = np.array([nx, ny, nz])
    lo = np.asarray(lo, np.float64)
    vox = np.asarray(vox, np.float64)
    hi = lo + n * vox
    tmax = box_chord(pos, d, lo, hi)
    ts = [np.zeros((len(pos), 1)), tmax[:, None]]
    for i in range(3):
        planes = lo[i] + np.arange(n[i] + 1) * vox[i]
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = (planes[None, :] - pos[:, i:i + 1]) / d[:, i:i + 1]
        tt = np.where((tt > 0) & (tt < tmax[:, None]), tt, np.inf)
        ts.append(tt)
    t = np.sort(np.concatenate(ts, 1), axis=1)
    t = np.where(np.isinf(t), tmax[:, None], t)
    seg = np.diff(t, axis=1)
    mid = 0.5 * (t[:, 1:] + t[:, :-1])
    p = pos[:, None, :] + mid[:, :, None] * d[:, None, :]
    idx = np.floor((p - lo) / vox).astype(np.int64)
    idx = np.clip(idx, 0, n - 1)
    vals = mu[idx[..., 2], idx[..., 1], idx[..., 0]].astype(np.float64)
    return (vals * seg).sum(1)
