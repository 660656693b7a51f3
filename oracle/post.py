"""Binary64 definitions of the sinogram post-processing steps.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``apply_sensitivity``: the final scatter estimate is the LUT-weighted
  simulator sinogram times the LUT-specific scatter-sensitivity sinogram
  (Methods, "Scatter sensitivity sinogram"), scaled to absolute units
  (the simulator output is intrinsically scaled, Discussion) and rounded once
  to binary32.
* ``gaussian_smooth``: separable Gaussian smoothing of the scatter sinogram
  along the radial, angular and planar axes (Methods, "Known activity
  distribution, very limited simulation time"; FWHM given in bins in Results).
  Readings: the kernel is the normalised Gaussian truncated at
  ``int(truncate * sigma + 0.5)`` bins; radial and planar edges reflect with
  the edge sample repeated; the angular axis is periodic over pi with the
  LOR flipped across the seam (radial index r -> n_rad - 1 - r, TOF bin
  t -> n_tof - 1 - t); TOF bins are not smoothed.
* ``emission_scale``: expected emissions per simulated history.
"""
from __future__ import annotations

import numpy as np


def apply_sensitivity(weights: np.ndarray, scale: float, sens: np.ndarray) -> np.ndarray:
    """float32(scale * W * sens), evaluated in binary64.  ``sens`` has the
    sinogram shape or lacks the leading TOF axis (then it is shared by all TOF
    bins)."""
    w = np.asarray(weights, np.float64)
    s = np.asarray(sens, np.float64)
    if s.ndim == w.ndim - 1:
        s = s[None]
    return ((scale * w) * s).astype(np.float32)


def total_scatter(weights: np.ndarray, scale: float, sens: np.ndarray) -> float:
    """Total of the estimate: the sum over bins of the binary64 products
    (scale * W) * sens, summed exactly and rounded once (math.fsum).  ``sens``
    as in apply_sensitivity."""
    import math
    w = np.asarray(weights, np.float64)
    s = np.asarray(sens, np.float64)
    if s.ndim == w.ndim - 1:
        s = s[None]
    return math.fsum(((scale * w) * s).ravel().tolist())


def gaussian_kernel(sigma: float, truncate: float = 4.0):
    radius = int(truncate * sigma + 0.5)
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * x * x / (sigma * sigma))
    return w / w.sum(), radius


def reflect_index(i: np.ndarray, n: int) -> np.ndarray:
    """Half-sample symmetric extension (d c b a | a b c d | d c b a)."""
    period = 2 * n
    m = np.mod(i, period)
    return np.where(m < n, m, period - 1 - m)


def _smooth_rad(x, sigma, truncate):
    w, rad = gaussian_kernel(sigma, truncate)
    n = x.shape[-1]
    idx = np.arange(n)
    out = np.zeros_like(x)
    for k in range(-rad, rad + 1):
        out += w[k + rad] * x[..., reflect_index(idx + k, n)]
    return out


def _smooth_plane(x, sigma, truncate):
    w, rad = gaussian_kernel(sigma, truncate)
    n = x.shape[1]
    idx = np.arange(n)
    out = np.zeros_like(x)
    for k in range(-rad, rad + 1):
        out += w[k + rad] * x[:, reflect_index(idx + k, n), :, :]
    return out


def _smooth_view(x, sigma, truncate):
    w, rad = gaussian_kernel(sigma, truncate)
    nt, _, nv, nr = x.shape
    flipped = x[::-1, :, :, ::-1]          # same LOR seen from the other end
    out = np.zeros_like(x)
    v = np.arange(nv)
    for k in range(-rad, rad + 1):
        m = np.mod(v + k, 2 * nv)
        is_flip = m >= nv
        src = np.where(is_flip, m - nv, m)
        contrib = np.where(is_flip[None, None, :, None], flipped[:, :, src, :], x[:, :, src, :])
        out += w[k + rad] * contrib
    return out


def gaussian_smooth(sino: np.ndarray, sigma_bins, truncate: float = 4.0) -> np.ndarray:
    """Smooth a [tof][plane][view][rad] sinogram with per-axis sigma
    (rad, view, plane) in bins; a sigma of 0 leaves that axis alone.
    Returns binary64."""
    x = np.asarray(sino, np.float64)
    if x.ndim == 3:
        x = x[None]
    s_rad, s_view, s_plane = (float(s) for s in sigma_bins)
    if s_rad > 0:
        x = _smooth_rad(x, s_rad, truncate)
    if s_view > 0:
        x = _smooth_view(x, s_view, truncate)
    if s_plane > 0:
        x = _smooth_plane(x, s_plane, truncate)
    return x


def emission_scale(activity: np.ndarray, voxel_mm, n_histories: int, acq_seconds: float = 1.0,
                   factor: float = 1.0) -> float:
    """Expected annihilations per simulated history: total activity (per ml)
    times voxel volume (ml) times acquisition time, over the history count,
    times a global factor."""
    vol_ml = float(voxel_mm[0]) * float(voxel_mm[1]) * float(voxel_mm[2]) * 1e-3
    total = float(np.sum(np.asarray(activity, np.float64)))
    return total * vol_ml * acq_seconds / n_histories * factor


def gaussian_smooth_at(sino: np.ndarray, sigma_bins, points, truncate: float = 4.0) -> np.ndarray:
    """``gaussian_smooth(sino, sigma_bins, truncate)`` evaluated only at the
    given (tof, plane, view, rad) points (array of shape [m, 4]), from the
    same definition: radial pass, then view pass with the seam flip, then
    planar pass.  For checking large sinograms on sampled bins."""
    x = np.asarray(sino)
    if x.ndim == 3:
        x = x[None]
    nt, npl, nv, nr = x.shape
    pts = np.asarray(points, np.int64)
    t0, p0, v0, r0 = pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]

    def taps(s):
        if s > 0:
            return gaussian_kernel(float(s), truncate)
        return np.ones(1), 0

    wr, rr = taps(sigma_bins[0])
    wv, rv = taps(sigma_bins[1])
    wp, rp = taps(sigma_bins[2])
    out = np.zeros(len(pts))
    for a in range(-rp, rp + 1):
        p = reflect_index(p0 + a, npl) if rp else p0
        for b in range(-rv, rv + 1):
            if rv:
                m = np.mod(v0 + b, 2 * nv)
                flip = m >= nv
                v = np.where(flip, m - nv, m)
            else:
                flip = np.zeros(len(pts), bool)
                v = v0
            t = np.where(flip, nt - 1 - t0, t0)
            rbase = np.where(flip, nr - 1 - r0, r0)
            acc = np.zeros(len(pts))
            for c in range(-rr, rr + 1):
                r = reflect_index(rbase + c, nr) if rr else rbase
                acc += wr[c + rr] * x[t, p, v, r].astype(np.float64)
            out += wp[a + rp] * wv[b + rv] * acc
    return out


def smoothing_normalisation(weights: np.ndarray, scale: float, sigma_bins, truncate: float = 4.0) -> np.ndarray:
    """Smoothing normalisation sinogram (Methods, "Known activity
    distribution, very limited simulation time"): the scaled LUT scatter S of
    a reference object, heavily smoothed and divided by itself,
    N = G_heavy(S) / S, in binary64; 1 where S or G_heavy(S) is not positive
    (a reading: the paper does not say)."""
    S = scale * np.asarray(weights, np.float64)
    G = gaussian_smooth(S, sigma_bins, truncate).reshape(S.shape)
    N = np.ones_like(S)
    ok = (S > 0) & (G > 0)
    N[ok] = G[ok] / S[ok]
    return N


def finalize_normalised(weights: np.ndarray, scale: float, norm: np.ndarray, sigma_bins, sens: np.ndarray,
                        truncate: float = 4.0) -> np.ndarray:
    """Normalised smoothing of the scaled LUT scatter S = scale * W (same
    passage): multiply by the normalisation N, smooth, divide by N (entries
    <= 0 count as 1), multiply by the scatter sensitivity; binary64."""
    S = scale * np.asarray(weights, np.float64)
    N = np.asarray(norm, np.float64).reshape(S.shape)
    Nd = np.where(N > 0, N, 1.0)
    x = S * N
    sm = gaussian_smooth(x, sigma_bins, truncate).reshape(S.shape)
    s = np.asarray(sens, np.float64)
    if s.ndim == S.ndim - 1:
        s = s[None]
    return sm / Nd * s
