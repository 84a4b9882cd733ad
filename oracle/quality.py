"""Stopping-criteria instrumentation, float64 (test infrastructure only).

The paper studies the choice of the CG iteration count with two tools
(Methods, "Reconstruction algorithm", and the CG-convergence figure): the
L-curve of the residual norm against the solution norm, whose point of
maximum curvature is a proposed stopping point, and the structural
similarity index (SSIM) of each iterate against a reference image.  Neither
formula is printed in the paper; the readings below are the published
definitions it cites.

SSIM (Wang, Bovik, Sheikh and Simoncelli, 2004), on magnitude images:
  * window: Gaussian, sigma = 1.5, truncated to 11 taps per axis and
    normalised to unit sum; the 2D/3D window is the outer product of the
    1D window over the image axes;
  * constants C1 = (0.01 D)^2, C2 = (0.03 D)^2 with D = max - min of the
    reference magnitude;
  * local statistics mu, sigma^2 and sigma_xy weighted by the window,
    without sample-size correction, at every window position that lies
    fully inside the image (no padding);
  * SSIM = mean over those positions of
      (2 mu_a mu_b + C1)(2 sigma_ab + C2) / ((mu_a^2 + mu_b^2 + C1)(sigma_a^2 + sigma_b^2 + C2)).

L-curve corner: the curve is (log ||rho_n||, log ||d_n||) for the iterates
n = 1, 2, ... (rho_0 = 0 has no logarithm); the curvature at an interior
point is the signed curvature of the circle through it and its two
neighbours (Menger curvature, 4 x signed area / product of the three side
lengths); the corner is the point of largest curvature.  Points whose norms
are not positive and finite are left out.

Only tests/, the smoke check and the benchmark's CPU baseline use this
module.
"""
from __future__ import annotations

import numpy as np

SSIM_SIGMA = 1.5
SSIM_TAPS = 11
SSIM_K1 = 0.01
SSIM_K2 = 0.03


def gaussian_window_1d(sigma: float = SSIM_SIGMA, taps: int = SSIM_TAPS):
    """Normalised 1D Gaussian of `taps` taps centred on the middle tap."""
    i = np.arange(taps, dtype=np.float64) - (taps - 1) / 2.0
    w = np.exp(-(i * i) / (2.0 * sigma * sigma))
    return w / w.sum()


def _window(ndim):
    w1 = gaussian_window_1d()
    w = w1
    for _ in range(ndim - 1):
        w = np.multiply.outer(w, w1)
    return w


def ssim(img, ref, dims, data_range=None) -> float:
    """Mean SSIM of |img| against |ref|; both [L] with voxel index
    x + nx (y + ny z) for dims (nx, ny) or (nx, ny, nz)."""
    shape = tuple(reversed(dims))  # (ny, nx) or (nz, ny, nx): x fastest
    a = np.abs(np.asarray(img, dtype=np.complex128)).reshape(shape)
    b = np.abs(np.asarray(ref, dtype=np.complex128)).reshape(shape)
    D = float(b.max() - b.min()) if data_range is None else float(data_range)
    c1 = (SSIM_K1 * D) ** 2
    c2 = (SSIM_K2 * D) ** 2
    W = _window(len(shape))
    wa = np.lib.stride_tricks.sliding_window_view(a, W.shape)
    wb = np.lib.stride_tricks.sliding_window_view(b, W.shape)
    axes = tuple(range(len(shape), 2 * len(shape)))
    idx = (Ellipsis,) + (None,) * len(shape)
    mu_a = np.tensordot(wa, W, axes=(axes, tuple(range(len(shape)))))
    mu_b = np.tensordot(wb, W, axes=(axes, tuple(range(len(shape)))))
    da = wa - mu_a[idx]
    db = wb - mu_b[idx]
    var_a = np.tensordot(da * da, W, axes=(axes, tuple(range(len(shape)))))
    var_b = np.tensordot(db * db, W, axes=(axes, tuple(range(len(shape)))))
    cov = np.tensordot(da * db, W, axes=(axes, tuple(range(len(shape)))))
    smap = ((2 * mu_a * mu_b + c1) * (2 * cov + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) * (var_a + var_b + c2))
    return float(smap.mean())


def menger_curvature(x, y):
    """Signed curvature of the circle through consecutive point triples:
    k[i] for the interior points i = 1 .. n-2 (NaN at both ends); positive
    for a counter-clockwise turn."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    k = np.full(x.shape, np.nan)
    for i in range(1, len(x) - 1):
        ax, ay = x[i] - x[i - 1], y[i] - y[i - 1]
        bx, by = x[i + 1] - x[i], y[i + 1] - y[i]
        cx, cy = x[i + 1] - x[i - 1], y[i + 1] - y[i - 1]
        cross = ax * by - ay * bx  # twice the signed triangle area
        den = np.hypot(ax, ay) * np.hypot(bx, by) * np.hypot(cx, cy)
        k[i] = 2.0 * cross / den if den > 0 else np.nan
    return k


def lcurve_corner(hist):
    """Corner of the L-curve from a CG history [n+1][3] (rows: ||r_n||,
    ||rho_n||, ||d_n||^2).  Returns (iterate index of the corner, or -1 if
    fewer than three usable points; curvature per row, NaN where undefined)."""
    h = np.asarray(hist, dtype=np.float64)
    rows = [n for n in range(len(h))
            if np.isfinite(h[n, 1]) and np.isfinite(h[n, 2]) and h[n, 1] > 0 and h[n, 2] > 0]
    kap = np.full(len(h), np.nan)
    if len(rows) < 3:
        return -1, kap
    xs = np.log(h[rows, 1])
    ys = 0.5 * np.log(h[rows, 2])
    k = menger_curvature(xs, ys)
    for j, n in enumerate(rows):
        kap[n] = k[j]
    best = -1
    for j in range(1, len(rows) - 1):
        if np.isfinite(k[j]) and (best < 0 or k[j] > kap[best]):
            best = rows[j]
    return best, kap
