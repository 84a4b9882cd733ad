"""k-space filter of the reconstructed image, float64 (test infrastructure).

Methods, "Computation of k-space filters" (and the last line of both
reconstruction listings): the filtered image is IFFT(FFT(rho) o f).  The
filter f marks the Cartesian k-space grid points that lie inside the convex
hull of the k-space positions given by the first-order field terms; the
paper computes it with a Delaunay triangulation of those positions and a
point-location test, which is what `kspace_filter_mask` does (scipy's
Delaunay triangulation and find_simplex as the library steps).

Conventions: images are [L] with voxel index x + nx (y + ny z); the filter
is [L] in the same index space, where index (u, v, w) is the FFT bin of
signed frequency (u if u < ceil(n/2) else u - n) along each axis, in cycles
per field of view (numpy.fft.fftfreq(n) * n).  First-order positions are
given in the same units.

Only tests/, the smoke check and the benchmark's CPU baseline use this
module.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay


def grid_frequencies(dims):
    """Signed frequency of every FFT bin, [L][d], in the image index order."""
    axes = [np.fft.fftfreq(n) * n for n in dims]  # (fx, fy[, fz])
    grids = np.meshgrid(*reversed(axes), indexing="ij")  # (..., fy, fx) arrays in (z, y, x) order
    cols = [g.ravel() for g in reversed(grids)]  # fx, fy[, fz], x fastest
    return np.stack(cols, axis=1)


def kspace_filter_mask(kpos, dims):
    """f (float64 0/1, [L]) = 1 where the grid frequency lies in the convex
    hull of the first-order positions kpos [K][d] (cycles per FOV)."""
    tri = Delaunay(np.asarray(kpos, dtype=np.float64))
    inside = tri.find_simplex(grid_frequencies(dims)) >= 0
    return inside.astype(np.float64)


def apply_kspace_filter(rho, f, dims):
    """IFFT(FFT(rho) o f) over the image grid."""
    shape = tuple(reversed(dims))
    x = np.asarray(rho, dtype=np.complex128).reshape(shape)
    F = np.fft.fftn(x)
    return np.fft.ifftn(F * np.asarray(f, dtype=np.float64).reshape(shape)).ravel()
