"""Pins of the FP64 k-space filter oracle (oracle/postproc.py)."""
import numpy as np
import pytest

from oracle import postproc as PP


def rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("dims", [(12, 10), (6, 8, 5)])
def test_all_pass_filter_is_identity(dims):
    L = int(np.prod(dims))
    x = rand(L, 1)
    assert np.allclose(PP.apply_kspace_filter(x, np.ones(L), dims), x, atol=1e-13)


def test_single_bin_filter_projects_on_one_fourier_mode():
    """f = indicator of bin (u, v): the result is (1/N) <e, x> e with
    e[n] = exp(2 pi i (u ix / nx + v iy / ny))."""
    nx, ny = 9, 8
    u, v = 2, 5
    ix = np.tile(np.arange(nx), ny)
    iy = np.repeat(np.arange(ny), nx)
    e = np.exp(2j * np.pi * (u * ix / nx + v * iy / ny))
    x = rand(nx * ny, 2)
    f = np.zeros(nx * ny)
    f[u + nx * v] = 1.0
    want = np.vdot(e, x) / (nx * ny) * e
    assert np.allclose(PP.apply_kspace_filter(x, f, (nx, ny)), want, atol=1e-13)


def test_grid_frequencies_order():
    fr = PP.grid_frequencies((4, 3))
    # x fastest; signed frequencies 0, 1, -2, -1 along x and 0, 1, -1 along y
    assert fr[:4, 0].tolist() == [0, 1, -2, -1] and fr[:4, 1].tolist() == [0, 0, 0, 0]
    assert fr[4:8, 1].tolist() == [1, 1, 1, 1] and fr[8:12, 1].tolist() == [-1, -1, -1, -1]


def test_mask_of_a_square_and_a_triangle():
    """Hull of a square's corners (plus interior points) = the grid points
    inside the square; a triangle against a barycentric brute force."""
    dims = (16, 16)
    sq = np.array([[-3.5, -2.5], [4.5, -2.5], [4.5, 5.5], [-3.5, 5.5], [0.1, 0.2], [1.3, -1.1]])
    f = PP.kspace_filter_mask(sq, dims)
    fr = PP.grid_frequencies(dims)
    want = (fr[:, 0] >= -3.5) & (fr[:, 0] <= 4.5) & (fr[:, 1] >= -2.5) & (fr[:, 1] <= 5.5)
    assert np.array_equal(f.astype(bool), want)
    tri = np.array([[-6.3, -5.1], [6.7, -2.2], [-1.4, 7.3]])
    f = PP.kspace_filter_mask(tri, dims)
    a, b, c = tri
    want = []
    for p in fr:
        d = (b[1] - c[1]) * (a[0] - c[0]) + (c[0] - b[0]) * (a[1] - c[1])
        l1 = ((b[1] - c[1]) * (p[0] - c[0]) + (c[0] - b[0]) * (p[1] - c[1])) / d
        l2 = ((c[1] - a[1]) * (p[0] - c[0]) + (a[0] - c[0]) * (p[1] - c[1])) / d
        want.append(l1 >= 0 and l2 >= 0 and 1 - l1 - l2 >= 0)
    assert np.array_equal(f.astype(bool), np.array(want))


def test_binary_filter_is_a_projection():
    dims = (14, 11)
    rng = np.random.default_rng(3)
    k = rng.uniform(-5, 5, size=(40, 2))
    f = PP.kspace_filter_mask(k, dims)
    x = rand(14 * 11, 4)
    y = PP.apply_kspace_filter(x, f, dims)
    assert np.allclose(PP.apply_kspace_filter(y, f, dims), y, atol=1e-13)
    assert np.linalg.norm(y) <= np.linalg.norm(x)
