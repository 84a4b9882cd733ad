"""Pins of the FP64 stopping-criteria oracle (oracle/quality.py): SSIM against
closed forms and invariants of its published definition, the L-curve
curvature against circles and polylines."""
import numpy as np
import pytest

from oracle import quality as Q


def rand_img(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).ravel()


@pytest.mark.parametrize("dims", [(20, 17), (14, 13, 12)])
def test_ssim_of_identical_images_is_one(dims):
    x = rand_img(tuple(reversed(dims)), 1)
    assert abs(Q.ssim(x, x, dims) - 1.0) < 1e-14


def test_ssim_of_constant_images_closed_form():
    dims = (16, 15)
    a, b = 0.7, 1.9
    x = np.full(16 * 15, a)
    y = np.full(16 * 15, b)
    D = 1.0
    c1 = (0.01 * D) ** 2
    expect = (2 * a * b + c1) / (a * a + b * b + c1)  # the structure term is C2 / C2
    assert abs(Q.ssim(x, y, dims, data_range=D) - expect) < 1e-14


@pytest.mark.parametrize("dims", [(19, 16), (13, 12, 14)])
def test_ssim_of_checkerboards_closed_form(dims):
    """a = 1 + c/2, b = 1 - c/2 with the +-1 checkerboard c: every window
    sees mu = 1 +- s^d / 2, var = (1 - s^(2d)) / 4 and cov = -var, with s the
    alternating sum of the 1D window, which gives one SSIM value for every
    position (and D = 1)."""
    shape = tuple(reversed(dims))
    c = np.ones(shape)
    for ax, n in enumerate(shape):
        sl = [None] * len(shape)
        sl[ax] = slice(None)
        c = c * ((-1.0) ** np.arange(n))[tuple(sl)]
    a = (1 + 0.5 * c).ravel()
    b = (1 - 0.5 * c).ravel()
    w = Q.gaussian_window_1d()
    s = float(np.sum(w * (-1.0) ** np.arange(len(w))))
    sd = s ** len(dims)
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    mumu = 1 - 0.25 * sd * sd
    musq = 2 + 0.5 * sd * sd
    var = 0.25 * (1 - sd * sd)
    expect = ((2 * mumu + c1) * (-2 * var + c2)) / ((musq + c1) * (2 * var + c2))
    assert abs(Q.ssim(a, b, dims) - expect) < 1e-13


def test_ssim_symmetry_and_scale_invariance():
    dims = (18, 21)
    x = rand_img((21, 18), 2)
    y = x + 0.3 * rand_img((21, 18), 3)
    D = 2.5
    assert abs(Q.ssim(x, y, dims, D) - Q.ssim(y, x, dims, D)) < 1e-14
    assert abs(Q.ssim(3.0 * x, 3.0 * y, dims, 3.0 * D) - Q.ssim(x, y, dims, D)) < 1e-13
    assert Q.ssim(x, y, dims, D) < 1.0


def test_ssim_brute_force_tiny():
    """Explicit window sums at every valid position of a 13 x 12 image."""
    nx, ny = 13, 12
    x = rand_img((ny, nx), 4)
    y = rand_img((ny, nx), 5)
    a = np.abs(x).reshape(ny, nx)
    b = np.abs(y).reshape(ny, nx)
    w = Q.gaussian_window_1d()
    D = b.max() - b.min()
    c1, c2 = (0.01 * D) ** 2, (0.03 * D) ** 2
    vals = []
    for py in range(ny - 10):
        for px in range(nx - 10):
            sa = sb = 0.0
            for dy in range(11):
                for dx in range(11):
                    sa += w[dy] * w[dx] * a[py + dy, px + dx]
                    sb += w[dy] * w[dx] * b[py + dy, px + dx]
            va = vb = cv = 0.0
            for dy in range(11):
                for dx in range(11):
                    wt = w[dy] * w[dx]
                    va += wt * (a[py + dy, px + dx] - sa) ** 2
                    vb += wt * (b[py + dy, px + dx] - sb) ** 2
                    cv += wt * (a[py + dy, px + dx] - sa) * (b[py + dy, px + dx] - sb)
            vals.append(((2 * sa * sb + c1) * (2 * cv + c2)) / ((sa * sa + sb * sb + c1) * (va + vb + c2)))
    assert abs(Q.ssim(x, y, (nx, ny)) - np.mean(vals)) < 1e-13


def test_menger_curvature_on_circles():
    R = 2.5
    th = np.linspace(0.1, 1.4, 9)
    x, y = 1.0 + R * np.cos(th), -3.0 + R * np.sin(th)
    k = Q.menger_curvature(x, y)
    assert np.isnan(k[0]) and np.isnan(k[-1])
    assert np.allclose(k[1:-1], 1.0 / R, rtol=1e-12)
    k = Q.menger_curvature(x[::-1], y[::-1])  # clockwise
    assert np.allclose(k[1:-1], -1.0 / R, rtol=1e-12)


def test_lcurve_corner_of_a_polyline():
    """log||d|| falls steeply for 7 iterates, then log||rho|| grows at
    nearly constant log||d||: the corner (largest counter-clockwise turn) is
    iterate 7; row 0 (rho = 0) is skipped; scaling either norm moves the
    curve without changing its curvature."""
    n = 15
    lx = np.concatenate([np.linspace(0.0, 0.1, 7), 0.1 + np.linspace(0.2, 2.0, n - 7)])
    ly = np.concatenate([np.linspace(3.0, 0.2, 7), 0.2 - np.linspace(0.01, 0.1, n - 7)])
    hist = np.zeros((n + 1, 3))
    hist[1:, 1] = np.exp(lx)
    hist[1:, 2] = np.exp(2 * ly)
    hist[:, 0] = 1.0
    corner, kap = Q.lcurve_corner(hist)
    assert corner == 7
    assert np.isnan(kap[0]) and np.isnan(kap[1]) and np.isnan(kap[n])
    h2 = hist.copy()
    h2[:, 1] *= 7.0
    h2[:, 2] *= 0.01
    c2, k2 = Q.lcurve_corner(h2)
    assert c2 == 7 and np.allclose(k2[2:n], kap[2:n], rtol=1e-9)
    assert Q.lcurve_corner(hist[:3])[0] == -1
