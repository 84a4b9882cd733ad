"""Pins of the FP64 map-estimation oracle (oracle/maps.py)."""
import numpy as np
import pytest

from oracle import maps as M


def test_difference_operators_on_polynomials():
    """D2 of x^2 along x is 2 at every interior row, D1 of x is 1; both
    vanish along the other axis; rows sit where the neighbours exist."""
    dims = (7, 5, 4)
    L = 7 * 5 * 4
    idx = np.arange(L)
    ix = idx % 7
    D2, r2 = M._diff_matrix(dims, 0, 2)
    D1, r1 = M._diff_matrix(dims, 0, 1)
    assert np.allclose(D2 @ (ix.astype(float) ** 2), 2.0)
    assert np.allclose(D1 @ ix.astype(float), 1.0)
    assert len(r2) == 5 * 5 * 4 and len(r1) == 6 * 5 * 4
    D2y, _ = M._diff_matrix(dims, 1, 2)
    D1z, _ = M._diff_matrix(dims, 2, 1)
    assert np.allclose(D2y @ (ix.astype(float) ** 2), 0.0)
    assert np.allclose(D1z @ ix.astype(float), 0.0)


def test_initial_sensitivities_of_rank_one_data():
    """x[c, n, l] = s_l[c] e_l[n]: the first left singular vector is s_l / |s_l|
    up to phase; with the coil-sum convention it is fixed exactly."""
    rng = np.random.default_rng(1)
    G, ne, L = 6, 5, 40
    s = rng.standard_normal((G, L)) + 1j * rng.standard_normal((G, L))
    e = rng.standard_normal((ne, L)) + 1j * rng.standard_normal((ne, L))
    X = s[:, None, :] * e[None, :, :]
    got = M.sens_initial(X)
    t = s.sum(axis=0)
    want = s / np.linalg.norm(s, axis=0) * (np.conj(t) / np.abs(t))
    assert np.allclose(got, want, atol=1e-12)
    assert np.allclose(np.imag(got.sum(axis=0)), 0.0, atol=1e-12) and np.all(np.real(got.sum(axis=0)) > 0)


def test_sensitivity_smoothing_keeps_data_without_penalty():
    dims = (9, 8)
    L = 72
    rng = np.random.default_rng(2)
    s = (1 + rng.random((3, L))) * np.exp(1j * rng.uniform(-3, 3, (3, L)))
    got = M.smooth_sens(s, np.ones(L), np.ones(L), dims, 0.0)
    assert np.allclose(got, s, atol=1e-12)


def test_sensitivity_smoothing_extrapolates_affine_maps_exactly():
    """|S^| affine and phase constant: both parts have zero second
    differences, so the solution equals S^ on all of M_R, also where M_T has
    no data."""
    dims = (16, 14)
    L = 16 * 14
    ix = np.arange(L) % 16
    iy = np.arange(L) // 16
    mag = 2.0 + 0.05 * ix - 0.03 * iy
    s = np.stack([mag * np.exp(0.7j), (3.0 - 0.02 * ix + 0.04 * iy) * np.exp(-1.1j)])
    mR = ((ix >= 2) & (ix <= 13) & (iy >= 1) & (iy <= 12)).astype(float)
    mT = ((ix >= 5) & (ix <= 10) & (iy >= 4) & (iy <= 9)).astype(float)
    got = M.smooth_sens(s, mT, mR, dims, 3.0)
    inner = (ix >= 2) & (ix <= 13) & (iy >= 1) & (iy <= 12)
    assert np.allclose(got[:, inner], s[:, inner], atol=1e-9)


def test_b0_fit_recovers_exact_phases_with_wraps():
    """Noise-free echoes with per-echo steps up to 0.9 pi (several wraps over
    the echo train) and an even/odd offset: slope, offset and zero residual."""
    rng = np.random.default_rng(3)
    G, ne, L, dte = 4, 7, 50, 1e-3
    S = rng.standard_normal((G, L)) + 1j * rng.standard_normal((G, L))
    w = rng.uniform(-0.9 * np.pi, 0.9 * np.pi, L) / dte
    beta = 0.3
    rho = rng.uniform(0.5, 2.0, L) * np.exp(1j * rng.uniform(-np.pi, np.pi, L))
    X = np.stack([S * (rho * np.exp(1j * (w * n * dte + beta * (n % 2))))[None, :] for n in range(ne)], axis=1)
    b0, b, eps = M.b0_initial(X, S, dte)
    assert np.allclose(b0, w, rtol=1e-10, atol=1e-7)
    assert np.allclose(b, beta, atol=1e-10)
    assert np.allclose(eps, 0.0, atol=1e-10)


def test_b0_smoothing_special_cases():
    dims = (10, 9)
    L = 90
    rng = np.random.default_rng(4)
    b = rng.standard_normal(L)
    assert np.allclose(M.smooth_b0(b, np.zeros(L), dims, 5.0), b, atol=1e-12)
    c = np.full(L, 3.7)
    assert np.allclose(M.smooth_b0(c, rng.random(L), dims, 5.0), c, atol=1e-12)
    # larger eps smooths more: the result moves towards the mean
    s1 = M.smooth_b0(b, np.full(L, 0.1), dims, 5.0)
    s2 = M.smooth_b0(b, np.full(L, 1.0), dims, 5.0)
    assert np.std(s2) < np.std(s1) < np.std(b)


def test_sensitivity_smoothing_weights_data_by_the_trusted_mask():
    """Without penalty the data rows read diag(M_T) S = S^, so a mask of
    constant value m gives S = S^ / m."""
    dims = (6, 5)
    rng = np.random.default_rng(5)
    s = (1 + rng.random((2, 30))) * np.exp(1j * rng.uniform(-3, 3, (2, 30)))
    got = M.smooth_sens(s, np.full(30, 0.5), np.ones(30), dims, 0.0)
    assert np.allclose(got, 2.0 * s, atol=1e-12)


def test_initial_sensitivities_of_an_empty_voxel_are_zero():
    X = np.zeros((3, 4, 5), dtype=np.complex128)
    X[:, :, 2] = np.arange(12).reshape(3, 4) + 1j
    got = M.sens_initial(X)
    assert np.all(got[:, [0, 1, 3, 4]] == 0)
    assert abs(np.linalg.norm(got[:, 2]) - 1.0) < 1e-12


def _stacked_rows(dims, order):
    """Rows of D_order along every axis, by explicit loops over voxels (no
    shared code with the oracle's sparse assembly): list of (centre voxel,
    {voxel: coefficient})."""
    nx = dims[0]
    ny = dims[1]
    nz = dims[2] if len(dims) == 3 else 1
    rows = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                c = (x, y, z)
                for ax, n in enumerate((nx, ny, nz)):
                    def vid(o):
                        q = list(c)
                        q[ax] += o
                        return q[0] + nx * (q[1] + ny * q[2])
                    if order == 2 and 1 <= c[ax] <= n - 2:
                        rows.append((vid(0), {vid(-1): 1.0, vid(0): -2.0, vid(1): 1.0}))
                    if order == 1 and c[ax] <= n - 2:
                        rows.append((vid(0), {vid(0): -1.0, vid(1): 1.0}))
    return rows


def _dense_lstsq(dims, data_w, data, pen_w, alpha, order):
    """Least-squares solution of the stacked system as printed in the
    smoothing equations: [diag(data_w); sqrt(alpha) diag(pen_w) D] x = [data; 0],
    by numpy's dense lstsq."""
    L = int(np.prod(dims))
    rows = _stacked_rows(dims, order)
    A = np.zeros((L + len(rows), L))
    A[np.arange(L), np.arange(L)] = data_w
    for r, (ctr, coefs) in enumerate(rows):
        for v, cf in coefs.items():
            A[L + r, v] = np.sqrt(alpha) * pen_w[ctr] * cf
    b = np.concatenate([data, np.zeros(len(rows))])
    return np.linalg.lstsq(A, b, rcond=None)[0], A


@pytest.mark.parametrize("dims", [(9, 7), (5, 4, 4)])
def test_sensitivity_smoothing_is_the_stacked_least_squares_solution(dims):
    """Random non-binary masks (every voxel carries data, so the system has
    full column rank): each smoothed component equals the dense lstsq
    solution of the stacked system [diag(M_T); sqrt(a) diag(M_R) D2] S = [S^; 0]."""
    rng = np.random.default_rng(8)
    L = int(np.prod(dims))
    mT = 0.3 + rng.random(L)
    mR = rng.random(L)
    s = (1 + rng.random((2, L))) * np.exp(1j * rng.uniform(-1, 1, (2, L)))
    alpha = 2.5
    got = M.smooth_sens(s, mT, mR, dims, alpha)
    for c in range(2):
        mag = np.abs(s[c])
        nrm = s[c] / mag
        m_s, _ = _dense_lstsq(dims, mT, mag, mR, alpha, 2)
        re_s, _ = _dense_lstsq(dims, mT, nrm.real, mR, alpha, 2)
        im_s, _ = _dense_lstsq(dims, mT, nrm.imag, mR, alpha, 2)
        n_s = re_s + 1j * im_s
        want = m_s * n_s / np.abs(n_s)
        assert np.allclose(got[c], want, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("dims", [(8, 6), (4, 5, 3)])
def test_b0_smoothing_is_the_stacked_least_squares_solution(dims):
    rng = np.random.default_rng(9)
    L = int(np.prod(dims))
    b0 = rng.standard_normal(L) * 50
    eps = rng.random(L)
    got = M.smooth_b0(b0, eps, dims, 7.0)
    want, _ = _dense_lstsq(dims, np.ones(L), b0, eps, 7.0, 1)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-10)
