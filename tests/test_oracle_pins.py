"""Pins of the FP64 oracle against facts fixed by the paper's model and by
mathematics: scalar brute force, the Cartesian DFT special case (checked
against an index-formula DFT and against numpy.fft), a hand-evaluated single
voxel, the adjoint identity, the Gram identity, dense normal-equation solves,
CG invariants and finite-difference gradients.

Each pin is chosen so that a plausible slip in the oracle (a dropped B0 or
higher-order term, a flipped exponent sign, a missing conjugate, a transposed
operand, a wrong CG scalar) fails at least one of them.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import synth


def _args(d):
    return (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------------------------- brute force
@pytest.mark.parametrize("L,K,G,P", [(12, 20, 3, 4), (7, 13, 2, 16), (5, 9, 1, 1)])
def test_E_and_EH_match_scalar_triple_loop(L, K, G, P):
    d = synth.random_problem(L, K, G, P, seed=1)
    a = _args(d)
    ref = np.array(oracle.E_brute(d["rho"], *a))
    assert _rel(oracle.apply_E(d["rho"], *a, block=4), ref) < 1e-12
    refh = np.array(oracle.EH_brute(d["m"], *a))
    assert _rel(oracle.apply_EH(d["m"], *a, block=4), refh) < 1e-12


# ------------------------------------------------------ Cartesian DFT special case
def _dft_index_formula(img, n):
    """m[ky, kx] = sum_{y, x} img[y, x] exp(+2 pi i ((kx - n/2)(x - n/2) + (ky - n/2)(y - n/2)) / n)."""
    out = np.zeros((n, n), dtype=np.complex128)
    for ky in range(n):
        for kx in range(n):
            acc = 0j
            for y in range(n):
                for x in range(n):
                    ang = 2 * math.pi * ((kx - n / 2) * (x - n / 2) + (ky - n / 2) * (y - n / 2)) / n
                    acc += img[y, x] * cmath.exp(1j * ang)
            out[ky, kx] = acc
    return out


@pytest.mark.parametrize("n", [4, 8])
def test_E_equals_dft_on_cartesian_grid(n, rng):
    d = synth.dft_problem(n, exact=True)
    img = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    m = oracle.apply_E(img.ravel(), *_args(d))[0].reshape(n, n)
    # index-formula DFT with a + sign
    assert _rel(m, _dft_index_formula(img, n)) < 1e-12
    # the same transform through numpy.fft, with explicit centring shifts
    via_fft = np.fft.fftshift(n * n * np.fft.ifft2(np.fft.ifftshift(img)))
    assert _rel(m, via_fft) < 1e-12
    # and the adjoint is the forward FFT with the same shifts
    data = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    x = oracle.apply_EH(data.ravel()[None, :], *_args(d)).reshape(n, n)
    assert _rel(x, np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(data)))) < 1e-12


def test_unitary_gram_on_full_cartesian_grid(rng):
    n = 8
    d = synth.dft_problem(n, exact=True)
    p = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    q = oracle.apply_EHE(p, *_args(d))
    assert _rel(q, d["K"] * p) < 1e-12


# ------------------------------------------------------------ closed forms
def test_single_voxel_closed_form():
    """rho = delta at one voxel gives m[c, k] = S_c exp(i phi) with a phase
    evaluated by hand for simple numbers (x = 0.5, k_x = 4 rad, dt = 1 ms,
    B0 = 2 pi 100 rad/s), so the B0 term and its sign are pinned."""
    fields = np.array([[0.5, -0.25]], dtype=np.float32)  # one basis term h = x
    b0 = np.array([2 * np.pi * 100.0, 0.0], dtype=np.float32)
    kcoef = np.array([[4.0], [-2.0], [0.0]], dtype=np.float32)
    t = np.array([0.0, 1e-3, 2e-3], dtype=np.float32)
    sens = np.array([[0.5 + 0.5j, 1.0], [2.0j, 1.0]], dtype=np.complex64)
    rho = np.array([1.0, 0.0], dtype=np.complex128)
    m = oracle.apply_E(rho, sens, fields, b0, kcoef, t)
    b0_32 = float(np.float32(2 * np.pi * 100.0))
    t1 = float(np.float32(1e-3))
    t2 = float(np.float32(2e-3))
    phis = [2.0, -1.0 + t1 * b0_32, t2 * b0_32]  # 4*0.5, -2*0.5 + 0.2*pi, 0.4*pi
    for c, s in enumerate([0.5 + 0.5j, 2.0j]):
        want = [s * cmath.exp(1j * ph) for ph in phis]
        np.testing.assert_allclose(m[c], want, rtol=1e-12, atol=1e-12)
    # second voxel only: phase -k*0.25, no B0
    m2 = oracle.apply_E(np.array([0, 1.0]), sens, fields, b0, kcoef, t)
    np.testing.assert_allclose(m2[0], [cmath.exp(-1j), cmath.exp(0.5j), 1.0], rtol=1e-12, atol=1e-12)


def test_phase_hand_evaluated_and_consistent_with_E():
    """oracle.phase (the exponent K R) on the numbers of the single-voxel
    pin, evaluated by hand: row k, column l is sum_b kcoef[k, b] h_b(l) +
    t[k] b0[l].  Two basis terms (h = x and h = 1) so that a transposed or
    dropped term shows.  Then exp(i phase) column l, weighted by S_c(l), is
    E applied to the unit vector at l (a sign slip in either fails)."""
    fields = np.array([[0.5, -0.25], [1.0, 1.0]], dtype=np.float32)
    b0 = np.array([2 * np.pi * 100.0, 0.0], dtype=np.float32)
    kcoef = np.array([[4.0, 0.25], [-2.0, 0.0], [0.0, -1.5]], dtype=np.float32)
    t = np.array([0.0, 1e-3, 2e-3], dtype=np.float32)
    ph = oracle.phase(kcoef, t, fields, b0)
    b0_32 = float(np.float32(2 * np.pi * 100.0))
    t1, t2 = float(np.float32(1e-3)), float(np.float32(2e-3))
    want = np.array([[2.0 + 0.25, -1.0 + 0.25],
                     [-1.0 + t1 * b0_32, 0.5],
                     [-1.5 + t2 * b0_32, -1.5]])
    np.testing.assert_allclose(ph, want, rtol=0, atol=1e-15)
    sens = np.array([[0.5 + 0.5j, 1.0], [2.0j, -1.0]], dtype=np.complex64)
    for l in range(2):
        e = np.zeros(2)
        e[l] = 1.0
        m = oracle.apply_E(e, sens, fields, b0, kcoef, t)
        np.testing.assert_allclose(m, sens[:, l:l + 1].astype(np.complex128) * np.exp(1j * ph[:, l])[None, :],
                                   rtol=1e-13, atol=1e-13)


def test_E_is_linear(rng):
    d = synth.random_problem(40, 50, 3, 5, seed=2)
    a = _args(d)
    x = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    y = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    lhs = oracle.apply_E((2 - 1j) * x + 0.5 * y, *a)
    rhs = (2 - 1j) * oracle.apply_E(x, *a) + 0.5 * oracle.apply_E(y, *a)
    assert _rel(lhs, rhs) < 1e-13


# ------------------------------------------------------------ adjoint / Gram
@pytest.mark.parametrize("shape", [(1024, 2048, 4, 4), (300, 777, 5, 16)])
def test_adjoint_identity(shape):
    L, K, G, P = shape
    d = synth.random_problem(L, K, G, P, seed=3)
    a = _args(d)
    lhs = np.vdot(oracle.apply_E(d["rho"], *a), d["m"])
    rhs = np.vdot(d["rho"], oracle.apply_EH(d["m"], *a))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_adjoint_identity_on_config_c1():
    d = synth.make_config("c1")
    rng = np.random.default_rng(7)
    rho = rng.standard_normal(d["L"]) + 1j * rng.standard_normal(d["L"])
    m = rng.standard_normal((d["n_coil"], d["K"])) + 1j * rng.standard_normal((d["n_coil"], d["K"]))
    a = _args(d)
    lhs = np.vdot(oracle.apply_E(rho, *a), m)
    rhs = np.vdot(rho, oracle.apply_EH(m, *a))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_gram_identity_and_split_form():
    d = synth.random_problem(200, 333, 4, 16, seed=4)
    a = _args(d)
    p = d["rho"].astype(np.complex128)
    q = oracle.apply_EHE(p, *a, block=37)
    Ep = oracle.apply_E(p, *a)
    quad = np.vdot(p, q)
    assert abs(quad.real - np.vdot(Ep, Ep).real) / abs(quad) < 1e-12
    assert abs(quad.imag) / abs(quad) < 1e-12
    assert _rel(q, oracle.apply_EH(Ep, *a)) < 1e-12


def test_block_size_does_not_change_results():
    d = synth.random_problem(64, 100, 3, 4, seed=5)
    a = _args(d)
    r1 = oracle.apply_EH(d["m"], *a, block=1)
    r2 = oracle.apply_EH(d["m"], *a, block=1000)
    assert _rel(r1, r2) < 1e-13


# ------------------------------------------------------------------- CG
def test_cg_reaches_dense_normal_equation_solve():
    d = synth.random_problem(6, 8, 2, 4, seed=6, phase_scale=3.0)
    a = _args(d)
    Ed = oracle.dense_E(*a)
    m = d["m"].astype(np.complex128)
    ref = np.linalg.solve(Ed.conj().T @ Ed, Ed.conj().T @ m.ravel())
    res = oracle.cg_solve(m, *a, n_iter=6)
    assert res["iters"] == 6
    assert _rel(res["rho"], ref) < 1e-9


def test_cg_rank_deficient_gives_minimum_norm_solution():
    d = synth.random_problem(10, 4, 2, 4, seed=7, phase_scale=3.0)  # 8 equations, 10 unknowns
    a = _args(d)
    Ed = oracle.dense_E(*a)
    m = d["m"].astype(np.complex128)
    ref = np.linalg.lstsq(Ed, m.ravel(), rcond=None)[0]
    res = oracle.cg_solve(m, *a, n_iter=8)
    assert _rel(res["rho"], ref) < 1e-8
    assert _rel(res["rho"], np.linalg.pinv(Ed) @ m.ravel()) < 1e-8


def test_cg_unitary_case_converges_in_one_step(rng):
    n = 8
    d = synth.dft_problem(n, exact=True)
    a = _args(d)
    m = rng.standard_normal((1, d["K"])) + 1j * rng.standard_normal((1, d["K"]))
    res = oracle.cg_solve(m, *a, n_iter=1)
    assert _rel(res["rho"], oracle.apply_EH(m, *a) / d["K"]) < 1e-13
    assert res["hist"][1, 0] / res["hist"][0, 0] < 1e-12
    # a tolerance stop fires right after that step
    res2 = oracle.cg_solve(m, *a, n_iter=5, tol=1e-8)
    assert res2["iters"] == 1 and res2["status"] == "tol"


def test_cg_krylov_invariants_and_residual_recurrence():
    d = synth.random_problem(30, 40, 3, 4, seed=8, phase_scale=4.0)
    a = _args(d)
    m = d["m"].astype(np.complex128)
    res = oracle.cg_solve(m, *a, n_iter=8, return_iterates=True, explicit_residual=True)
    rhs = oracle.apply_EH(m, *a)
    its = [np.zeros(30)] + res["iterates"]
    rs = [rhs - oracle.apply_EHE(x, *a) for x in its]
    # residuals are mutually orthogonal
    for i in range(len(rs)):
        for j in range(i):
            assert abs(np.vdot(rs[i], rs[j])) < 1e-9 * np.linalg.norm(rs[i]) * np.linalg.norm(rs[j]) + 1e-20
    # directions are A-conjugate: consecutive iterate differences
    ds = [its[i + 1] - its[i] for i in range(len(its) - 1)]
    for i in range(len(ds)):
        Ai = oracle.apply_EHE(ds[i], *a)
        for j in range(i):
            assert abs(np.vdot(ds[j], Ai)) < 1e-8 * np.linalg.norm(ds[j]) * np.linalg.norm(Ai)
    # recursive residual norm equals the true one; data-residual recurrence holds
    for n in range(len(its)):
        assert abs(res["hist"][n, 0] - np.linalg.norm(rs[n])) < 1e-9 * res["hist"][0, 0]
    np.testing.assert_allclose(res["hist"][1:, 2], res["dres"], rtol=1e-9)
    # the A-norm of the error decreases monotonically towards the LS solution
    Ed = oracle.dense_E(*a)
    xs = np.linalg.lstsq(Ed, m.ravel(), rcond=None)[0]
    errs = [np.real(np.vdot(x - xs, oracle.apply_EHE(x - xs, *a))) for x in its]
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_cg_constant_intensity_correction_is_invisible():
    d = synth.random_problem(20, 30, 2, 4, seed=9, phase_scale=4.0)
    a = _args(d)
    m = d["m"].astype(np.complex128)
    r0 = oracle.cg_solve(m, *a, n_iter=5)
    r1 = oracle.cg_solve(m, *a, n_iter=5, icorr=np.full(20, 2.5))
    assert _rel(r1["rho"], r0["rho"]) < 1e-12


def test_cg_converged_solution_independent_of_intensity_correction():
    d = synth.random_problem(6, 8, 2, 4, seed=10, phase_scale=3.0)
    a = _args(d)
    m = d["m"].astype(np.complex128)
    Ed = oracle.dense_E(*a)
    ref = np.linalg.lstsq(Ed, m.ravel(), rcond=None)[0]
    j = np.random.default_rng(3).uniform(0.5, 2.0, size=6)
    res = oracle.cg_solve(m, *a, n_iter=6, icorr=j)
    assert _rel(res["rho"], ref) < 1e-8


def test_cg_zero_data_stops_immediately():
    d = synth.random_problem(10, 12, 2, 4, seed=11)
    res = oracle.cg_solve(np.zeros((2, 12)), *_args(d), n_iter=5)
    assert res["iters"] == 0 and res["status"] == "exact"
    assert not np.any(res["rho"])


# ------------------------------------------------------------ gradients
def test_gradients_match_central_differences():
    d = synth.random_problem(9, 14, 2, 4, seed=12, phase_scale=3.0)
    sens, fields, b0, kcoef, t = (np.asarray(x, dtype=np.complex128 if np.iscomplexobj(x) else np.float64)
                                  for x in _args(d))
    rho = d["rho"].astype(np.complex128)
    m = d["m"].astype(np.complex128)
    loss, g_rho, g_b0, g_k = oracle.encode_grads(rho, m, sens, fields, b0, kcoef, t)

    def L(rho_=rho, b0_=b0, k_=kcoef):
        y = oracle.apply_E(rho_, sens, fields, b0_, k_, t)
        return float(np.real(np.vdot(y - m, y - m)))

    assert abs(loss - L()) < 1e-12 * loss
    h = 1e-5
    r = np.random.default_rng(0)
    for _ in range(3):
        v = r.standard_normal(9) + 1j * r.standard_normal(9)
        fd = (L(rho_=rho + h * v) - L(rho_=rho - h * v)) / (2 * h)
        assert abs(fd - np.real(np.vdot(g_rho, v))) < 1e-7 * abs(fd) + 1e-9
    for l in [0, 4, 8]:
        e = np.zeros(9)
        e[l] = 1.0
        hb = 1e-3  # b0 is in rad/s, t ~ 1e-5 s: a larger step keeps the FD well above rounding
        fd = (L(b0_=b0 + hb * e) - L(b0_=b0 - hb * e)) / (2 * hb)
        assert abs(fd - g_b0[l]) < 1e-6 * max(abs(fd), 1e-6 * loss)
    # per-term gains g_b: kcoef[:, b] <- (1 + g_b) kcoef[:, b]
    for b in range(4):
        e = np.zeros_like(kcoef)
        e[:, b] = kcoef[:, b]
        fd = (L(k_=kcoef + h * e) - L(k_=kcoef - h * e)) / (2 * h)
        assert abs(fd - np.sum(kcoef[:, b] * g_k[:, b])) < 1e-6 * max(abs(fd), 1e-3)
    # one random direction over all of kcoef
    v = r.standard_normal(kcoef.shape)
    fd = (L(k_=kcoef + h * v) - L(k_=kcoef - h * v)) / (2 * h)
    assert abs(fd - np.sum(v * g_k)) < 1e-6 * abs(fd)


# ------------------------------------------------- re-orthogonalised CG
def _galerkin_iterates(A, b, n):
    """Exact-arithmetic CG iterates as Galerkin solutions on the Krylov space
    K_n(A, b): x_n = Q_n (Q_n^H A Q_n)^{-1} Q_n^H b with Q_n an orthonormal
    basis built by Arnoldi with two Gram-Schmidt passes (dense, tiny)."""
    Q = [b / np.linalg.norm(b)]
    out = []
    for k in range(1, n + 1):
        Qm = np.stack(Q, axis=1)
        H = Qm.conj().T @ A @ Qm
        out.append(Qm @ np.linalg.solve(H, Qm.conj().T @ b))
        w = A @ Q[-1]
        for _ in range(2):
            w = w - Qm @ (Qm.conj().T @ w)
        Q.append(w / np.linalg.norm(w))
    return out


def test_reorth_cg_equals_krylov_galerkin_solution():
    d = synth.random_problem(40, 30, 2, 4, seed=13, phase_scale=6.0)
    a = _args(d)
    Ed = oracle.dense_E(*a)
    A = Ed.conj().T @ Ed
    m = d["m"].astype(np.complex128)
    b = Ed.conj().T @ m.ravel()
    ref = _galerkin_iterates(A, b, 12)
    res = oracle.cg_solve(m, *a, n_iter=12, return_iterates=True, reorth=True)
    for n in range(12):
        assert _rel(res["iterates"][n], ref[n]) < 1e-8, n


def test_reorth_matches_plain_cg_on_a_well_conditioned_problem():
    d = synth.random_problem(50, 200, 3, 4, seed=14, phase_scale=20.0)
    a = _args(d)
    m = d["m"].astype(np.complex128)
    r0 = oracle.cg_solve(m, *a, n_iter=10, return_iterates=True)
    r1 = oracle.cg_solve(m, *a, n_iter=10, return_iterates=True, reorth=True)
    for x, y in zip(r0["iterates"], r1["iterates"]):
        assert _rel(x, y) < 1e-12


def test_reorth_keeps_residuals_orthogonal_on_the_2d_spiral_config():
    d = synth.make_config("c1")
    a = _args(d)
    m = oracle.apply_E(d["rho_true"], *a) + 0.1 * d["noise"]
    res = oracle.cg_solve(m, *a, n_iter=20, return_iterates=True, reorth=True)
    rhs = oracle.apply_EH(m, *a)
    rs = [rhs] + [rhs - oracle.apply_EHE(x, *a) for x in res["iterates"]]
    U = np.stack([r / np.linalg.norm(r) for r in rs], axis=1)
    G = U.conj().T @ U
    assert np.max(np.abs(G - np.eye(len(rs)))) < 1e-6


# ---------------------------------------------------------------- rounding probe
def test_bf16_rounding_definition():
    """bfloat16 = float32 with the low 16 bits rounded off, nearest, ties to
    even: representable values stay, halfway cases go to the even neighbour,
    and every result is within half a unit in the last place."""
    from oracle.nfs_oracle import _bf16

    exact = np.array([1.0, -2.5, 0.0078125, 3.140625, 65280.0])
    assert np.array_equal(_bf16(exact), exact)
    ulp1 = 2.0 ** -7
    ties = np.array([1 + ulp1 / 2, 1 + 3 * ulp1 / 2, -(1 + ulp1 / 2)])
    assert np.array_equal(_bf16(ties), np.array([1.0, 1 + 2 * ulp1, -1.0]))
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).uniform(-3, 3, 10000)
    y = _bf16(x)
    assert np.all(y.astype(np.float32).view(np.uint32) & 0xFFFF == 0)
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))


def test_rounding_probe_is_exact_on_representable_operands():
    """Phases on multiples of pi/2 (cos, sin in {0, +-1}) and small integer
    data: every operand the probe rounds is representable, so E^H E and
    E^H sigma with fp16 or bf16 operand rounding equal the FP64 values."""
    from oracle import nfs_oracle as o

    rng = np.random.default_rng(4)
    L, K, G = 40, 64, 3
    fields = rng.integers(0, 4, size=(1, L)).astype(np.float64)
    kcoef = (np.pi / 2) * rng.integers(0, 2, size=(K, 1)).astype(np.float64)
    b0, t = np.zeros(L), np.zeros(K)
    sens = rng.integers(-2, 3, size=(G, L)) + 1j * rng.integers(-2, 3, size=(G, L))
    p = rng.integers(-3, 4, size=L) + 1j * rng.integers(-3, 4, size=L)
    m = rng.integers(-5, 6, size=(G, K)) + 1j * rng.integers(-5, 6, size=(G, K))
    a = (sens, fields, b0, kcoef, t)
    for fmt in ("fp16", "bf16"):
        q, qr = o.apply_EHE(p, *a), o.apply_EHE_rounded(p, *a, fmt)
        x, xr = o.apply_EH(m, *a), o.apply_EH_rounded(m, *a, fmt)
        assert np.max(np.abs(qr - q)) <= 1e-12 * np.max(np.abs(q)), fmt
        assert np.max(np.abs(xr - x)) <= 1e-12 * np.max(np.abs(x)), fmt


def test_rounding_probe_error_is_at_the_format_unit():
    """On a random problem the rounded E^H E differs from the FP64 one by the
    order of the format's unit roundoff (fp16 2^-11, bf16 2^-8 on the cos and
    sin operands), and the fp16 data scale puts the largest part in
    [2^13, 2^14)."""
    from oracle import nfs_oracle as o

    d = synth.random_problem(200, 400, 5, 6, seed=8)
    a = (d["sens"], d["fields"], d["b0"], d["kcoef"], d["t"])
    q = o.apply_EHE(d["rho"], *a)
    for fmt, lo, hi in (("fp16", 2.0 ** -16, 2.0 ** -10), ("bf16", 2.0 ** -13, 2.0 ** -7)):
        e = np.linalg.norm(o.apply_EHE_rounded(d["rho"], *a, fmt) - q) / np.linalg.norm(q)
        assert lo < e < hi, (fmt, e)
    z = d["m"] * 37.0
    sc = o._pow2_scale(z)
    top = max(np.max(np.abs(z.real)), np.max(np.abs(z.imag))) * sc
    assert 2.0 ** 13 <= top < 2.0 ** 14
