"""Seeded synthetic workloads shaped like the paper's 2D and 3D spiral data.

The paper reconstructs measured 2D single-shot spirals and 3D T-Hex spirals
(Methods, "Dataset description"; captions of the 2D/3D spiral figures: 1 mm
in-plane resolution, 16 receive coils, readouts up to 71.5 ms, R up to 7,
dynamic field terms up to 3rd order from a 16-probe field camera).  That
dataset is not available, so every workload here is synthetic, with the
shapes, value ranges and structure listed below.  All arrays are produced in
float64 and rounded once to float32 / complex64; those rounded values are the
canonical inputs seen by both the oracle and the GPU library.

Conventions (signal model of the "Implementation" section: the temporal basis
K holds t and k_p(t), the spatial basis R holds B0(r) and h_p(r)):

* voxel coordinates are normalised per axis, x = (n - N/2) / (N/2) in [-1, 1);
  2D slices sit at z = 0.1 so that z-dependent basis terms are not trivial;
  voxel index l = (iz * Ny + iy) * Nx + ix;
* the spatial basis h_p is the list of unnormalised real solid harmonics up to
  3rd order given by ``solid_harmonics`` (the paper names field terms "up to
  3rd order" but does not print their definition);
* k_p(t) are in radians per unit of h_p; k_1, k_2 (and k_3 in 3D) follow an
  Archimedean spiral-out with k_max = pi * N / 2 (Nyquist for the normalised
  coordinates); k_0 and higher-order terms are 1e-3 * k_max times a seeded
  smooth waveform of unit RMS (3 sinusoids, 1-3 cycles per readout);
* t restarts at every shot, 2 us dwell;
* b0 is returned in rad/s (2*pi times the Hz map), so that t * b0 is a phase;
* sensitivities: |S| = exp(-|r - c|^2 / 2) around coil centres c on a circle
  of radius 1.5 (rings in 3D), phase 2*pi*j/G + 0.5 (r - c) . u_j;
* phantom: 10 random ellipses (ellipsoids in 3D) times exp(0.3 i x);
* noise: unit complex Gaussian (each component N(0, 1)); callers scale it to
  the SNR they want once the noiseless data exist.

Seeds come from numpy.random.SeedSequence(260409233 + config index), spawned
once per component, so every component is reproducible on its own.
"""
from __future__ import annotations

import math

import numpy as np

DWELL = 2e-6  # s

# name -> (index, recipe)
CONFIGS = {
    "c1": dict(index=0, dims=(32, 32), n_coil=4, n_basis=4, shots=1, interleaves=1,
               k_shot=2048, b0_hz=50.0, b0_kind="bump", n_iter=20),
    "c2": dict(index=1, dims=(128, 128), n_coil=16, n_basis=16, shots=4, interleaves=16,
               k_shot=15000, b0_hz=100.0, b0_kind="smooth_noise", n_iter=30),
    "c3": dict(index=2, dims=(96, 96, 48), n_coil=32, n_basis=16, shots=16, interleaves=16,
               k_shot=35750, b0_hz=150.0, b0_kind="gauss3d", n_iter=15),
    # gradient workload: same shapes as c2
    "c4": dict(index=3, dims=(128, 128), n_coil=16, n_basis=16, shots=4, interleaves=16,
               k_shot=15000, b0_hz=100.0, b0_kind="smooth_noise", n_iter=0),
    # scaled-down 3D case for iterate-level tests (48x48x24, 8 coils, 4 x 8000 samples)
    "c3s": dict(index=10, dims=(48, 48, 24), n_coil=8, n_basis=16, shots=4, interleaves=4,
                k_shot=8000, b0_hz=150.0, b0_kind="gauss3d", n_iter=15),
}

_SEED_BASE = 260409233


def _streams(index: int, n: int = 8):
    ss = np.random.SeedSequence(_SEED_BASE + index)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def grid_coords(dims, z_slice: float = 0.1):
    """Normalised voxel coordinates (x, y, z), each of length L, float64."""
    if len(dims) == 2:
        nx, ny = dims
        ix = np.arange(nx)
        iy = np.arange(ny)
        xx = (ix - nx / 2) / (nx / 2)
        yy = (iy - ny / 2) / (ny / 2)
        y, x = np.meshgrid(yy, xx, indexing="ij")
        z = np.full_like(x, z_slice)
        return x.ravel(), y.ravel(), z.ravel()
    nx, ny, nz = dims
    xx = (np.arange(nx) - nx / 2) / (nx / 2)
    yy = (np.arange(ny) - ny / 2) / (ny / 2)
    zz = (np.arange(nz) - nz / 2) / (nz / 2)
    z, y, x = np.meshgrid(zz, yy, xx, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def solid_harmonics(x, y, z, n_terms: int):
    """Real solid harmonics up to 3rd order, unnormalised, in a fixed order.

    Order: 1, x, y, z, xy, zy, 3z^2-r^2, xz, x^2-y^2, 3x^2y-y^3, xyz,
    (5z^2-r^2)y, 5z^3-3zr^2, (5z^2-r^2)x, z(x^2-y^2), x^3-3xy^2.
    Returns float64 [n_terms][L].
    """
    r2 = x * x + y * y + z * z
    terms = [
        np.ones_like(x), x, y, z,
        x * y, z * y, 3 * z * z - r2, x * z, x * x - y * y,
        3 * x * x * y - y ** 3, x * y * z, (5 * z * z - r2) * y, 5 * z ** 3 - 3 * z * r2,
        (5 * z * z - r2) * x, z * (x * x - y * y), x ** 3 - 3 * x * y * y,
    ]
    if n_terms > len(terms):
        raise ValueError("at most 16 basis terms are defined")
    return np.stack(terms[:n_terms])


def _smooth_waveforms(rng, n_wave: int, tau):
    """n_wave seeded sums of 3 sinusoids (1-3 cycles per readout), unit RMS."""
    out = np.zeros((n_wave, tau.size))
    for w in range(n_wave):
        g = np.zeros(tau.size)
        for _ in range(3):
            f = rng.uniform(1.0, 3.0)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(0.5, 1.0)
            g += a * np.sin(2 * np.pi * f * tau + ph)
        g /= np.sqrt(np.mean(g * g))
        out[w] = g
    return out


def _trajectory(cfg, rng):
    """kcoef [K][P] (rad) and t [K] (s) for the spiral recipe of a config."""
    dims = cfg["dims"]
    n = cfg.get("k_grid", dims[0])  # acquisition matrix (k_max); the grid may be coarser
    k_shot = cfg["k_shot"]
    shots = cfg["shots"]
    P = cfg["n_basis"]
    kmax = math.pi * n / 2
    tau = np.arange(k_shot) / k_shot
    blocks_k = []
    blocks_t = []
    for s in range(shots):
        kc = np.zeros((k_shot, P))
        if len(dims) == 2:
            n_turns = n / (2 * cfg["interleaves"])
            theta0 = 2 * np.pi * s / shots
            kz = np.zeros(k_shot)
        else:
            n_turns = round(48 / 7) if n >= 96 else max(1, round(n / 14))
            theta0 = 2 * np.pi * s / shots
            nz = dims[2]
            # tilted shots: each covers 3 kz lines around its own centre
            spread = nz / shots
            kz = math.pi * ((s - (shots - 1) / 2) * spread + spread * (tau - 0.5))
        theta = 2 * np.pi * n_turns * tau + theta0
        kc[:, 1] = kmax * tau * np.cos(theta)
        if P > 2:
            kc[:, 2] = kmax * tau * np.sin(theta)
        if P > 3:
            kc[:, 3] = kz
        extra = [0] + list(range(4, P))
        wav = _smooth_waveforms(rng, len(extra), tau)
        for i, b in enumerate(extra):
            kc[:, b] = 1e-3 * kmax * wav[i]
        blocks_k.append(kc)
        blocks_t.append(np.arange(k_shot) * DWELL)
    return np.concatenate(blocks_k), np.concatenate(blocks_t)


def _gauss_filter(a, sigma):
    from scipy.ndimage import gaussian_filter

    return gaussian_filter(a, sigma, mode="wrap")


def _b0_map(cfg, rng, x, y, z):
    dims = cfg["dims"]
    kind = cfg["b0_kind"]
    if kind == "bump":
        cx, cy = rng.uniform(-0.3, 0.3, size=2)
        f = np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 0.4 ** 2))
    elif kind == "smooth_noise":
        w = rng.standard_normal(dims[::-1])
        f = _gauss_filter(w, dims[0] / 16).ravel()
    else:
        f = np.zeros_like(x)
        for _ in range(8):
            c = rng.uniform(-0.6, 0.6, size=3)
            wdt = rng.uniform(0.15, 0.4)
            sgn = rng.choice([-1.0, 1.0])
            f += sgn * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * wdt * wdt))
    lo, hi = f.min(), f.max()
    f = (f - lo) / (hi - lo) * 2 - 1 if hi > lo else np.zeros_like(f)
    return 2 * np.pi * cfg["b0_hz"] * f  # rad/s


def _sensitivities(n_coil, rng, x, y, z, three_d):
    L = x.size
    S = np.zeros((n_coil, L), dtype=np.complex128)
    r = np.stack([x, y, z], axis=1)
    if three_d:
        per_ring = 8
        n_ring = max(1, int(math.ceil(n_coil / per_ring)))
        zs = np.linspace(-0.75, 0.75, n_ring)
    for j in range(n_coil):
        if three_d:
            ring, k = divmod(j, per_ring)
            ang = 2 * np.pi * k / per_ring + 0.3 * ring
            c = np.array([1.5 * np.cos(ang), 1.5 * np.sin(ang), zs[ring]])
        else:
            ang = 2 * np.pi * j / n_coil
            c = np.array([1.5 * np.cos(ang), 1.5 * np.sin(ang), 0.0])
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        d = r - c
        mag = np.exp(-np.sum(d * d, axis=1) / 2)
        ph = 2 * np.pi * j / n_coil + 0.5 * d @ u
        S[j] = mag * np.exp(1j * ph)
    return S


def _phantom(rng, x, y, z, three_d, n_obj=10):
    rho = np.zeros(x.size)
    for _ in range(n_obj):
        c = rng.uniform(-0.5, 0.5, size=3)
        ax = rng.uniform(0.1, 0.5, size=3)
        a = rng.uniform(0.2, 1.0)
        th = rng.uniform(0, np.pi)
        xr = (x - c[0]) * np.cos(th) + (y - c[1]) * np.sin(th)
        yr = -(x - c[0]) * np.sin(th) + (y - c[1]) * np.cos(th)
        q = (xr / ax[0]) ** 2 + (yr / ax[1]) ** 2
        if three_d:
            q = q + ((z - c[2]) / ax[2]) ** 2
        rho += a * (q <= 1.0)
    return rho * np.exp(0.3j * x)


def unit_noise(rng, shape):
    """Complex Gaussian noise with N(0, 1) real and imaginary parts."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def make_config(name: str, with_noise: bool = True):
    """Build one named workload.  Returns a dict of numpy arrays and sizes.

    Keys: name, dims, L, K, n_coil, n_basis, n_iter, sens [G][L] c64,
    fields [P][L] f32, b0 [L] f32 (rad/s), kcoef [K][P] f32 (rad),
    t [K] f32 (s), rho_true [L] c64, noise [G][K] c64 (unit) if with_noise.
    """
    cfg = CONFIGS[name]
    rs = _streams(cfg["index"])
    dims = cfg["dims"]
    three_d = len(dims) == 3
    x, y, z = grid_coords(dims)
    P = cfg["n_basis"]
    kcoef, t = _trajectory(cfg, rs[0])
    fields = solid_harmonics(x, y, z, P)
    b0 = _b0_map(cfg, rs[1], x, y, z)
    sens = _sensitivities(cfg["n_coil"], rs[2], x, y, z, three_d)
    rho = _phantom(rs[3], x, y, z, three_d)
    out = dict(
        name=name, dims=dims, L=x.size, K=t.size, n_coil=cfg["n_coil"], n_basis=P,
        n_iter=cfg["n_iter"],
        sens=sens.astype(np.complex64), fields=fields.astype(np.float32),
        b0=b0.astype(np.float32), kcoef=kcoef.astype(np.float32), t=t.astype(np.float32),
        rho_true=rho.astype(np.complex64),
    )
    if with_noise:
        out["noise"] = unit_noise(rs[4], (cfg["n_coil"], t.size))
    return out


def reconstruction_mask(d, dilate: int = 2):
    """Reconstruction mask M_R of a synthetic workload: the voxels where the
    phantom is non-zero, dilated by ``dilate`` voxels (grid connectivity 1
    per step).  The paper reconstructs only inside M_R, the head region of
    its prescan (Methods, "Computation of masks"); for the synthetic phantom
    its support plays that part.  Returns bool [L] in voxel order."""
    from scipy.ndimage import binary_dilation

    shape = tuple(reversed(d["dims"]))
    inside = (np.abs(d["rho_true"]) > 0).reshape(shape)
    if dilate > 0:
        inside = binary_dilation(inside, iterations=dilate)
    return inside.ravel()


def restrict_voxels(d, mask):
    """The workload with its voxel set restricted to ``mask`` (bool [L]):
    sens, fields, b0 and rho_true keep the masked voxels in voxel order;
    the sample side (kcoef, t, noise) is unchanged.  Since rho_true is zero
    outside its support, data built from it are the same for the full and
    the restricted problem."""
    mask = np.asarray(mask, dtype=bool)
    out = dict(d)
    out.update(sens=np.ascontiguousarray(d["sens"][:, mask]), fields=np.ascontiguousarray(d["fields"][:, mask]),
               b0=np.ascontiguousarray(d["b0"][mask]), rho_true=np.ascontiguousarray(d["rho_true"][mask]),
               L=int(mask.sum()), mask=mask, name=d.get("name", "") + "_masked")
    return out


def random_problem(L: int, K: int, n_coil: int, n_basis: int, seed: int,
                   phase_scale: float = 20.0, b0_hz: float = 100.0):
    """Small random problem with realistic magnitudes (tests only).

    fields are uniform in [-1, 1]; kcoef are uniform with a spread of
    ``phase_scale`` rad for the first three terms and 1e-3 of that for the
    rest; t is a 2 us raster; b0 is uniform in +-b0_hz (as rad/s); sens has
    magnitude in [0.2, 1] and random phase; rho and m are complex Gaussian.
    """
    rng = np.random.default_rng(np.random.SeedSequence([_SEED_BASE, L, K, n_coil, n_basis, seed]))
    fields = rng.uniform(-1, 1, size=(n_basis, L))
    kcoef = rng.uniform(-1, 1, size=(K, n_basis)) * phase_scale
    if n_basis > 3:
        kcoef[:, 4:] *= 1e-3
        kcoef[:, 0] *= 1e-3
    t = np.arange(K) * DWELL
    b0 = rng.uniform(-1, 1, size=L) * 2 * np.pi * b0_hz
    sens = rng.uniform(0.2, 1.0, size=(n_coil, L)) * np.exp(2j * np.pi * rng.uniform(size=(n_coil, L)))
    rho = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    m = rng.standard_normal((n_coil, K)) + 1j * rng.standard_normal((n_coil, K))
    return dict(
        L=L, K=K, n_coil=n_coil, n_basis=n_basis,
        sens=sens.astype(np.complex64), fields=fields.astype(np.float32),
        b0=b0.astype(np.float32), kcoef=kcoef.astype(np.float32), t=t.astype(np.float32),
        rho=rho.astype(np.complex64), m=m.astype(np.complex64),
    )


def dft_problem(n: int, n_coil: int = 1, full: bool = True, exact: bool = False):
    """Cartesian special case: b0 = 0, only the linear terms, k on the grid.

    2D n x n image at z = 0 with basis (1, x, y); k samples on the Cartesian
    grid k_m = pi * (m - n/2) per normalised unit, so that
    k_m * x_j = 2*pi*(m - n/2)*(j - n/2)/n.  With ``full`` every grid point is
    sampled once (row-major in (ky, kx)); otherwise every other ky row.
    Sensitivities are 1.  With ``exact`` the arrays stay float64 (pi is
    not representable in float32, which would perturb the grid by ~1e-7).
    """
    x, y, z = grid_coords((n, n), z_slice=0.0)
    fields = solid_harmonics(x, y, z, 3)
    m_idx = np.arange(n)
    ky, kx = np.meshgrid(m_idx, m_idx, indexing="ij")
    if not full:
        ky, kx = ky[::2], kx[::2]
    kx = np.pi * (kx.ravel() - n / 2)
    ky = np.pi * (ky.ravel() - n / 2)
    kcoef = np.stack([np.zeros_like(kx), kx, ky], axis=1)
    K = kcoef.shape[0]
    fr, cx = (np.float64, np.complex128) if exact else (np.float32, np.complex64)
    return dict(
        L=n * n, K=K, n_coil=n_coil, n_basis=3,
        sens=np.ones((n_coil, n * n), dtype=cx),
        fields=fields.astype(fr), b0=np.zeros(n * n, dtype=fr),
        kcoef=kcoef.astype(fr), t=(np.arange(K) * DWELL).astype(fr),
    )


def batched_slices(n_slices: int = 24, seed: int = 0, n_range=(96, 160), g_range=(8, 32),
                   k_range=(8000, 30000)):
    """Batched workload: uneven 2D slices (by default 96..160 square, 8..32
    coils, 8000..30000 samples, 16 basis terms, per-slice B0).  Returns a list
    of dicts shaped like ``make_config`` output."""
    ss = np.random.SeedSequence([_SEED_BASE + 4, seed])
    rng_sizes = np.random.default_rng(ss.spawn(1)[0])
    out = []
    for s in range(n_slices):
        n = int(rng_sizes.integers(n_range[0], n_range[1] + 1)) // 2 * 2
        G = int(rng_sizes.integers(g_range[0], g_range[1] + 1))
        Ks = int(rng_sizes.integers(k_range[0], k_range[1] + 1))
        cfg = dict(index=100 + s, dims=(n, n), n_coil=G, n_basis=16, shots=1,
                   interleaves=4, k_shot=Ks, b0_hz=100.0, b0_kind="smooth_noise", n_iter=30)
        rs = _streams(cfg["index"] + 1000 * seed)
        x, y, z = grid_coords(cfg["dims"])
        kcoef, t = _trajectory(cfg, rs[0])
        out.append(dict(
            name=f"slice{s}", dims=cfg["dims"], L=x.size, K=t.size, n_coil=G, n_basis=16,
            n_iter=30,
            sens=_sensitivities(G, rs[2], x, y, z, False).astype(np.complex64),
            fields=solid_harmonics(x, y, z, 16).astype(np.float32),
            b0=_b0_map(cfg, rs[1], x, y, z).astype(np.float32),
            kcoef=kcoef.astype(np.float32), t=t.astype(np.float32),
            rho_true=_phantom(rs[3], x, y, z, False).astype(np.complex64),
            noise=unit_noise(rs[4], (G, t.size)),
        ))
    return out


def _head_phantom(x, y, z, three_d):
    """Piecewise-constant head for the prescan: a low-intensity scalp shell
    (0.12) around a brain (0.8) holding two low-intensity ventricles (0.25).
    In 3D the head is an elongated ellipsoid cut by the slab, so every slice
    holds tissue as in an axial slab through the brain."""
    zz = (z / 2.5) ** 2 if three_d else 0.0
    head = (x / 0.84) ** 2 + (y / 0.92) ** 2 + zz <= 1.0
    brain = (x / 0.70) ** 2 + (y / 0.78) ** 2 + zz <= 1.0
    vent = np.zeros_like(head)
    for cx in (-0.17, 0.17):
        vent |= ((x - cx) / 0.09) ** 2 + ((y + 0.05) / 0.26) ** 2 + (z / 1.2 if three_d else 0.0) ** 2 <= 1.0
    rho = np.where(head, 0.12, 0.0)
    rho = np.where(brain, 0.8 + 0.1 * np.cos(6.0 * x) * np.cos(5.0 * y), rho)
    return np.where(brain & vent, 0.25, rho)


def prescan(dims=(64, 64), n_coil=8, n_echo=6, delta_te=2.3e-3, b0_hz=100.0, beta=0.2, snr=40.0, seed=0):
    """Multi-echo prescan images for the map-estimation step (Methods,
    "Computation of sensitivity maps" and "... of B0 maps"): per coil and
    echo n, S_c(r) rho(r) exp(i (omega(r) n dTE + beta mod(n, 2))) plus
    complex Gaussian noise (per-component sigma = max|rho S| / (snr sqrt 2)),
    on the head phantom above.  Also the two masks the estimation takes as
    inputs (their segmentation is outside this work): M_R = the head
    dilated by 2 voxels, M_T = brain tissue of intensity above 0.5 (the
    scalp and the ventricles are left to the extrapolation).
    Returns imgs [G][n_echo][L] complex64, S_true [G][L], omega_true [L]
    (rad/s), beta, mask_T / mask_R [L] float32, rho [L], dims, delta_te."""
    from scipy.ndimage import binary_dilation

    ss = np.random.default_rng(np.random.SeedSequence([_SEED_BASE + 7, seed]))
    rs = [np.random.default_rng(s) for s in ss.bit_generator.seed_seq.spawn(5)]
    x, y, z = grid_coords(dims)
    three_d = len(dims) == 3
    S = _sensitivities(n_coil, rs[0], x, y, z, three_d)
    cfg = dict(dims=dims, b0_kind="bump" if not three_d else "gaussians", b0_hz=b0_hz)
    omega = _b0_map(cfg, rs[1], x, y, z)
    rho = _head_phantom(x, y, z, three_d)
    shape = tuple(reversed(dims))
    mask_R = binary_dilation((rho > 0).reshape(shape), iterations=2).ravel().astype(np.float32)
    mask_T = (rho > 0.5).astype(np.float32)
    sigma = np.abs(S * rho[None, :]).max() / (snr * np.sqrt(2.0))
    imgs = np.empty((n_coil, n_echo, x.size), dtype=np.complex64)
    for n in range(n_echo):
        ph = np.exp(1j * (omega * n * delta_te + beta * (n % 2)))
        imgs[:, n, :] = S * (rho * ph)[None, :] + sigma * unit_noise(rs[3], (n_coil, x.size))
    return dict(imgs=imgs, S_true=S.astype(np.complex64), omega_true=omega, beta=beta, mask_T=mask_T,
                mask_R=mask_R, rho=rho, dims=tuple(dims), delta_te=delta_te, n_coil=n_coil, n_echo=n_echo)
