"""Plain FP64 implementation of the encoding operator, its adjoint and CG.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Notation follows the paper (Methods, "Implementation of the higher-order
SENSE reconstruction", and the legend of the reconstruction-algorithm
figure):

* R, the (P+1) x L spatial basis: row 0 is B0(r_l) (here in rad/s), row p+1
  is the field basis h_p(r_l);
* K, the K x (P+1) temporal basis: column 0 is t_kappa, column p+1 is the
  dynamic field term k_p(t_kappa);
* P = exp(i K R) elementwise, so P[kappa, l] = exp(i phi(kappa, l)) with
  phi(kappa, l) = sum_p k_p(t_kappa) h_p(r_l) + t_kappa B0(r_l);
* S, the L x Gamma sensitivity matrix.  Arrays here store it coil-major as
  ``sens[Gamma][L]`` (that is S^T); coil data are stored ``m[Gamma][K]``
  (that is Sigma^T).

The signal-model equations give E p = P (S o (p 1^T)) and
E^H sigma = (S* o (P^H Sigma)) 1, evaluated without forming P^H.  Memory is
bounded by building P one block of samples at a time, as the split form of
the reconstruction figure does; block results are combined in block order.
All arithmetic is complex128 / float64.  ``numpy.exp`` and ``matmul`` are the
only library steps.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_DEF_BLOCK = 512


def _threads(n):
    return max(1, min(n, os.cpu_count() or 1))


def _spatial_basis(fields, b0):
    """R: row 0 = B0, rows 1..P = h_p (legend of the algorithm figure)."""
    fields = np.asarray(fields, dtype=np.float64)
    b0 = np.asarray(b0, dtype=np.float64)
    return np.concatenate([b0[None, :], fields], axis=0)


def _temporal_basis(kcoef, t):
    """K: column 0 = t, columns 1..P = k_p(t) (legend of the algorithm figure)."""
    kcoef = np.asarray(kcoef, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return np.concatenate([t[:, None], kcoef], axis=1)


def phase(kcoef, t, fields, b0):
    """phi = K R, the exponent of P = exp(i K R) (signal-model equation)."""
    return _temporal_basis(kcoef, t) @ _spatial_basis(fields, b0)


def _blocks(K, block):
    return [(s, min(K, s + block)) for s in range(0, K, block)]


def apply_E(rho, sens, fields, b0, kcoef, t, block=_DEF_BLOCK, threads=None):
    """E rho = P (S o (rho 1^T)), returned as m[Gamma][K] (complex128).

    Signal-model equation for E; P is built per sample block as in the split
    form of the reconstruction figure (P' = exp(i K_block R), then P' Q).
    """
    R = _spatial_basis(fields, b0)
    Kt = _temporal_basis(kcoef, t)
    Q = np.asarray(sens, dtype=np.complex128).T * np.asarray(rho, dtype=np.complex128)[:, None]
    out = np.empty((Kt.shape[0], Q.shape[1]), dtype=np.complex128)

    def work(se):
        s, e = se
        Pb = np.exp(1j * (Kt[s:e] @ R))
        out[s:e] = Pb @ Q

    blocks = _blocks(Kt.shape[0], block)
    with ThreadPoolExecutor(_threads(threads or len(blocks))) as ex:
        list(ex.map(work, blocks))
    return out.T.copy()


def apply_EH(m, sens, fields, b0, kcoef, t, block=_DEF_BLOCK, threads=None):
    """E^H sigma, returned as x[L] (complex128).

    Follows the adjoint equation and the split listing of the reconstruction
    figure: Sigma is conjugate-transposed once, the products Sigma^H_block P'
    are accumulated over sample blocks (in block order), and the result is
    weighted by S, summed over coils and conjugated ("reverse sensitivity
    weighting"), which yields sum_c conj(S_c) o (P^H sigma_c).
    """
    R = _spatial_basis(fields, b0)
    Kt = _temporal_basis(kcoef, t)
    SigH = np.conj(np.asarray(m, dtype=np.complex128))  # Gamma x K, i.e. Sigma^H
    blocks = _blocks(Kt.shape[0], block)

    def work(se):
        s, e = se
        Pb = np.exp(1j * (Kt[s:e] @ R))
        return SigH[:, s:e] @ Pb

    acc = np.zeros((SigH.shape[0], R.shape[1]), dtype=np.complex128)
    with ThreadPoolExecutor(_threads(threads or len(blocks))) as ex:
        for part in ex.map(work, blocks):
            acc += part
    S_T = np.asarray(sens, dtype=np.complex128)  # Gamma x L = S^T
    return np.conj(np.sum(acc * S_T, axis=0))


def apply_EHE(p, sens, fields, b0, kcoef, t, block=_DEF_BLOCK, threads=None):
    """E^H E p with one P' per sample block used for both products.

    Split listing of the reconstruction figure: Q = S o (p 1^T); for every
    block Q' += (P' Q)^H P'; then reverse sensitivity weighting of Q'.
    """
    R = _spatial_basis(fields, b0)
    Kt = _temporal_basis(kcoef, t)
    S_T = np.asarray(sens, dtype=np.complex128)
    Q = S_T.T * np.asarray(p, dtype=np.complex128)[:, None]  # L x Gamma
    blocks = _blocks(Kt.shape[0], block)

    def work(se):
        s, e = se
        Pb = np.exp(1j * (Kt[s:e] @ R))
        return np.conj(Pb @ Q).T @ Pb  # (P'Q)^H P', Gamma x L

    acc = np.zeros_like(S_T)
    with ThreadPoolExecutor(_threads(threads or len(blocks))) as ex:
        for part in ex.map(work, blocks):
            acc += part
    return np.conj(np.sum(acc * S_T, axis=0))


# ---------------------------------------------------------------------------
# Operand-rounding probe (not part of the method).  E^H E evaluated with the
# matrix-core operands rounded as a reduced-precision operand form rounds
# them, everything else in FP64: models how far a working precision moves
# the CG trajectory of a particular problem.  Rounding is round-to-nearest-
# even, from the IEEE formats' definitions:
#   "fp16": cos and sin rounded to float16; each data operand (S o p, the E
#           output, the coil data) scaled by a power of two that puts its
#           largest real or imaginary part just below 2^14 (the E output by
#           2^-(ceil(log2 L) + 1) relative to the E operand's scale) and
#           rounded to float16;
#   "bf16": cos and sin rounded to bfloat16 (float32 with its low 16 bits
#           rounded off); each data operand split into a bfloat16 high part
#           and the bfloat16 rounding of the remainder.

def _bf16(x):
    """Round float64 values to bfloat16 (via float32; nearest, ties to even)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _round_parts(z, fn):
    return fn(np.real(z)) + 1j * fn(np.imag(z))


def _pow2_scale(z):
    """2^(14 - e) with max(|re|, |im|) < 2^e (1 for an all-zero operand)."""
    mx = max(float(np.max(np.abs(np.real(z)), initial=0.0)), float(np.max(np.abs(np.imag(z)), initial=0.0)))
    if not mx > 0.0:
        return 1.0
    _, e = np.frexp(mx)
    return float(np.ldexp(1.0, 14 - int(e)))


def _round_exp(phi, fmt):
    c, s = np.cos(phi), np.sin(phi)
    fn = (lambda v: v.astype(np.float16).astype(np.float64)) if fmt == "fp16" else _bf16
    return fn(c) + 1j * fn(s)


def _round_data(z, fmt, scale):
    """Data operand z as the operand form holds it (z * scale rounded), unscaled."""
    if fmt == "fp16":
        return _round_parts(z * scale, lambda v: v.astype(np.float16).astype(np.float64)) / scale
    hi = _round_parts(z, _bf16)
    return hi + _round_parts(z - hi, _bf16)


def apply_EH_rounded(m, sens, fields, b0, kcoef, t, fmt, block=_DEF_BLOCK, threads=None):
    """E^H sigma with operand rounding ``fmt`` (probe; see above)."""
    R = _spatial_basis(fields, b0)
    Kt = _temporal_basis(kcoef, t)
    m = np.asarray(m, dtype=np.complex128)
    sig = _round_data(m, fmt, _pow2_scale(m))
    blocks = _blocks(Kt.shape[0], block)

    def work(se):
        s, e = se
        return np.conj(sig[:, s:e]) @ _round_exp(Kt[s:e] @ R, fmt)

    acc = np.zeros((sig.shape[0], R.shape[1]), dtype=np.complex128)
    with ThreadPoolExecutor(_threads(threads or len(blocks))) as ex:
        for part in ex.map(work, blocks):
            acc += part
    return np.conj(np.sum(acc * np.asarray(sens, dtype=np.complex128), axis=0))


def apply_EHE_rounded(p, sens, fields, b0, kcoef, t, fmt, block=_DEF_BLOCK, threads=None):
    """E^H E p with operand rounding ``fmt`` (probe; see above)."""
    R = _spatial_basis(fields, b0)
    Kt = _temporal_basis(kcoef, t)
    S_T = np.asarray(sens, dtype=np.complex128)
    L = S_T.shape[1]
    Q = S_T.T * np.asarray(p, dtype=np.complex128)[:, None]
    sq = _pow2_scale(Q)
    Q = _round_data(Q, fmt, sq)
    sy = sq * float(np.ldexp(1.0, -(int(np.ceil(np.log2(L))) + 1))) if L > 1 else sq * 0.5
    blocks = _blocks(Kt.shape[0], block)

    def work(se):
        s, e = se
        Pb = _round_exp(Kt[s:e] @ R, fmt)
        y = _round_data(Pb @ Q, fmt, sy)
        return np.conj(y).T @ Pb

    acc = np.zeros_like(S_T)
    with ThreadPoolExecutor(_threads(threads or len(blocks))) as ex:
        for part in ex.map(work, blocks):
            acc += part
    return np.conj(np.sum(acc * S_T, axis=0))


def dense_E(sens, fields, b0, kcoef, t):
    """The explicit (Gamma*K) x L encoding matrix, built column by column by
    applying E to unit vectors (tiny problems only)."""
    L = np.asarray(fields).shape[1]
    cols = []
    for l in range(L):
        e = np.zeros(L, dtype=np.complex128)
        e[l] = 1.0
        cols.append(apply_E(e, sens, fields, b0, kcoef, t).ravel())
    return np.stack(cols, axis=1)


def cg_solve(m, sens, fields, b0, kcoef, t, n_iter, icorr=None, tol=0.0,
             return_iterates=False, explicit_residual=False, block=_DEF_BLOCK, threads=None,
             perturb=None, reorth=False, operands=None):
    """CG on E^H E rho = E^H sigma, as in the reconstruction figure.

    Steps: optional intensity correction S <- S o (j 1^T); p = E^H sigma;
    r = p; rho = 0; then per iteration q = E^H E p, alpha = r^H r,
    beta = p^H q, rho += (alpha/beta) p, r -= (alpha/beta) q, beta <- alpha,
    alpha = r^H r, p = r + (alpha/beta) p; finally rho <- rho o j.  The
    k-space filter f is not part of this path.

    Readings where the figure is silent (also listed in the design notes):
    alpha and beta are taken as real parts (they are real in exact
    arithmetic); the alpha at the top of an iteration equals the alpha
    computed at the end of the previous one, so it is reused; the loop stops
    early on exact convergence (alpha = 0), on breakdown (beta <= 0 or a
    non-finite scalar) and, when tol > 0, once ||r_n|| <= tol ||r_0||.

    ``reorth``: after each residual update, r is orthogonalised against the
    normalised earlier residuals r_j / ||r_j|| (modified Gram-Schmidt).  In
    exact arithmetic the CG residuals are already mutually orthogonal, so
    this leaves the iterates of the figure unchanged; in floating point it
    keeps them on the exact-arithmetic trajectory on ill-conditioned
    problems, where plain recurrences lose orthogonality within a few tens
    of iterations.

    ``perturb = (delta, seed)`` is a sensitivity probe, not part of the
    method: every E^H E p is multiplied elementwise by (1 + delta * xi) with
    xi complex Gaussian (seeded), which models a working precision whose
    relative rounding error is about delta.  Comparing such a run with the
    unperturbed one measures how far the iterates of this particular problem
    can move under rounding at that level.  ``operands = "fp16" | "bf16"``
    is the other probe: E^H sigma and every E^H E p with the matrix-core
    operands rounded as that operand form rounds them (apply_EH_rounded,
    apply_EHE_rounded), the CG arithmetic itself in FP64.

    Returns dict(rho, iters, status, hist[iters+1][3], iterates?, dres?)
    where hist row n holds (||r_n||, ||rho_n||, ||d_n||^2 from the
    recurrence ||d_{n+1}||^2 = ||d_n||^2 - alpha^2/beta, d_n = sigma - E rho_n).
    """
    sens = np.asarray(sens, dtype=np.complex128)
    if icorr is not None:
        sens = sens * np.asarray(icorr, dtype=np.float64)[None, :]
    args = (sens, fields, b0, kcoef, t)
    kw = dict(block=block, threads=threads)
    m = np.asarray(m, dtype=np.complex128)
    p = apply_EH(m, *args, **kw) if operands is None else apply_EH_rounded(m, *args, operands, **kw)
    r = p.copy()
    rho = np.zeros_like(p)
    alpha = float(np.real(np.vdot(r, r)))
    alpha0 = alpha
    d2 = float(np.real(np.vdot(m, m)))
    hist = [(np.sqrt(alpha), 0.0, d2)]
    iterates = []
    dres = []
    status = "max_iter"
    n = 0
    prng = np.random.default_rng(perturb[1]) if perturb else None
    basis = [r / np.sqrt(alpha)] if (reorth and alpha > 0.0) else []
    if alpha == 0.0:
        status = "exact"
    else:
        while n < n_iter:
            q = apply_EHE(p, *args, **kw) if operands is None else apply_EHE_rounded(p, *args, operands, **kw)
            if prng is not None:
                xi = prng.standard_normal(q.shape) + 1j * prng.standard_normal(q.shape)
                q = q * (1.0 + perturb[0] * xi / np.sqrt(2.0))
            beta = float(np.real(np.vdot(p, q)))
            if not np.isfinite(beta) or beta <= 0.0:
                status = "breakdown"
                break
            gamma = alpha / beta
            rho = rho + gamma * p
            r = r - gamma * q
            for v in basis:
                r = r - np.vdot(v, r) * v
            d2 = d2 - alpha * alpha / beta
            beta = alpha
            alpha = float(np.real(np.vdot(r, r)))
            p = r + (alpha / beta) * p
            n += 1
            if reorth and alpha > 0.0:
                basis.append(r / np.sqrt(alpha))
            hist.append((np.sqrt(alpha), float(np.linalg.norm(rho)), d2))
            if return_iterates:
                iterates.append(rho.copy())
            if explicit_residual:
                dres.append(float(np.linalg.norm(m - apply_E(rho, *args, **kw)) ** 2))
            if not np.isfinite(alpha):
                status = "breakdown"
                break
            if alpha == 0.0:
                status = "exact"
                break
            if tol > 0.0 and np.sqrt(alpha) <= tol * np.sqrt(alpha0):
                status = "tol"
                break
    if icorr is not None:
        rho = rho * np.asarray(icorr, dtype=np.float64)
    out = dict(rho=rho, iters=n, status=status, hist=np.array(hist))
    if return_iterates:
        out["iterates"] = iterates
    if explicit_residual:
        out["dres"] = np.array(dres)
    return out


def encode_grads(rho, m, sens, fields, b0, kcoef, t, block=_DEF_BLOCK, threads=None):
    """Loss ||E rho - sigma||^2 and its gradients (derived, not printed in the paper).

    With G = 2 (E rho - sigma) (the gradient with respect to the conjugate
    output, PyTorch's convention for complex tensors):
      grad_rho        = E^H G
      dL/db0[l]       = Im(conj(rho[l]) [E^H (t o G)][l])
      dL/dkcoef[k, b] = Im(sum_c G[c, k] conj([E (h_b o rho)][c, k]))
    obtained by differentiating phi = K R with respect to B0(r_l) and
    k_b(t_kappa).  Returns (loss, grad_rho, grad_b0, grad_kcoef).
    """
    args = (sens, fields, b0, kcoef, t)
    kw = dict(block=block, threads=threads)
    rho = np.asarray(rho, dtype=np.complex128)
    y = apply_E(rho, *args, **kw)
    res = y - np.asarray(m, dtype=np.complex128)
    loss = float(np.real(np.vdot(res, res)))
    G = 2.0 * res
    grad_rho = apply_EH(G, *args, **kw)
    tG = G * np.asarray(t, dtype=np.float64)[None, :]
    grad_b0 = np.imag(np.conj(rho) * apply_EH(tG, *args, **kw))
    fields64 = np.asarray(fields, dtype=np.float64)
    P = fields64.shape[0]
    grad_k = np.empty((np.asarray(t).shape[0], P))
    for b in range(P):
        Z = apply_E(fields64[b] * rho, *args, **kw)
        grad_k[:, b] = np.imag(np.sum(G * np.conj(Z), axis=0))
    return loss, grad_rho, grad_b0, grad_k
