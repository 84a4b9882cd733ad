"""Scalar triple-loop forms of E and E^H (pure Python, tiny sizes only).

TEST INFRASTRUCTURE ONLY.  These evaluate the discretised signal model entry
by entry, m[c, k] = sum_l S_c(r_l) exp(i phi(k, l)) rho(r_l) with
phi(k, l) = sum_p k_p(t_k) h_p(r_l) + t_k B0(r_l), and its conjugate
transpose, with no matrices at all.  They pin the vectorised oracle.
"""
import cmath


def _phi(kcoef, t, fields, b0, k, l):
    s = 0.0
    for p in range(len(fields)):
        s += float(kcoef[k][p]) * float(fields[p][l])
    return s + float(t[k]) * float(b0[l])


def E_brute(rho, sens, fields, b0, kcoef, t):
    G = len(sens)
    K = len(t)
    L = len(b0)
    out = [[0j] * K for _ in range(G)]
    for c in range(G):
        for k in range(K):
            acc = 0j
            for l in range(L):
                acc += complex(sens[c][l]) * cmath.exp(1j * _phi(kcoef, t, fields, b0, k, l)) * complex(rho[l])
            out[c][k] = acc
    return out


def EH_brute(m, sens, fields, b0, kcoef, t):
    G = len(sens)
    K = len(t)
    L = len(b0)
    out = [0j] * L
    for l in range(L):
        acc = 0j
        for c in range(G):
            inner = 0j
            for k in range(K):
                inner += cmath.exp(-1j * _phi(kcoef, t, fields, b0, k, l)) * complex(m[c][k])
            acc += complex(sens[c][l]).conjugate() * inner
        out[l] = acc
    return out
