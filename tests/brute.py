"""Brute-force O(N^3) triplet projection, used only to pin the oracle.

For every primary p and every ordered pair of distinct neighbours (j, k) it
evaluates the tripolar basis of eq. (TSHbasis) directly,

  S_{l1 l2 L}(r1, r2, n) = (1/H) sum_{m1 m2 M} (l1 l2 L; m1 m2 M)
                            y_l1^m1(r1) y_l2^m2(r2) y_L^M(n),

with Schmidt semi-normalised y_l^m = sqrt(4 pi / (2l+1)) Y_l^m taken from
scipy, n = z (the fixed line of sight), and projects the triplet counts:

  c_{l1 l2 L}(b1, b2) = H^2 (2l1+1)(2l2+1)(2L+1)
                        sum w_p w_j w_k conj(S) / RRR(b1, b2).

The Wigner symbols come from Racah's formula evaluated in exact rational
arithmetic (fractions), pinned separately in test_oracle_pins.py.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np
from scipy.special import eval_legendre, sph_harm_y


@lru_cache(maxsize=None)
def _fact(n: int) -> int:
    return math.factorial(n)


@lru_cache(maxsize=None)
def wigner3j_exact(j1, j2, j3, m1, m2, m3):
    """(j1 j2 j3; m1 m2 m3) as a float, computed as sign * sqrt(Fraction) * Fraction."""
    if m1 + m2 + m3 != 0 or j3 > j1 + j2 or j3 < abs(j1 - j2):
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    tri = Fraction(_fact(j1 + j2 - j3) * _fact(j1 - j2 + j3) * _fact(-j1 + j2 + j3),
                   _fact(j1 + j2 + j3 + 1))
    sq = tri * _fact(j1 + m1) * _fact(j1 - m1) * _fact(j2 + m2) * _fact(j2 - m2) \
        * _fact(j3 + m3) * _fact(j3 - m3)
    s = Fraction(0)
    for k in range(0, j1 + j2 + j3 + 2):
        args = (k, j3 - j2 + k + m1, j3 - j1 + k - m2, j1 + j2 - j3 - k, j1 - k - m1, j2 - k + m2)
        if min(args) < 0:
            continue
        den = 1
        for a in args:
            den *= _fact(a)
        s += Fraction((-1) ** k, den)
    sign = -1.0 if (j1 - j2 - m3) % 2 else 1.0
    return sign * math.sqrt(sq) * float(s)


def _ylm(l, m, v):
    """Orthonormal Y_l^m (any m) at unit vectors v (n, 3), Condon-Shortley phase (scipy)."""
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi = np.arctan2(v[:, 1], v[:, 0])
    return sph_harm_y(l, m, theta, phi)


def _schmidt(l, m, v):
    return math.sqrt(4.0 * math.pi / (2 * l + 1)) * _ylm(l, m, v)


def neighbours(pos, box, edges, p):
    """Indices, bins and unit vectors of the in-shell neighbours of p
    (half-open bins by squared separation, minimum image, r = 0 dropped)."""
    d = pos - pos[p]
    d = d - box * np.round(d / box)
    r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    e2 = np.asarray(edges, dtype=np.float64) ** 2
    b = np.searchsorted(e2, r2, side="right") - 1
    ok = (r2 > 0) & (b >= 0) & (b < len(edges) - 1)
    ok[p] = False
    idx = np.nonzero(ok)[0]
    r = np.sqrt(r2[idx])
    return idx, b[idx], d[idx] / r[:, None]


def rrr(n_data, box, edges):
    e = np.asarray(edges, dtype=np.float64)
    V = 4.0 * math.pi / 3.0 * (e[1:] ** 3 - e[:-1] ** 3)
    return n_data * (n_data - 1.0) * (n_data - 2.0) * np.outer(V, V) / box ** 6


def triplet_multipoles(pos, box, edges, mults, w=None, n_data=None, self_pairs=False):
    """Direct projection of distinct ordered triplets onto S_{l1 l2 L}(., ., z).
    Returns complex [n_mult][b1][b2]."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    n_data = n if n_data is None else n_data
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    nb = len(edges) - 1
    zhat = np.array([[0.0, 0.0, 1.0]])
    out = np.zeros((len(mults), nb, nb), dtype=np.complex128)
    for p in range(n):
        idx, bins, u = neighbours(pos, box, edges, p)
        if idx.size == 0:
            continue
        onehot = np.zeros((idx.size, nb))
        onehot[np.arange(idx.size), bins] = w[idx]
        for t, (l1, l2, L) in enumerate(mults):
            H = wigner3j_exact(l1, l2, L, 0, 0, 0)
            A = np.stack([_schmidt(l1, m1, u) for m1 in range(-l1, l1 + 1)])  # (2l1+1, n)
            B = np.stack([_schmidt(l2, m2, u) for m2 in range(-l2, l2 + 1)])
            yz = np.array([_schmidt(L, M, zhat)[0] for M in range(-L, L + 1)])
            C = np.zeros((2 * l1 + 1, 2 * l2 + 1), dtype=np.complex128)
            for i1, m1 in enumerate(range(-l1, l1 + 1)):
                for i2, m2 in enumerate(range(-l2, l2 + 1)):
                    M = -m1 - m2
                    if abs(M) <= L:
                        C[i1, i2] = wigner3j_exact(l1, l2, L, m1, m2, M) * yz[M + L]
            S = A.T @ C @ B / H          # S[j, k] = S(r_j, r_k, z)
            Sc = np.conj(S)
            if not self_pairs:
                np.fill_diagonal(Sc, 0.0)
            out[t] += w[p] * (onehot.T @ Sc @ onehot)
    for t, (l1, l2, L) in enumerate(mults):
        H = wigner3j_exact(l1, l2, L, 0, 0, 0)
        out[t] *= H * H * (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    return out / rrr(n_data, box, edges)[None]


def legendre_isotropic(pos, box, edges, ells, w=None, n_data=None):
    """Y-free route (addition theorem): (2l+1) sum w w w P_l(rhat_pj . rhat_pk) / RRR
    over distinct ordered triplets. Returns [n_ell][b1][b2]."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    n_data = n if n_data is None else n_data
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    nb = len(edges) - 1
    out = np.zeros((len(ells), nb, nb))
    for p in range(n):
        idx, bins, u = neighbours(pos, box, edges, p)
        if idx.size == 0:
            continue
        onehot = np.zeros((idx.size, nb))
        onehot[np.arange(idx.size), bins] = w[idx]
        cosg = np.clip(u @ u.T, -1.0, 1.0)
        for t, l in enumerate(ells):
            P = eval_legendre(l, cosg)
            np.fill_diagonal(P, 0.0)
            out[t] += w[p] * (onehot.T @ P @ onehot)
    for t, l in enumerate(ells):
        out[t] *= 2 * l + 1
    return out / rrr(n_data, box, edges)[None]


def pair_counts(pos, box, edges):
    """n_p(b) for every point: integer in-shell neighbour counts [n][nb]."""
    n = pos.shape[0]
    nb = len(edges) - 1
    out = np.zeros((n, nb), dtype=np.int64)
    for p in range(n):
        _, bins, _ = neighbours(pos, box, edges, p)
        out[p] = np.bincount(bins, minlength=nb)
    return out
