"""ctypes wrapper of the double-precision CPU oracle (``tpcf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's CPU-baseline leg, never by the product path. It shares no
code with the GPU library (paper_2408_03036_amd/csrc).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpcf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("pos", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("box", ctypes.c_double), ("nbins", ctypes.c_int), ("edges", ctypes.c_void_p),
                ("lmax", ctypes.c_int), ("subtract_self", ctypes.c_int),
                ("prim_first", ctypes.c_int64), ("prim_count", ctypes.c_int64),
                ("nthreads", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        _lib.oracle_estimate.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        _lib.oracle_estimate.restype = ctypes.c_int
        _lib.oracle_multipoles.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p]
        _lib.oracle_multipoles.restype = ctypes.c_int
        _lib.oracle_wigner3j.argtypes = [ctypes.c_int] * 6
        _lib.oracle_wigner3j.restype = ctypes.c_double
        _lib.oracle_ylm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p]
        _lib.oracle_ylm.restype = None
        _lib.oracle_legendre_bin_integral.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        _lib.oracle_legendre_bin_integral.restype = ctypes.c_double
        _lib.oracle_xi_counts.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        _lib.oracle_xi_counts.restype = ctypes.c_int
        _lib.oracle_xi_multipoles.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                              ctypes.c_void_p]
        _lib.oracle_xi_multipoles.restype = ctypes.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def wigner3j(j1, j2, j3, m1, m2, m3) -> float:
    return lib().oracle_wigner3j(j1, j2, j3, m1, m2, m3)


def ylm(lmax: int, v) -> np.ndarray:
    """Complex array [l, m] (m >= 0) of orthonormal Y_lm at direction v."""
    out = np.zeros((lmax + 1) * (lmax + 1) * 2)
    lib().oracle_ylm(lmax, float(v[0]), float(v[1]), float(v[2]), out.ctypes.data)
    out = out.reshape(lmax + 1, lmax + 1, 2)
    return out[..., 0] + 1j * out[..., 1]


def nlm_count(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def all_multipoles(lmax: int, Lmax: int):
    """Every (l1, l2, L) with l1, l2 <= lmax, |l1-l2| <= L <= min(l1+l2, Lmax)
    and l1 + l2 + L even (eq. (TripoSH))."""
    out = []
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for L in range(abs(l1 - l2), min(l1 + l2, Lmax) + 1):
                if (l1 + l2 + L) % 2 == 0:
                    out.append((l1, l2, L))
    return out


class OracleResult:
    def __init__(self, nnn, npairs, alm):
        self.nnn = nnn          # complex [m][l1][l2][b1][b2]
        self.npairs = npairs
        self.alm = alm          # complex [p][b][l][m] or None


def estimate(pos, box, edges, lmax, w=None, subtract_self=True, prim_first=0,
             prim_count=-1, want_alm=False, want_nnn=True, nthreads=0) -> OracleResult:
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    nb = edges.shape[0] - 1
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    pc = n - prim_first if prim_count < 0 else prim_count
    s1 = lmax + 1
    prm = _Params(n, pos.ctypes.data, _ptr(wv), float(box), nb, edges.ctypes.data, lmax,
                  1 if subtract_self else 0, prim_first, pc, nthreads)
    nnn = np.zeros(s1 ** 3 * nb * nb * 2) if want_nnn else None
    alm = np.zeros(pc * nb * s1 * s1 * 2) if want_alm else None
    npairs = ctypes.c_int64(0)
    rc = lib().oracle_estimate(ctypes.byref(prm), _ptr(alm), _ptr(nnn), ctypes.addressof(npairs))
    if rc != 0:
        raise ValueError("oracle_estimate rejected its arguments")
    nnn_c = None
    if nnn is not None:
        nnn = nnn.reshape(s1, s1, s1, nb, nb, 2)
        nnn_c = nnn[..., 0] + 1j * nnn[..., 1]
    alm_c = None
    if alm is not None:
        alm = alm.reshape(pc, nb, s1, s1, 2)
        alm_c = alm[..., 0] + 1j * alm[..., 1]
    return OracleResult(nnn_c, int(npairs.value), alm_c)


def multipoles(nnn, n_data, box, edges, lmax, mults, literal=False):
    """Returns (re, im) arrays [n_mult][b1][b2] of the TripoSH coefficients."""
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    nb = edges.shape[0] - 1
    s1 = lmax + 1
    flat = np.zeros((s1, s1, s1, nb, nb, 2))
    flat[..., 0] = nnn.real
    flat[..., 1] = nnn.imag
    flat = np.ascontiguousarray(flat)
    tr = np.ascontiguousarray(np.array(mults, dtype=np.int32).reshape(-1, 3))
    re = np.zeros((tr.shape[0], nb, nb))
    im = np.zeros((tr.shape[0], nb, nb))
    rc = lib().oracle_multipoles(flat.ctypes.data, int(n_data), float(box), nb, edges.ctypes.data,
                                 lmax, tr.shape[0], tr.ctypes.data, 1 if literal else 0,
                                 re.ctypes.data, im.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_multipoles rejected its arguments")
    return re, im


def run(pos, box, edges, lmax, mults, w=None, n_data=None, subtract_self=True, nthreads=0,
        literal=False):
    """Full estimator: returns (c_re, c_im, OracleResult)."""
    n_data = pos.shape[0] if n_data is None else n_data
    res = estimate(pos, box, edges, lmax, w=w, subtract_self=subtract_self, nthreads=nthreads)
    re, im = multipoles(res.nnn, n_data, box, edges, lmax, mults, literal=literal)
    return re, im, res


# ------------------------------------------------------------------ 2PCF (Sec. 4.1)


def legendre_bin_integral(l: int, a: float, b: float) -> float:
    """Integral of P_l over [a, b]."""
    return lib().oracle_legendre_bin_integral(int(l), float(a), float(b))


def xi_counts(pos, box, edges, nmu, nthreads=0) -> np.ndarray:
    """DD(r, mu): int64 [nbins][nmu] ordered-pair counts, mu = rhat . z over [-1, 1]."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    nb = edges.shape[0] - 1
    out = np.zeros((nb, nmu), dtype=np.int64)
    rc = lib().oracle_xi_counts(pos.shape[0], pos.ctypes.data, float(box), nb, edges.ctypes.data,
                                int(nmu), int(nthreads), out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_xi_counts rejected its arguments")
    return out


def xi_multipoles(counts, n_data, box, edges, ells) -> np.ndarray:
    """xi_l(r_b) of eq. (xi_meas_leg) from DD(r, mu): float64 [len(ells)][nbins]."""
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    nb, nmu = counts.shape
    el = np.ascontiguousarray(np.array(ells, dtype=np.int32).reshape(-1))
    out = np.zeros((el.shape[0], nb))
    rc = lib().oracle_xi_multipoles(counts.ctypes.data, int(n_data), float(box), nb, edges.ctypes.data,
                                    int(nmu), el.shape[0], el.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_xi_multipoles rejected its arguments")
    return out


# ------------------------------------------------------------------ edge correction (isotropic)


def edge_correct_isotropic(N, R):
    """Edge-corrected isotropic multipoles zeta_l(b1, b2) from the Legendre
    multipoles N_l of the data-minus-randoms triplet counts and R_l of the
    random triplet counts (both normalised the same way), by the published
    Slepian-Eisenstein (2015) relation N(cos t) = zeta(cos t) R(cos t), which
    with P_a P_b = sum_l (2l+1) (a b l; 0 0 0)^2 P_l reads
        N_l = sum_{l'} M_{l l'} zeta_{l'},  M_{l l'} = sum_{l''} (2l+1) (l l' l''; 0 0 0)^2 R_{l''},
    solved for each (b1, b2). N, R: [n_ell][nb][nb]; R is truncated at n_ell - 1."""
    N = np.asarray(N, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    nl, nb1, nb2 = N.shape
    out = np.zeros_like(N)
    w3 = np.zeros((nl, nl, nl))
    for l in range(nl):
        for lp in range(nl):
            for lpp in range(nl):
                w3[l, lp, lpp] = (2 * l + 1) * wigner3j(l, lp, lpp, 0, 0, 0) ** 2
    for b1 in range(nb1):
        for b2 in range(nb2):
            M = np.zeros((nl, nl))
            for l in range(nl):
                for lp in range(nl):
                    M[l, lp] = sum(w3[l, lp, lpp] * R[lpp, b1, b2] for lpp in range(nl))
            out[:, b1, b2] = np.linalg.solve(M, N[:, b1, b2])
    return out
