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
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
# ORACLE_LIBRARY selects another build (for example the sanitized one)
_LIB = os.environ.get("ORACLE_LIBRARY") or _LIB_DEFAULT
_lib = None


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FMA contraction). With
    sanitize, an AddressSanitizer + UndefinedBehaviorSanitizer build
    (liboracle_san.so), to be loaded with gcc's libasan preloaded."""
    out = _LIB_SAN if sanitize else _LIB_DEFAULT
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        san = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer"] if sanitize else []
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math"] + san + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("pos", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("box", ctypes.c_double), ("nbins", ctypes.c_int), ("edges", ctypes.c_void_p),
                ("lmax", ctypes.c_int), ("subtract_self", ctypes.c_int),
                ("prim_first", ctypes.c_int64), ("prim_count", ctypes.c_int64),
                ("nthreads", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if _LIB == _LIB_DEFAULT:
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


# ------------------------------------------------------------------ edge correction (anisotropic)


def gaunt_conj(l, m, lp, mp, lpp, mpp):
    """Integral over the sphere of conj(Y_lm) Y_l'm' Y_l''m'' (orthonormal,
    Condon-Shortley phase), from the 3j symbols: conj(Y_lm) = (-1)^m Y_l,-m and
    the integral of three harmonics is
    sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi)) (l1 l2 l3; 0 0 0) (l1 l2 l3; m1 m2 m3)."""
    if m != mp + mpp or abs(m) > l or abs(mp) > lp or abs(mpp) > lpp:
        return 0.0
    if lpp < abs(l - lp) or lpp > l + lp or (l + lp + lpp) % 2:
        return 0.0
    f = np.sqrt((2 * l + 1) * (2 * lp + 1) * (2 * lpp + 1) / (4.0 * np.pi))
    sign = -1.0 if m % 2 else 1.0
    return sign * f * wigner3j(l, lp, lpp, 0, 0, 0) * wigner3j(l, lp, lpp, -m, mp, mpp)


def edge_correct_anisotropic(N, R):
    """Edge-corrected anisotropic 3PCF coefficients from the data-minus-randoms
    triplet counts N and the random triplet counts R (Szapudi-Szalay estimator,
    eq. (ssest): zeta = (D - R)^3 / R^3 as functions of the triangle).

    N and R are complex arrays [m][l1][l2][b1][b2], m = 0..lmax, of the
    coefficients of real functions of the two sides' directions in the basis
    Y_{l1 m}(r1) conj(Y_{l2 m}(r2)) (the coefficients of m < 0 are the
    conjugates), normalised alike (for example NNN^m / RRR of each run). The
    relation N(r1, r2) = zeta(r1, r2) R(r1, r2) at every pair of directions
    reads, coefficient by coefficient,
        N^m_{l1 l2} = sum zeta^{m'}_{l1' l2'} R^{m-m'}_{l1'' l2''}
                      G(l1 m; l1' m'; l1'' m-m') G(l2 m; l2' m'; l2'' m-m'),
    G(l m; l' m'; l'' m'') = integral of conj(Y_lm) Y_l'm' Y_l''m''; every
    index is truncated at lmax. The system is solved for zeta at each
    (b1, b2); zeta is returned in the layout of N (complex, m >= 0)."""
    N = np.asarray(N, dtype=np.complex128)
    R = np.asarray(R, dtype=np.complex128)
    s1 = N.shape[0]
    nb1, nb2 = N.shape[3], N.shape[4]
    idx = [(l1, l2, m) for l1 in range(s1) for l2 in range(s1)
           for m in range(-min(l1, l2), min(l1, l2) + 1)]
    n = len(idx)
    # coupling entries (row, column, l1'', l2'', m'', weight), independent of (b1, b2)
    I, J, C1, C2, MM, W = [], [], [], [], [], []
    for i, (l1, l2, m) in enumerate(idx):
        for j, (a1, a2, mp) in enumerate(idx):
            mpp = m - mp
            for c1 in range(abs(mpp), s1):
                g1 = gaunt_conj(l1, m, a1, mp, c1, mpp)
                if g1 == 0.0:
                    continue
                for c2 in range(abs(mpp), s1):
                    g2 = gaunt_conj(l2, m, a2, mp, c2, mpp)
                    if g2 == 0.0:
                        continue
                    I.append(i)
                    J.append(j)
                    C1.append(c1)
                    C2.append(c2)
                    MM.append(mpp)
                    W.append(g1 * g2)
    I, J, C1, C2, MM, W = (np.array(v) for v in (I, J, C1, C2, MM, W))
    am = np.abs(MM)

    def value(X, l1, l2, m, b1, b2):
        v = X[np.abs(m), l1, l2, b1, b2]
        return np.where(m < 0, np.conj(v), v)

    rl1 = np.array([t[0] for t in idx])
    rl2 = np.array([t[1] for t in idx])
    rm = np.array([t[2] for t in idx])
    out = np.zeros_like(N)
    for b1 in range(nb1):
        for b2 in range(nb2):
            rv = R[am, C1, C2, b1, b2]
            rv = np.where(MM < 0, np.conj(rv), rv)
            M = np.zeros((n, n), dtype=np.complex128)
            np.add.at(M, (I, J), W * rv)
            rhs = value(N, rl1, rl2, rm, b1, b2)
            z = np.linalg.solve(M, rhs)
            for k, (l1, l2, m) in enumerate(idx):
                if m >= 0:
                    out[m, l1, l2, b1, b2] = z[k]
    return out


def multipoles_from_coefficients(Z, lmax, mults, literal=False):
    """TripoSH coefficients c_{l1 l2 L}(b1, b2) of the function whose
    orthonormal-basis coefficients are Z (complex [m][l1][l2][b1][b2], m >= 0,
    already normalised): the formula of oracle_multipoles without the
    division by RRR. Returns (re, im) [n_mult][b1][b2]."""
    Z = np.asarray(Z, dtype=np.complex128)
    nb1, nb2 = Z.shape[3], Z.shape[4]
    re = np.zeros((len(mults), nb1, nb2))
    im = np.zeros((len(mults), nb1, nb2))
    for t, (l1, l2, L) in enumerate(mults):
        H = wigner3j(l1, l2, L, 0, 0, 0)
        pref = ((2 * L + 1) * H * 16.0 * np.pi ** 2 if literal
                else 4.0 * np.pi * np.sqrt((2 * l1 + 1) * (2 * l2 + 1)) * (2 * L + 1) * H)
        s = np.zeros((nb1, nb2), dtype=np.complex128)
        for m in range(-min(l1, l2), min(l1, l2) + 1):
            v = Z[abs(m), l1, l2]
            v = np.conj(v) if m < 0 else v
            s += wigner3j(l1, l2, L, m, -m, 0) * (-1.0 if m % 2 else 1.0) * v
        re[t] = pref * s.real
        im[t] = pref * s.imag
    return re, im


def rrr(n_data, box, edges):
    """Analytic random-triplet count RRR(b1, b2) = N (N-1)(N-2) V_b1 V_b2 / L^6 (periodic box)."""
    e = np.asarray(edges, dtype=np.float64)
    V = 4.0 * np.pi / 3.0 * (e[1:] ** 3 - e[:-1] ** 3)
    nd = float(n_data)
    return nd * (nd - 1.0) * (nd - 2.0) * np.outer(V, V) / box ** 6
