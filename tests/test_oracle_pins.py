"""Pins of the CPU oracle against things other than itself: library routines,
closed forms, brute-force triplet counting, exact invariants and statistical
nulls. No GPU needed."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y, eval_legendre
from numpy.polynomial.legendre import leggauss

from oracle import oracle as O
from paper_2408_03036_amd import catalogs as C
import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Y_lm


def _rand_dirs(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_ylm_matches_scipy():
    lmax = 16
    dirs = np.vstack([_rand_dirs(40, 1), [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0]]])
    for v in dirs:
        Y = O.ylm(lmax, v)
        th = math.acos(max(-1.0, min(1.0, v[2])))
        ph = math.atan2(v[1], v[0])
        for l in range(lmax + 1):
            for m in range(l + 1):
                ref = complex(sph_harm_y(l, m, th, ph))
                assert abs(Y[l, m] - ref) < 1e-12 * max(1.0, abs(ref)), (l, m, v)


def test_unsold_theorem():
    lmax = 16
    for v in _rand_dirs(20, 2):
        Y = O.ylm(lmax, v)
        for l in range(lmax + 1):
            s = abs(Y[l, 0]) ** 2 + 2.0 * np.sum(np.abs(Y[l, 1:l + 1]) ** 2)
            assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-12


# ------------------------------------------------------------------ 3j


def _threej_000_closed(l1, l2, L):
    """(l1 l2 L; 0 0 0) from its closed form (DLMF 34.3.5)."""
    s = l1 + l2 + L
    if s % 2:
        return 0.0
    g = s // 2
    f = math.factorial
    val = math.sqrt(f(2 * g - 2 * l1) * f(2 * g - 2 * l2) * f(2 * g - 2 * L) / f(2 * g + 1))
    val *= f(g) / (f(g - l1) * f(g - l2) * f(g - L))
    return (-1) ** g * val


def test_threej_000_closed_form():
    for l1 in range(9):
        for l2 in range(9):
            for L in range(abs(l1 - l2), l1 + l2 + 1):
                assert abs(O.wigner3j(l1, l2, L, 0, 0, 0) - _threej_000_closed(l1, l2, L)) < 1e-13


def test_threej_golden_table():
    with open(os.path.join(GOLDEN, "wigner3j_closed_forms.json")) as fh:
        table = json.load(fh)
    for row in table["values"]:
        j = row["args"]
        want = row["sign"] * math.sqrt(row["square_num"] / row["square_den"])
        assert abs(O.wigner3j(*j) - want) < 1e-14, row


def test_threej_orthogonality():
    for l1 in range(7):
        for l2 in range(7):
            for L in range(abs(l1 - l2), l1 + l2 + 1):
                s = sum(O.wigner3j(l1, l2, L, m, -m, 0) ** 2 for m in range(-min(l1, l2), min(l1, l2) + 1))
                assert abs(s - 1.0 / (2 * L + 1)) < 1e-13


def test_threej_gaunt_quadrature():
    """int Y_l1^m Y_l2^-m Y_L^0 dOmega = sqrt((2l1+1)(2l2+1)(2L+1)/4pi) (l1 l2 L;000)(l1 l2 L;m -m 0),
    integrated on a Gauss-Legendre x uniform-phi grid (exact for these band limits)."""
    x, wx = leggauss(40)
    th = np.arccos(x)
    for (l1, l2, L) in [(1, 1, 2), (2, 3, 1), (4, 4, 4), (5, 3, 2), (6, 6, 0), (7, 5, 4)]:
        for m in range(-min(l1, l2), min(l1, l2) + 1):
            ph = 0.3
            integrand = (sph_harm_y(l1, m, th, ph) * sph_harm_y(l2, -m, th, ph)
                         * sph_harm_y(L, 0, th, ph))
            val = 2 * math.pi * np.sum(wx * integrand).real  # phi integral is trivial (M=0)
            want = (math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1) / (4 * math.pi))
                    * O.wigner3j(l1, l2, L, 0, 0, 0) * O.wigner3j(l1, l2, L, m, -m, 0))
            assert abs(val - want) < 1e-12, (l1, l2, L, m)


def test_threej_matches_exact_rational():
    for args in [(3, 4, 5, 1, 2, -3), (10, 10, 4, 3, -3, 0), (10, 8, 2, 7, -7, 0), (6, 6, 12, 0, 0, 0)]:
        assert abs(O.wigner3j(*args) - brute.wigner3j_exact(*args)) < 1e-14


def test_threej_to_lmax16_matches_exact_rational():
    """The symbols (l1 l2 L; m -m 0) the multipoles use at the top of the lmax
    range (l1, l2 <= 16, L <= 32), on a seeded sample, against exact rational
    arithmetic: Racah's alternating sum must not lose digits there."""
    rng = np.random.default_rng(16)
    n = 0
    for _ in range(600):
        l1, l2 = (int(v) for v in rng.integers(0, 17, 2))
        L = int(rng.integers(abs(l1 - l2), l1 + l2 + 1))
        m = int(rng.integers(0, min(l1, l2) + 1))
        want = brute.wigner3j_exact(l1, l2, L, m, -m, 0)
        got = O.wigner3j(l1, l2, L, m, -m, 0)
        assert abs(got - want) <= 1e-14 * max(abs(want), 1e-3), (l1, l2, L, m)
        n += want != 0.0
    assert n > 200


# ------------------------------------------------------------------ estimator vs brute force


def _mixed_weights(n, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random(n) < 0.7, 1.0, -0.4) * (0.5 + rng.random(n))


@pytest.mark.parametrize("box,n,edges", [
    (10.0, 110, [0.6, 1.4, 2.2, 3.0]),        # 3 cells per side
    (7.0, 70, [0.0, 1.2, 2.4, 3.5]),         # single-cell path, first bin from 0, rmax = L/2
])
def test_oracle_matches_bruteforce_triplets(box, n, edges):
    lmax, Lmax = 3, 3
    mults = O.all_multipoles(lmax, Lmax)
    pos = C.poisson(n, box, 11)
    w = _mixed_weights(n, 12)
    re, im, _ = O.run(pos, box, edges, lmax, mults, w=w)
    ref = brute.triplet_multipoles(pos, box, edges, mults, w=w)
    scale = np.abs(ref).max()
    assert np.abs(re - ref.real).max() < 1e-11 * scale
    assert np.abs(im).max() < 1e-11 * scale
    assert np.abs(ref.imag).max() < 1e-11 * scale


def test_oracle_keeps_degenerate_triangles_when_asked():
    box, edges, lmax = 10.0, [0.6, 1.4, 2.2, 3.0], 2
    mults = O.all_multipoles(lmax, 2)
    pos = C.poisson(90, box, 5)
    re, _, _ = O.run(pos, box, edges, lmax, mults, subtract_self=False)
    ref = brute.triplet_multipoles(pos, box, edges, mults, self_pairs=True)
    assert np.abs(re - ref.real).max() < 1e-11 * np.abs(ref).max()


def test_addition_theorem_isotropic_multipoles():
    box, edges, lmax = 10.0, [0.5, 1.5, 2.5, 3.2], 6
    pos = C.poisson(150, box, 21)
    mults = [(l, l, 0) for l in range(lmax + 1)]
    re, _, _ = O.run(pos, box, edges, lmax, mults)
    ref = brute.legendre_isotropic(pos, box, edges, list(range(lmax + 1)))
    assert np.abs(re - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("kind", ["poisson", "lattice_ties"])
def test_lmax0_integer_counts(kind):
    """lmax = 0: c_000 * RRR is an integer triplet count built from plain
    neighbour counts. The dyadic lattice puts pairs exactly on bin edges and
    pins the half-open [e_b, e_b+1) convention."""
    box, edges = 12.0, [0.0, 1.0, 2.0, 3.0, 4.0]
    if kind == "poisson":
        pos = C.poisson(300, box, 31)
    else:
        pos = np.unique(C.dyadic_lattice(300, box, 4, 32), axis=0)
    n = pos.shape[0]
    re, _, res = O.run(pos, box, edges, 0, [(0, 0, 0)])
    cnt = brute.pair_counts(pos, box, edges)
    trip = cnt.T.astype(np.float64) @ cnt - np.diag(cnt.sum(axis=0))
    got = re[0] * brute.rrr(n, box, edges)
    assert np.abs(got - trip).max() < 1e-9 * trip.max()
    assert res.npairs == int(cnt.sum())


def test_negative_m_is_conjugate():
    """NNN^{-m} computed directly from Y_{l,-m} equals conj(NNN^m)."""
    box, edges, lmax = 10.0, [0.6, 1.8, 3.0], 3
    pos = C.poisson(80, box, 41)
    w = _mixed_weights(80, 42)
    res = O.estimate(pos, box, edges, lmax, w=w)
    nb = len(edges) - 1
    for m in range(1, lmax + 1):
        direct = np.zeros((lmax + 1, lmax + 1, nb, nb), dtype=complex)
        for p in range(80):
            idx, bins, u = brute.neighbours(pos, box, edges, p)
            th = np.arccos(np.clip(u[:, 2], -1, 1))
            ph = np.arctan2(u[:, 1], u[:, 0])
            for l1 in range(m, lmax + 1):
                y1 = np.conj(sph_harm_y(l1, -m, th, ph)) * w[idx]
                for l2 in range(m, lmax + 1):
                    y2 = np.conj(sph_harm_y(l2, -m, th, ph)) * w[idx]
                    a1 = np.array([y1[bins == b].sum() for b in range(nb)])
                    a2 = np.array([y2[bins == b].sum() for b in range(nb)])
                    self_t = np.array([(y1[bins == b] * np.conj(y2[bins == b])).sum() for b in range(nb)])
                    direct[l1, l2] += w[p] * (np.outer(a1, np.conj(a2)) - np.diag(self_t))
        for l1 in range(m, lmax + 1):
            for l2 in range(m, lmax + 1):
                ref = np.conj(res.nnn[m, l1, l2])
                assert np.abs(direct[l1, l2] - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


def test_literal_normalisation_relation():
    box, edges, lmax = 10.0, [0.6, 1.8, 3.0], 3
    pos = C.poisson(120, box, 51)
    mults = O.all_multipoles(lmax, 2)
    res = O.estimate(pos, box, edges, lmax)
    c, _ = O.multipoles(res.nnn, 120, box, edges, lmax, mults)
    lit, _ = O.multipoles(res.nnn, 120, box, edges, lmax, mults, literal=True)
    for t, (l1, l2, L) in enumerate(mults):
        f = 4 * math.pi / math.sqrt((2 * l1 + 1) * (2 * l2 + 1))
        assert np.abs(lit[t] - f * c[t]).max() < 1e-12 * max(1.0, np.abs(lit[t]).max())


# ------------------------------------------------------------------ invariants


def _mult_index(mults):
    return {m: i for i, m in enumerate(mults)}


def test_swap_symmetry_and_real():
    box, edges, lmax = 20.0, [1.0, 2.0, 3.0, 4.0, 5.0], 5
    pos = C.zeldovich(1500, box, 0.5, 0.8, 61, grid=32)
    mults = O.all_multipoles(lmax, 4)
    re, im, _ = O.run(pos, box, edges, lmax, mults)
    scale = np.abs(re).max()
    assert np.abs(im).max() < 1e-12 * scale
    idx = _mult_index(mults)
    for (l1, l2, L), t in idx.items():
        assert np.abs(re[t] - re[idx[(l2, l1, L)]].T).max() < 1e-12 * scale


def test_lattice_symmetries():
    box = 16.0
    edges = [0.5, 1.5, 2.5, 3.5, 4.5]
    lmax = 4
    pos = C.dyadic_lattice(700, box, 6, 71)
    mults = O.all_multipoles(lmax, 4)
    base, _, _ = O.run(pos, box, edges, lmax, mults)
    scale = np.abs(base).max()

    def wrapped(p):
        p = np.mod(p, box)
        p[p >= box] -= box
        return p

    rot = wrapped(np.stack([-pos[:, 1], pos[:, 0], pos[:, 2]], axis=1))
    refl_x = wrapped(np.stack([-pos[:, 0], pos[:, 1], pos[:, 2]], axis=1))
    refl_z = wrapped(np.stack([pos[:, 0], pos[:, 1], -pos[:, 2]], axis=1))
    shift = wrapped(pos + np.array([3.25, -5.5, 7.125]))
    for p2, sign_by_L in [(rot, False), (refl_x, False), (shift, False), (refl_z, True)]:
        got, _, _ = O.run(p2, box, edges, lmax, mults)
        for t, (_, _, L) in enumerate(mults):
            s = (-1) ** L if sign_by_L else 1
            assert np.abs(got[t] - s * base[t]).max() < 1e-12 * scale


# ------------------------------------------------------------------ statistical nulls


def test_poisson_null():
    """Poisson catalogues: E[c_000] = 1 (the RRR normalisation) and every other
    multipole vanishes in expectation."""
    box, edges, lmax = 200.0, np.linspace(10.0, 40.0, 4), 2
    mults = O.all_multipoles(lmax, 2)
    vals = []
    for s in range(24):
        re, _, _ = O.run(C.poisson(2000, box, 1000 + s), box, edges, lmax, mults)
        vals.append(re)
    v = np.array(vals)
    mean = v.mean(0)
    sd = v.std(0, ddof=1) / math.sqrt(v.shape[0])
    expect = np.zeros_like(mean)
    expect[mults.index((0, 0, 0))] = 1.0
    z = np.abs(mean - expect) / np.maximum(sd, 1e-300)
    assert np.all(z < 5.0), float(z.max())


# ------------------------------------------------------------------ stored references


def test_c5_reference_catalogue_reproducible():
    """The stored oracle multipoles of the large data + 5x randoms catalogue
    (tests/golden/make_c5_reference.py) belong to the catalogue the seeded
    numpy generator gives now: same SHA-256 of the positions, one multipole
    row per stored triple, finite values."""
    import importlib.util
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_c5_reference", os.path.join(golden, "make_c5_reference.py"))
    G = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(G)
    ref = np.load(os.path.join(golden, "c5_catalogue_reference.npz"))
    pos, w, nd = G.catalogue()
    assert pos.shape == (6 * nd, 3) and w.shape == (6 * nd,)
    assert G.digest(pos) == str(ref["pos_sha256"])
    nb = len(G.EDGES) - 1
    assert ref["multipoles"].shape == (len(ref["mults"]), nb, nb)
    assert np.isfinite(ref["multipoles"]).all()
    assert [tuple(t) for t in ref["mults"].tolist()] == [tuple(t) for t in O.all_multipoles(G.LMAX, G.LMAX_L)]
