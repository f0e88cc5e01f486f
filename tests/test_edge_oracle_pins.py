"""Pins of the isotropic edge correction of the oracle (the data-minus-
randoms multipoles divided by the random ones as functions of the opening
angle, solved multipole by multipole) against Gauss-Legendre quadrature of
the product of two Legendre series, and against its special cases. No GPU."""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy.special import eval_legendre

from oracle import oracle as O


def legendre_coeffs_of_product(z, r, nl):
    """Coefficients c_l (l < nl) of (sum z_a P_a)(sum r_b P_b) by quadrature:
    c_l = (2l+1)/2 int f(x) P_l(x) dx."""
    x, w = leggauss(64)
    f = sum(z[a] * eval_legendre(a, x) for a in range(len(z))) * \
        sum(r[b] * eval_legendre(b, x) for b in range(len(r)))
    return np.array([(2 * l + 1) / 2.0 * np.sum(w * f * eval_legendre(l, x)) for l in range(nl)])


def test_recovers_zeta_from_quadrature_products():
    """zeta and R with l <= 2: their product has degree <= 4, so with five
    multipoles the relation is exact and the solve returns zeta."""
    rng = np.random.default_rng(3)
    nl, nb = 5, 3
    N = np.zeros((nl, nb, nb))
    R = np.zeros((nl, nb, nb))
    Z = np.zeros((nl, nb, nb))
    for b1 in range(nb):
        for b2 in range(nb):
            z = rng.uniform(-0.5, 0.5, 3)
            r = np.array([1.0 + rng.uniform(-0.2, 0.2), rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1)])
            Z[:3, b1, b2] = z
            R[:3, b1, b2] = r
            N[:, b1, b2] = legendre_coeffs_of_product(z, r, nl)
    got = O.edge_correct_isotropic(N, R)
    assert np.abs(got - Z).max() < 1e-12


def test_isotropic_randoms_leave_the_ratio():
    """R = R_0 (no angular dependence): zeta_l = N_l / R_0."""
    rng = np.random.default_rng(4)
    N = rng.standard_normal((6, 4, 4))
    R = np.zeros((6, 4, 4))
    R[0] = rng.uniform(0.5, 2.0, (4, 4))
    assert np.abs(O.edge_correct_isotropic(N, R) - N / R[0]).max() < 1e-13


def test_coupling_is_symmetric_in_the_weighted_sense():
    """(2l'+1) M_{l l'} = (2l+1) M_{l' l}: the 3j squares are symmetric, which a
    transposed index would break (checked through the solve on unit vectors)."""
    rng = np.random.default_rng(5)
    nl = 5
    R = np.zeros((nl, 1, 1))
    R[:, 0, 0] = np.concatenate([[1.0], rng.uniform(-0.2, 0.2, nl - 1)])
    # columns of M^-1 from the solve, then M itself
    Minv = np.zeros((nl, nl))
    for j in range(nl):
        e = np.zeros((nl, 1, 1))
        e[j] = 1.0
        Minv[:, j] = O.edge_correct_isotropic(e, R)[:, 0, 0]
    M = np.linalg.inv(Minv)
    L = 2 * np.arange(nl) + 1.0
    assert np.abs(M * L[None, :] - (M * L[None, :]).T).max() < 1e-12


# ------------------------------------------------------------------ anisotropic


def _sph_grid(lmax):
    """Quadrature on the sphere exact for products of harmonics up to degree
    3 lmax: Gauss-Legendre nodes in cos(theta) times equally spaced phi.
    Returns Y[(l, m)] -> values at the nodes (scipy), and the weights."""
    from scipy.special import sph_harm_y
    nt, nphi = 3 * lmax // 2 + 2, 3 * lmax + 2
    x, wx = leggauss(nt)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    th = np.arccos(x)
    TH, PH = np.meshgrid(th, phi, indexing="ij")
    W = np.outer(wx, np.full(nphi, 2.0 * np.pi / nphi)).ravel()
    Y = {(l, m): sph_harm_y(l, m, TH, PH).ravel() for l in range(lmax + 1) for m in range(-l, l + 1)}
    return Y, W


def _random_real_function(rng, lmax, nb, scale, const=0.0):
    """Coefficients [m][l1][l2][b1][b2] (m >= 0) of a real function: complex
    values for m > 0 (those of m < 0 are their conjugates) and real values for
    m = 0."""
    s1 = lmax + 1
    X = np.zeros((s1, s1, s1, nb, nb), dtype=np.complex128)
    for m in range(s1):
        for l1 in range(m, s1):
            for l2 in range(m, s1):
                re = rng.uniform(-scale, scale, (nb, nb))
                im = rng.uniform(-scale, scale, (nb, nb)) if m > 0 else 0.0
                X[m, l1, l2] = re + 1j * im
    X[0, 0, 0] += const
    return X


def _evaluate(X, Y, lmax):
    """f(r1, r2) = sum X^m_{l1 l2} Y_{l1 m}(r1) conj(Y_{l2 m}(r2)) on the grid
    (all m, the m < 0 coefficients being conjugates): [b1][b2][q1][q2]."""
    nb = X.shape[3]
    q = len(next(iter(Y.values())))
    F = np.zeros((nb, nb, q, q), dtype=np.complex128)
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for m in range(-min(l1, l2), min(l1, l2) + 1):
                c = X[abs(m), l1, l2] if m >= 0 else np.conj(X[abs(m), l1, l2])
                F += c[:, :, None, None] * np.outer(Y[(l1, m)], np.conj(Y[(l2, m)]))[None, None]
    return F


def _project(F, Y, W, lmax):
    """Coefficients (m >= 0) of F by quadrature: integral of F conj(Y_l1m(r1)) Y_l2m(r2)."""
    nb = F.shape[0]
    s1 = lmax + 1
    X = np.zeros((s1, s1, s1, nb, nb), dtype=np.complex128)
    for m in range(s1):
        for l1 in range(m, s1):
            for l2 in range(m, s1):
                a = W * np.conj(Y[(l1, m)])
                b = W * Y[(l2, m)]
                X[m, l1, l2] = np.einsum("ijpq,p,q->ij", F, a, b)
    return X


@pytest.mark.parametrize("lmax", [1, 2, 3])
def test_anisotropic_recovers_zeta_from_quadrature_products(lmax):
    """zeta and R band-limited at lmax: N, the projection on l <= lmax of the
    product zeta R evaluated on a quadrature grid of both directions (scipy
    harmonics, no 3j symbols), gives back zeta through the solve."""
    rng = np.random.default_rng(11 + lmax)
    nb = 2
    Y, W = _sph_grid(lmax)
    Z = _random_real_function(rng, lmax, nb, 0.3)
    R = _random_real_function(rng, lmax, nb, 0.02, const=4.0 * np.pi)
    N = _project(_evaluate(Z, Y, lmax) * _evaluate(R, Y, lmax), Y, W, lmax)
    got = O.edge_correct_anisotropic(N, R)
    assert np.abs(got - Z).max() < 1e-11 * np.abs(Z).max()


def test_anisotropic_reduces_to_isotropic():
    """Functions of r1 . r2 only (P_l(r1 . r2) = 4 pi/(2l+1) sum_m Y_lm conj(Y_lm)):
    the anisotropic solve returns the isotropic solution on the l1 = l2 blocks
    and zero elsewhere."""
    rng = np.random.default_rng(21)
    lmax, nb = 3, 3
    nl = lmax + 1
    Niso = rng.standard_normal((nl, nb, nb))
    Riso = np.zeros((nl, nb, nb))
    Riso[0] = rng.uniform(0.8, 1.2, (nb, nb))
    Riso[1:] = rng.uniform(-0.1, 0.1, (nl - 1, nb, nb))
    ziso = O.edge_correct_isotropic(Niso, Riso)
    s1 = nl

    def to_m(X):
        out = np.zeros((s1, s1, s1, nb, nb), dtype=np.complex128)
        for l in range(nl):
            for m in range(l + 1):
                out[m, l, l] = 4.0 * np.pi / (2 * l + 1) * X[l]
        return out

    got = O.edge_correct_anisotropic(to_m(Niso), to_m(Riso))
    assert np.abs(got - to_m(ziso)).max() < 1e-12 * np.abs(to_m(ziso)).max()


def test_anisotropic_constant_randoms_leave_the_ratio():
    """R = R_0 (only the l1 = l2 = 0 term, the function R_0 / (4 pi)): zeta = 4 pi N / R_0."""
    rng = np.random.default_rng(31)
    lmax, nb = 2, 2
    N = _random_real_function(rng, lmax, nb, 1.0)
    R = np.zeros_like(N)
    R[0, 0, 0] = rng.uniform(0.5, 2.0, (nb, nb))
    got = O.edge_correct_anisotropic(N, R)
    assert np.abs(got - 4.0 * np.pi * N / R[0, 0, 0]).max() < 1e-12 * np.abs(got).max()


def test_gaunt_pins():
    """Closed forms: the integral of |Y_lm|^2 Y_00 is 1/sqrt(4 pi); the integral
    of conj(Y_10) Y_10 Y_20 is 1/sqrt(5 pi) (from Y_10 = sqrt(3/4pi) z,
    Y_20 = sqrt(5/16pi)(3z^2 - 1): 3/4pi sqrt(5/16pi) 2pi (6/5 - 2/3));
    m selection: zero unless m = m' + m''."""
    for l in range(4):
        for m in range(-l, l + 1):
            assert abs(O.gaunt_conj(l, m, l, m, 0, 0) - 1.0 / np.sqrt(4.0 * np.pi)) < 1e-14
    assert abs(O.gaunt_conj(1, 0, 1, 0, 2, 0) - 1.0 / np.sqrt(5.0 * np.pi)) < 1e-14
    assert O.gaunt_conj(2, 1, 1, 1, 1, 1) == 0.0


def test_multipoles_from_coefficients_match_oracle_multipoles():
    """The TripoSH sum applied to NNN^m / RRR equals the oracle's multipoles of
    NNN^m (which divide by RRR themselves), on a real catalogue."""
    from paper_2408_03036_amd import catalogs as C
    box, edges, lmax = 60.0, np.array([2.0, 6.0, 10.0]), 3
    pos = C.poisson(300, box, 41)
    res = O.estimate(pos, box, edges, lmax)
    mults = O.all_multipoles(lmax, 3)
    re, im = O.multipoles(res.nnn, 300, box, edges, lmax, mults)
    gre, gim = O.multipoles_from_coefficients(res.nnn / O.rrr(300, box, edges)[None, None, None], lmax, mults)
    assert np.abs(gre - re).max() < 1e-13 * np.abs(re).max()
    # the imaginary parts are rounding residues of the even-parity sums
    assert np.abs(gim - im).max() < 1e-13 * np.abs(re).max()
