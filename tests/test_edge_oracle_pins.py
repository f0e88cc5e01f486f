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
