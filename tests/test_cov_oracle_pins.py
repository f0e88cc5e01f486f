"""Pins of the covariance part of the CPU oracle (Sec. 4.3: eq. (covariance),
the Hartlap factor of eq. (Hartlap), the Percival factor of eqs. (Perc1),
(Perc), and the eta / r_min triangle selection) against library routines,
statistics with known answers, closed-form counts and limits. No GPU needed."""
import math

import numpy as np
import pytest

from oracle import cov_oracle as V


def test_covariance_matches_numpy():
    rng = np.random.default_rng(11)
    d = rng.standard_normal((37, 9)) @ rng.standard_normal((9, 9)) + rng.standard_normal(9)
    mean, cov = V.covariance(d)
    assert np.allclose(mean, d.mean(axis=0), rtol=0, atol=1e-13)
    ref = np.cov(d, rowvar=False, ddof=1)
    assert np.abs(cov - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.array_equal(cov, cov.T)


def test_covariance_is_unbiased():
    """E[C_hat] = Sigma for Gaussian mocks (the 1/(N_m - 1) normalisation)."""
    rng = np.random.default_rng(12)
    nd, nm, trials = 3, 6, 4000
    L = np.array([[1.0, 0.0, 0.0], [0.5, 1.2, 0.0], [-0.3, 0.4, 0.8]])
    sigma = L @ L.T
    acc = np.zeros((nd, nd))
    samples = rng.standard_normal((trials, nm, nd)) @ L.T
    for t in range(trials):
        acc += V.covariance(samples[t])[1]
    acc /= trials
    # standard error of a sample-covariance entry ~ sqrt((S_ii S_jj + S_ij^2) / (N_m - 1) / trials)
    se = np.sqrt((np.outer(np.diag(sigma), np.diag(sigma)) + sigma ** 2) / (nm - 1) / trials)
    assert np.all(np.abs(acc - sigma) < 5 * se)


def test_hartlap_makes_the_precision_unbiased():
    """The inverse of a sample covariance overestimates Sigma^-1 by
    (N_m - 1) / (N_m - N_d - 2); the Hartlap factor removes that bias."""
    rng = np.random.default_rng(13)
    nd, nm, trials = 4, 16, 6000
    L = np.tril(rng.uniform(0.2, 1.0, (nd, nd))) + np.eye(nd)
    sigma_inv = np.linalg.inv(L @ L.T)
    acc = np.zeros((nd, nd))
    raw = np.zeros((nd, nd))
    samples = rng.standard_normal((trials, nm, nd)) @ L.T
    for t in range(trials):
        c = np.cov(samples[t], rowvar=False)
        acc += V.precision_matrix(c, nm)
        raw += np.linalg.inv(c)
    acc /= trials
    raw /= trials
    ratio_corr = np.trace(acc) / np.trace(sigma_inv)
    ratio_raw = np.trace(raw) / np.trace(sigma_inv)
    assert abs(ratio_corr - 1.0) < 0.02
    assert abs(ratio_raw - (nm - 1.0) / (nm - nd - 2.0)) < 0.03


def test_precision_times_covariance_is_scaled_identity():
    rng = np.random.default_rng(14)
    d = rng.standard_normal((200, 20))
    _, cov = V.covariance(d)
    p = V.precision_matrix(cov, 200)
    assert np.abs(p @ cov - V.hartlap_factor(200, 20) * np.eye(20)).max() < 1e-10


def test_percival_limits():
    # many mocks: no correction
    assert abs(V.percival_m1(10 ** 9, 300, 6) - 1.0) < 1e-6
    # fewer parameters than data: the parameter variance is inflated, the more
    # so the fewer mocks there are
    m_a, m_b = V.percival_m1(3000, 336, 6), V.percival_m1(1000, 336, 6)
    assert 1.0 < m_a < m_b
    # first order in 1/N_m (A ~ 2 / N_m^2, B ~ 1 / N_m):
    # m1 = 1 + (N_d - N_p) / N_m - (N_p + 1) / N_m + O(N_m^-2)
    nm = 10 ** 6
    assert abs((V.percival_m1(nm, 200, 5) - 1.0) * nm - (200 - 2 * 5 - 1)) < 0.1


def _golden_percival():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "percival_m1.json")) as f:
        return json.load(f)["values"]


@pytest.mark.parametrize("g", _golden_percival(), ids=lambda g: f"Nm{g['n_mocks']}_Nd{g['n_d']}_Np{g['n_params']}")
def test_percival_golden_fractions(g):
    """m1 and the Hartlap factor against exact fractions evaluated by hand from
    eqs. (Perc1), (Perc) and (Hartlap) (tests/golden/percival_m1.json). At
    N_m = 298 a changed constant in A (2 -> 3) moves m1 by 3e-5 and a changed
    "-2" in B by 4e-3 relative, far above the 4-ulp tolerance."""
    from fractions import Fraction
    nm, nd, npar = g["n_mocks"], g["n_d"], g["n_params"]
    m1 = Fraction(*g["m1"])
    assert abs(V.percival_m1(nm, nd, npar) - float(m1)) <= 4 * np.spacing(float(m1))
    hl = Fraction(*g["hartlap"])
    assert abs(V.hartlap_factor(nm, nd) - float(hl)) <= 2 * np.spacing(float(hl))
    # the fractions are consistent with each other (A, B -> m1)
    a, b = Fraction(*g["A"]), Fraction(*g["B"])
    assert (1 + b * (nd - npar)) / (1 + a + b * (npar + 1)) == m1


@pytest.mark.parametrize("nb,eta", [(12, 1), (12, 3), (12, 11), (5, 2)])
def test_triangle_counts_closed_form(nb, eta):
    """Without r_min, the pairs b1 < b2 with b2 - b1 >= eta number (nb - eta)(nb - eta + 1) / 2."""
    edges = 30.0 + 10.0 * np.arange(nb + 1)
    sel = V.select_triangles(edges, eta, 0.0)
    assert len(sel) == (nb - eta) * (nb - eta + 1) // 2
    assert sel == sorted(sel)
    assert all(b2 - b1 >= eta for b1, b2 in sel)


def test_triangle_selection_rmin():
    """Paper's variance figure: bins of 10 over [30, 150], r_min = 40, eta >= 1:
    the shortest side's bin centre must be >= 40 (centre 35 is dropped)."""
    edges = np.linspace(30.0, 150.0, 13)
    sel = V.select_triangles(edges, 1, 40.0)
    assert all(b1 >= 1 for b1, _ in sel)
    assert len(sel) == 10 * 11 // 2
    # eta = 3 over the same bins (the paper's covariance figure)
    assert len(V.select_triangles(edges, 3, 0.0)) == 45
