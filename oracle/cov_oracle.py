"""Plain CPU reference of the covariance step of Sec. 4.3 (numerical covariance
from mock catalogues, eq. (covariance); the Hartlap factor of eq. (Hartlap);
the Percival correction m1 of eqs. (Perc1), (Perc)) and of the selection of
triangle configurations by eta and r_min (Sec. 4.3, Sec. 5).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's
CPU-baseline leg, never by the product path. It shares no code with the GPU
library. Everything is float64 with explicit loops in the order of the
definitions (numpy only holds the arrays), except the matrix inverse, which
is numpy's.
"""
from __future__ import annotations

import numpy as np


def covariance(data):
    """Mean and unbiased covariance of the rows of data (n_mocks x n_d), eq. (covariance):
    C_ij = 1/(N_m - 1) sum_k (d_i^k - dbar_i)(d_j^k - dbar_j)."""
    d = np.asarray(data, dtype=np.float64)
    nm, nd = d.shape
    mean = np.zeros(nd)
    for i in range(nd):
        s = 0.0
        for k in range(nm):
            s += d[k, i]
        mean[i] = s / nm
    cov = np.zeros((nd, nd))
    for i in range(nd):
        for j in range(i, nd):
            s = 0.0
            for k in range(nm):
                s += (d[k, i] - mean[i]) * (d[k, j] - mean[j])
            cov[i, j] = cov[j, i] = s / (nm - 1)
    return mean, cov


def hartlap_factor(n_mocks, n_d):
    """(N_m - N_d - 2) / (N_m - 1), eq. (Hartlap)."""
    return (n_mocks - n_d - 2.0) / (n_mocks - 1.0)


def precision_matrix(cov, n_mocks):
    """Hartlap-corrected inverse covariance, eq. (Hartlap)."""
    return hartlap_factor(n_mocks, cov.shape[0]) * np.linalg.inv(cov)


def percival_m1(n_mocks, n_d, n_params):
    """m1 = (1 + B (N_d - N_p)) / (1 + A + B (N_p + 1)) with
    A = 2 / ((N_m - N_d - 1)(N_m - N_d - 4)), B = (N_m - N_d - 2) / ((N_m - N_d - 1)(N_m - N_d - 4)),
    eqs. (Perc1), (Perc)."""
    nm, nd, npar = float(n_mocks), float(n_d), float(n_params)
    a = 2.0 / ((nm - nd - 1.0) * (nm - nd - 4.0))
    b = (nm - nd - 2.0) / ((nm - nd - 1.0) * (nm - nd - 4.0))
    return (1.0 + b * (nd - npar)) / (1.0 + a + b * (npar + 1.0))


def select_triangles(edges, eta, r_min):
    """Triangle configurations (b1, b2) of one multipole, in the order of the
    flattened (r1, r2) grid: unique configurations r1 < r2 (bin centres), side
    difference r2 - r1 >= eta * dr and shortest side r1 >= r_min (equal-width bins)."""
    edges = np.asarray(edges, dtype=np.float64)
    nb = len(edges) - 1
    dr = (edges[-1] - edges[0]) / nb
    centres = [(edges[b] + edges[b + 1]) / 2.0 for b in range(nb)]
    out = []
    for b1 in range(nb):
        for b2 in range(nb):
            r1, r2 = centres[b1], centres[b2]
            if r1 < r2 and r2 - r1 >= eta * dr - 1e-9 * dr and r1 >= r_min - 1e-9 * dr:
                out.append((b1, b2))
    return out
