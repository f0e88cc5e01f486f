"""Pins of the 2PCF part of the CPU oracle (Sec. 4.1: DD(r, mu), the natural
estimator of eq. (xi_natest) with analytic periodic RR, and the Legendre
multipoles of eq. (xi_meas_leg)) against things other than itself: an O(N^2)
loop over all pairs, exact counts on an integer lattice, library quadrature,
closed forms of the multipole sums, exact symmetries and a statistical null.
No GPU needed."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import eval_legendre

from oracle import oracle as O
from paper_2408_03036_amd import catalogs as C


def mu_bin(dz, r2, nmu):
    """mu bin of one separation, every step rounded in double (Python floats)."""
    r = math.sqrt(r2)
    t = (dz / r + 1.0) * (nmu / 2.0)
    return min(max(int(math.floor(t)), 0), nmu - 1)


def brute_counts(pos, box, edges, nmu):
    """Every ordered pair (p, j != p) with numpy, no cell list."""
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    e2 = np.asarray(edges, dtype=np.float64) ** 2
    nb = len(edges) - 1
    out = np.zeros((nb, nmu), dtype=np.int64)
    for p in range(pos.shape[0]):
        d = pos - pos[p]
        d -= box * np.rint(d / box)
        r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        keep = (r2 > 0.0) & (r2 >= e2[0]) & (r2 < e2[-1])
        keep[p] = False
        r2k, dzk = r2[keep], d[keep, 2]
        b = np.searchsorted(e2, r2k, side="right") - 1
        t = (dzk / np.sqrt(r2k) + 1.0) * (nmu / 2.0)
        k = np.clip(np.floor(t).astype(np.int64), 0, nmu - 1)
        np.add.at(out, (b, k), 1)
    return out


@pytest.mark.parametrize("kind", ["poisson", "zeldovich"])
@pytest.mark.parametrize("nmu", [1, 7, 20, 200])
def test_counts_match_all_pairs_loop(kind, nmu):
    box = 100.0
    if kind == "poisson":
        pos = C.poisson(500, box, C.catalogue_seed(40))
        edges = np.array([0.0, 3.0, 7.5, 12.0, 20.0, 31.0])
    else:
        pos = C.zeldovich(600, box, 3.0, 0.8, C.catalogue_seed(41), grid=32)
        edges = np.linspace(0.0, 50.0, 11)  # r_max = L/2: one-cell oracle grid
    got = O.xi_counts(pos, box, edges, nmu)
    ref = brute_counts(pos, box, edges, nmu)
    assert np.array_equal(got, ref)


def test_counts_integer_lattice_exact():
    """Simple cubic lattice of unit spacing in a periodic box of 20: every point
    sees the same offsets v in Z^3, so DD(b, k) = N #{v : |v| in bin b, mu(v)
    in bin k}. Edges at integer radii and mu bins of 0.2 put many separations
    exactly on bin edges (3-4-5 triangles, mu = 0, +-0.6, +-0.8, +-1)."""
    n1, box, nmu = 20, 20.0, 10
    g = np.arange(n1, dtype=np.float64)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    edges = np.array([0.0, 1.0, 2.0, 3.0, 5.0, 7.0, 10.0])
    e2 = edges ** 2
    per_point = np.zeros((len(edges) - 1, nmu), dtype=np.int64)
    h = n1 // 2
    for vx in range(-h + 1, h):
        for vy in range(-h + 1, h):
            for vz in range(-h + 1, h):
                r2 = vx * vx + vy * vy + vz * vz
                if r2 == 0 or r2 < e2[0] or r2 >= e2[-1]:
                    continue
                b = int(np.searchsorted(e2, r2, side="right") - 1)
                per_point[b, mu_bin(float(vz), float(r2), nmu)] += 1
    got = O.xi_counts(pos, box, edges, nmu)
    assert np.array_equal(got, per_point * pos.shape[0])
    # the mu = 0 offsets sit on the edge between bins 4 and 5 and go up
    assert per_point[:, 4].sum() != per_point[:, 5].sum()


def test_total_matches_3pcf_pair_count():
    box = 150.0
    pos = C.zeldovich(1500, box, 4.0, 0.8, C.catalogue_seed(42), grid=32)
    edges = np.linspace(5.0, 35.0, 7)
    tot = int(O.xi_counts(pos, box, edges, 13).sum())
    assert tot == O.estimate(pos, box, edges, 0, want_nnn=False).npairs


def test_legendre_bin_integral_matches_quadrature():
    rng = np.random.default_rng(5)
    for l in range(0, 13):
        for _ in range(6):
            a, b = np.sort(rng.uniform(-1.0, 1.0, 2))
            ref = quad(lambda x: eval_legendre(l, x), a, b, epsabs=1e-15, epsrel=1e-12, limit=200)[0]
            assert abs(O.legendre_bin_integral(l, a, b) - ref) < 1e-13, (l, a, b)


@pytest.mark.parametrize("nmu", [1, 3, 200])
def test_legendre_bin_integrals_partition_sum(nmu):
    """Over a partition of [-1, 1] the bin integrals add up to 2 delta_{l0}."""
    mu = -1.0 + 2.0 * np.arange(nmu + 1) / nmu
    for l in range(0, 11):
        s = sum(O.legendre_bin_integral(l, mu[k], mu[k + 1]) for k in range(nmu))
        assert abs(s - (2.0 if l == 0 else 0.0)) < 1e-13, (l, s)


def test_monopole_is_isotropic_natural_estimator():
    """xi_0(r_b) = DD_b / RR_b - 1 with DD_b the pairs in shell b and
    RR_b = N (N-1) (4 pi / 3)(e_{b+1}^3 - e_b^3) / L^3."""
    box, n = 150.0, 1500
    pos = C.zeldovich(n, box, 4.0, 0.8, C.catalogue_seed(43), grid=32)
    edges = np.linspace(0.0, 40.0, 9)
    dd = O.xi_counts(pos, box, edges, 50)
    x0 = O.xi_multipoles(dd, n, box, edges, [0])[0]
    vol = 4.0 * math.pi / 3.0 * (edges[1:] ** 3 - edges[:-1] ** 3)
    ref = dd.sum(axis=1) / (n * (n - 1) * vol / box ** 3) - 1.0
    assert np.allclose(x0, ref, rtol=0, atol=1e-13)


def test_single_mu_bin_table():
    """A table with pairs in one mu bin only: xi_l(r_b) = (2l+1)/2 D / RR_bk
    times the integral of P_l over that bin, minus delta_{l0} (odd l included,
    so a reversed mu axis would show)."""
    box, n, nmu = 100.0, 1000, 40
    edges = np.array([10.0, 20.0, 30.0])
    k0, D = 31, 12345
    dd = np.zeros((2, nmu), dtype=np.int64)
    dd[1, k0] = D
    ells = [0, 1, 2, 3, 4]
    got = O.xi_multipoles(dd, n, box, edges, ells)
    v1 = 4.0 * math.pi / 3.0 * (30.0 ** 3 - 20.0 ** 3)
    rr = n * (n - 1) * v1 / (nmu * box ** 3)
    lo, hi = -1.0 + 2.0 * k0 / nmu, -1.0 + 2.0 * (k0 + 1) / nmu
    for i, l in enumerate(ells):
        integ = quad(lambda x: eval_legendre(l, x), lo, hi, epsabs=1e-15)[0]
        ref = (2 * l + 1) / 2.0 * D / rr * integ - (1.0 if l == 0 else 0.0)
        assert abs(got[i, 1] - ref) < 1e-12 * max(1.0, abs(ref)), l
        assert abs(got[i, 0] - (-1.0 if l == 0 else 0.0)) < 1e-13, l


def _dyadic(pos, box):
    return np.mod(np.round(np.asarray(pos) * 1024.0) / 1024.0, box)


def test_z_reflection_reverses_mu():
    """z -> -z maps mu to -mu: the counts reverse along the mu axis (dyadic
    positions make every separation exact)."""
    box = 128.0
    pos = _dyadic(C.zeldovich(1200, box, 3.0, 0.8, C.catalogue_seed(44), grid=32), box)
    edges = np.linspace(2.0, 30.0, 8)
    a = O.xi_counts(pos, box, edges, 20)
    flip = pos.copy()
    flip[:, 2] = np.mod(box - flip[:, 2], box)
    b = O.xi_counts(flip, box, edges, 20)
    assert np.array_equal(b, a[:, ::-1])
    # the line of sight is z: exchanging x and z changes the counts of an
    # anisotropic (redshift-space) catalogue, not their shell totals
    sw = pos[:, [2, 1, 0]].copy()
    c = O.xi_counts(sw, box, edges, 20)
    assert np.array_equal(c.sum(axis=1), a.sum(axis=1))
    assert not np.array_equal(c, a)


def test_poisson_null():
    """Uniform points: E[DD(b, k)] = RR(b, k), so every xi_l averages to 0."""
    box, n, nseeds = 200.0, 2000, 32
    edges = np.linspace(0.0, 40.0, 5)
    ells = [0, 2, 4]
    vals = []
    for s in range(nseeds):
        pos = C.poisson(n, box, C.catalogue_seed(1000 + s))
        vals.append(O.xi_multipoles(O.xi_counts(pos, box, edges, 20), n, box, edges, ells))
    vals = np.array(vals)
    mean, sd = vals.mean(axis=0), vals.std(axis=0, ddof=1)
    t = np.abs(mean) / (sd / math.sqrt(nseeds))
    assert np.all(t < 4.0), t


def test_rejects_bad_arguments():
    pos = C.poisson(10, 10.0, 1)
    with pytest.raises(ValueError):
        O.xi_counts(pos, 10.0, [0.0, 6.0], 10)  # r_max > L/2
    with pytest.raises(ValueError):
        O.xi_counts(pos, 10.0, [2.0, 1.0], 10)
    with pytest.raises(ValueError):
        O.xi_counts(pos, 10.0, [0.0, 1.0], 0)
