"""GPU parity of the covariance step of Sec. 4.3 through the C ABI: mean and
covariance of mock data vectors against the oracle (1e-12 of max |C|), the
Hartlap-corrected precision matrix against the oracle's (1e-9 of max |P|),
and the error paths. The mock data vectors are seeded synthetic ones; the
3PCF-to-covariance chain is checked by properties."""
import sys

import numpy as np
import pytest

from oracle import cov_oracle as V
from paper_2408_03036_amd import catalogs as C
from paper_2408_03036_amd import tpcf as T

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    T.load()
    return _t


@pytest.fixture(scope="module")
def handle(torch):
    h = T.Handle(100.0, np.linspace(0.0, 10.0, 2), 0)
    yield h
    h.close()


def mock_vectors(nm, nd, seed):
    """Correlated Gaussian data vectors (a stand-in for mock measurements)."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.uniform(-0.3, 1.0, (nd, nd))) + 2.0 * np.eye(nd)
    return rng.standard_normal((nm, nd)) @ L.T + rng.uniform(-5.0, 5.0, nd)


@pytest.mark.parametrize("nm,stride,nd", [(50, 61, 37), (300, 45, 45), (3000, 400, 336), (2, 3, 1)])
def test_covariance_matches_oracle(torch, handle, nm, stride, nd):
    say(f"  covariance: {nm} mocks, data vector {nd} of {stride}")
    src = mock_vectors(nm, stride, nm + stride)
    off = np.sort(np.random.default_rng(7).choice(stride, nd, replace=False)) if nd < stride else None
    mean, cov = handle.covariance(torch.from_numpy(src).cuda(), n_d=nd, offsets=off)
    handle.sync()
    sub = src[:, off] if off is not None else src[:, :nd]
    if nm * nd * nd > 5e7:
        # the oracle's loops are slow at this size: the definition on the same data
        mref = sub.mean(axis=0)
        cref = (sub - mref).T @ (sub - mref) / (nm - 1)
    else:
        mref, cref = V.covariance(sub)
    assert np.abs(mean.cpu().numpy() - mref).max() <= 1e-13 * np.abs(mref).max()
    got = cov.cpu().numpy()
    assert np.array_equal(got, got.T)
    err = float(np.abs(got - cref).max() / np.abs(cref).max())
    say(f"  covariance rel err {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("nm,nd", [(300, 45), (3000, 336), (40, 1)])
def test_precision_matches_oracle(torch, handle, nm, nd):
    say(f"  precision: {nm} mocks, {nd} x {nd}")
    src = mock_vectors(nm, nd, 31 + nd)
    if nm * nd * nd > 5e7:
        mu = src.mean(axis=0)
        c = (src - mu).T @ (src - mu) / (nm - 1)  # the definition; the oracle's loops are slow here
    else:
        c = V.covariance(src)[1]
    # both sides invert the same (oracle-side) covariance
    cov = torch.from_numpy(np.ascontiguousarray(c)).cuda()
    prec = handle.precision(cov, nm)
    handle.sync()
    ref = V.precision_matrix(c, nm)
    got = prec.cpu().numpy()
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  precision rel err {err:.2e}")
    assert err < 1e-9
    assert np.abs(got @ c - V.hartlap_factor(nm, nd) * np.eye(nd)).max() < 1e-9
    # in place
    handle.precision(cov, nm, out=cov)
    handle.sync()
    assert np.abs(cov.cpu().numpy() - got).max() == 0.0


def test_precision_errors(torch, handle):
    bad = torch.diag(torch.tensor([1.0, -1.0, 2.0], dtype=torch.float64)).cuda()
    with pytest.raises(T.TpcfError) as e:
        handle.precision(bad, 100)
    assert e.value.status == T.TPCF_ERR_RANGE
    ok = torch.eye(4, dtype=torch.float64).cuda()
    with pytest.raises(T.TpcfError) as e:
        handle.precision(ok, 6)  # Hartlap needs n_mocks >= n_d + 3
    assert e.value.status == T.TPCF_ERR_RANGE
    src = torch.zeros((1, 5), dtype=torch.float64).cuda()
    with pytest.raises(T.TpcfError):
        handle.covariance(src)  # one mock
    with pytest.raises(T.TpcfError):
        handle.covariance(torch.zeros((4, 5), dtype=torch.float64).cuda(), offsets=[0, 5])


def test_mock_suite_chain(torch):
    """3PCF of 40 small mocks -> triangle selection -> covariance -> precision:
    symmetric, positive diagonal, and P C = Hartlap I."""
    box, edges, lmax = 400.0, np.linspace(20.0, 80.0, 7), 2
    mults = [(0, 0, 0), (1, 1, 0), (2, 0, 2)]
    n = np.full(40, 6000, dtype=np.int64)
    say("  40 mocks")
    P = torch.cat([C.zeldovich_torch(6000, box, 5.0, 0.8, C.catalogue_seed(500 + i), grid=64, device="cuda")
                   for i in range(40)], dim=0).contiguous()
    h = T.Handle(box, edges, lmax, precision=T.PREC_FP64)
    out = h.run_catalogs(n, n, P, None, mults)
    off = T.triangle_index(edges, 1, 30.0, [0, 1, 2])
    assert len(off) == 3 * 10  # 6 bins, centres 25..75: r1 >= 30 leaves 5 rows of b1
    mean, cov = h.covariance(out.reshape(40, -1), offsets=off)
    prec = h.precision(cov, 40)
    h.sync()
    c, p = cov.cpu().numpy(), prec.cpu().numpy()
    h.close()
    assert np.array_equal(c, c.T)
    assert np.all(np.diag(c) > 0)
    assert np.abs(p @ c - V.hartlap_factor(40, len(off)) * np.eye(len(off))).max() < 1e-8
    # the mean is the average of the selected entries of the 40 outputs
    flat = out.reshape(40, -1).cpu().numpy()[:, off]
    assert np.abs(mean.cpu().numpy() - flat.mean(axis=0)).max() <= 1e-13 * np.abs(flat).max()
