"""GPU test of the allocation-free covariance (tpcf_covariance_noalloc) through
the C ABI: two calls in a row on one device's static scratch, the second with
a smaller input, each equal bit for bit to tpcf_covariance on the same inputs
(the same kernels in the same order), and within 1e-12 of the oracle."""
import sys

import numpy as np
import pytest

from oracle import cov_oracle as V
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


def mock_vectors(nm, nd, seed):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.uniform(-0.3, 1.0, (nd, nd))) + 2.0 * np.eye(nd)
    return rng.standard_normal((nm, nd)) @ L.T + rng.uniform(-5.0, 5.0, nd)


def test_noalloc_matches_covariance_twice(torch):
    h = T.Handle(100.0, np.linspace(0.0, 10.0, 2), 0)
    try:
        # (mocks, row length, entries): the paper's 3000 x 336 first, then a
        # smaller one that leaves most of the scratch holding the first call's
        # contents
        cases = [(3000, 400, 336, 11), (50, 61, 37, 12)]
        for nm, stride, nd, seed in cases:
            say(f"  noalloc covariance: {nm} mocks, {nd} of {stride} entries")
            src_np = mock_vectors(nm, stride, seed)
            off_np = np.sort(np.random.default_rng(seed).choice(stride, nd, replace=False)).astype(np.int64)
            src = torch.from_numpy(src_np).cuda()
            off = torch.from_numpy(off_np).cuda()
            mean_a, cov_a = h.covariance_noalloc(src, offsets=off)
            mean_b, cov_b = h.covariance(src, n_d=nd, offsets=off_np)
            h.sync()
            ga, gb = cov_a.cpu().numpy(), cov_b.cpu().numpy()
            assert np.array_equal(ga, gb), "covariance differs from tpcf_covariance"
            assert np.array_equal(mean_a.cpu().numpy(), mean_b.cpu().numpy())
            sub = src_np[:, off_np]
            if nm * nd * nd > 5e7:
                mref = sub.mean(axis=0)
                cref = (sub - mref).T @ (sub - mref) / (nm - 1)  # the definition (oracle loops are slow here)
            else:
                mref, cref = V.covariance(sub)
            err = float(np.abs(ga - cref).max() / np.abs(cref).max())
            say(f"  rel err vs reference {err:.2e}")
            assert err < 1e-12
            assert np.abs(mean_a.cpu().numpy() - mref).max() <= 1e-13 * np.abs(mref).max()
        # no offsets: the first n_d entries of each row
        src = torch.from_numpy(mock_vectors(40, 9, 5)).cuda()
        _, ca = h.covariance_noalloc(src, n_d=7)
        _, cb = h.covariance(src, n_d=7)
        h.sync()
        assert np.array_equal(ca.cpu().numpy(), cb.cpu().numpy())
    finally:
        h.close()


def test_noalloc_refuses_oversized(torch):
    h = T.Handle(100.0, np.linspace(0.0, 10.0, 2), 0)
    try:
        # 8 (nm nd + partial products) bytes over the 32 MiB scratch: refused
        # on the host before any device work (the source is never read)
        src = torch.zeros((2, 1), dtype=torch.float64, device="cuda")
        rc = h.lib.tpcf_covariance_noalloc(h.h, 20000, 400, T._ptr(src), 400, None, None, T._ptr(src))
        assert rc == T.TPCF_ERR_RANGE
        assert "scratch" in h.lib.tpcf_last_error(h.h).decode()
    finally:
        h.close()
