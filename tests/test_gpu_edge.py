"""GPU parity of the Szapudi-Szalay estimator with explicit randoms
(isotropic multipoles, edge-corrected by the random triplet counts) through the
C ABI: the correction kernel against the oracle on synthetic multipoles, and
the whole chain (data-minus-randoms run, randoms run, correction) against the
oracle's chain on a small catalogue."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
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


@pytest.mark.parametrize("nl,nb", [(5, 4), (11, 10), (1, 3), (25, 2)])
def test_correction_matches_oracle(torch, nl, nb):
    rng = np.random.default_rng(nl * 100 + nb)
    N = rng.standard_normal((nl, nb, nb))
    R = rng.uniform(-0.05, 0.05, (nl, nb, nb))
    R[0] += 1.0
    h = T.Handle(100.0, np.linspace(1.0, 20.0, nb + 1), 0)
    got = h.edge_correct_isotropic(torch.from_numpy(N).cuda(), torch.from_numpy(R).cuda()).cpu().numpy()
    h.close()
    ref = O.edge_correct_isotropic(N, R)
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  edge correction n_ell={nl} nb={nb}: rel err {err:.2e}")
    assert err < 1e-12


def test_singular_coupling_rejected(torch):
    h = T.Handle(100.0, np.linspace(1.0, 20.0, 3), 0)
    N = torch.ones((3, 2, 2), dtype=torch.float64).cuda()
    R = torch.zeros((3, 2, 2), dtype=torch.float64).cuda()
    with pytest.raises(T.TpcfError) as e:
        h.edge_correct_isotropic(N, R)
    assert e.value.status == T.TPCF_ERR_RANGE
    h.close()


@pytest.mark.parametrize("prec,tol", [(T.PREC_FP64, 1e-10), (T.PREC_FP32, 1e-5)])
def test_explicit_randoms_chain(torch, prec, tol):
    """1,500 clustered data points and 10x randoms in a 150 Mpc/h box, 5 bins
    over [8, 48], lmax 4: N from the data-minus-randoms run, R from the randoms
    run, corrected; the oracle runs the same chain."""
    box, edges, lmax = 150.0, np.linspace(8.0, 48.0, 6), 4
    nd, nr = 1500, 15000
    D = C.zeldovich(nd, box, 4.0, 0.8, C.catalogue_seed(80), grid=32)
    Rp = C.randoms(nr, box, C.randoms_seed(80))
    pos = np.vstack([D, Rp])
    w = C.dr_weights(nd, nr)
    iso = [(l, l, 0) for l in range(lmax + 1)]
    say("  oracle: data-minus-randoms and randoms runs")
    n_or, _, _ = O.run(pos, box, edges, lmax, iso, w=w, n_data=nd)
    r_or, _, _ = O.run(Rp, box, edges, lmax, iso, n_data=nr)
    ref = O.edge_correct_isotropic(n_or, r_or)

    def run(p, wt, n_data):
        h = T.Handle(box, edges, lmax, precision=prec, flags=T.F_ISOTROPIC)
        h.build_grid(torch.from_numpy(p).cuda(), None if wt is None else torch.from_numpy(wt).cuda(), n_data)
        h.alm_accumulate()
        h.contract()
        out = h.multipoles(iso)
        h.sync()
        return h, out

    hN, Nm = run(pos, w, nd)
    hR, Rm = run(Rp, None, nr)
    got = hN.edge_correct_isotropic(Nm, Rm).cpu().numpy()
    hN.close()
    hR.close()
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  explicit-randoms chain rel err {err:.2e}")
    assert err < tol
