"""GPU parity through the C ABI on the paths that large inputs take:

* a catalogue split over several chunks of primaries (the workspace limit
  forces at least three), whose multipoles are compared element by element with
  the oracle at every precision, and with the same catalogue run in one chunk,
  bit for bit (every subchunk's partial sums are formed by the same kernels on
  the same lists, whatever chunk holds it);
* data-minus-randoms lists of thousands of weighted records per (primary, bin)
  (50x randoms, as in the paper, Sec. 4), which run through the
  wavefront-per-list harmonic kernel: a_lm slices of data and random primaries
  against the oracle (eq. (alm)) on a catalogue whose a_lm fit in one chunk,
  and at the paper's halo density the multipoles of every precision against
  the FP64 path.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_03036_amd import catalogs as C
from paper_2408_03036_amd import tpcf as T

pytestmark = pytest.mark.gpu

PRECS = [(T.PREC_FP64, 1e-12), (T.PREC_FP32, 1e-5), (T.PREC_MIXED_BF16X3, 1e-4), (T.PREC_MIXED_BF16X6, 1e-5)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    T.load()
    return _t


def run_steps(torch, P, box, edges, lmax, mults, prec, limit=0, W=None, n_data=None):
    """Steps 1-4 twice on one handle; returns (multipoles, pair count,
    harmonic-pass launches) of the second run. The first run settles the
    list room: a clustered catalogue can overflow the room predicted from its
    mean density, and the pass is then run again with more room, which the
    handle keeps."""
    h = T.Handle(box, edges, lmax, precision=prec, workspace_limit=limit)
    h.set_timing(True)
    for rep in range(2):
        h.build_grid(P, W, n_data)
        h.alm_accumulate()
        h.contract()
        out = h.multipoles(mults)
        h.sync()
        n = h.pair_count()
        _, launches = h.stage_times()
    h.close()
    return out.cpu().numpy(), n, int(launches[2])


# 2x10^4 clustered points in a 500 Mpc/h box (the C2 density x 16), 10 bins
# over [20, 120], lmax 10, L <= 2; subchunks of 4096 primaries, so a chunk of
# 8192 makes three chunks.
MC_BOX, MC_EDGES, MC_LMAX = 500.0, np.linspace(20.0, 120.0, 11), 10
# workspace limits (bytes) that cap a chunk at 8192 primaries: the planner
# gives half of the limit to the a_lm operand and the hit lists of a chunk
MC_LIMIT = {T.PREC_FP64: 300 << 20, T.PREC_FP32: 400 << 20, T.PREC_MIXED_BF16X3: 400 << 20,
            T.PREC_MIXED_BF16X6: 400 << 20}


@pytest.fixture(scope="module")
def multichunk_case(torch):
    pos = C.zeldovich(20_000, MC_BOX, 6.0, 0.8, C.catalogue_seed(91), grid=64)
    mults = O.all_multipoles(MC_LMAX, 2)
    say("  oracle: 2e4-point catalogue, lmax 10")
    re, im, res = O.run(pos, MC_BOX, MC_EDGES, MC_LMAX, mults)
    return pos, mults, re, res.npairs


@pytest.mark.parametrize("prec,tol", PRECS)
def test_multichunk_matches_oracle_and_single_chunk(torch, multichunk_case, prec, tol):
    pos, mults, ref, npairs = multichunk_case
    P = torch.from_numpy(pos).cuda()
    say(f"  precision {prec}: three or more chunks")
    got, n, launches = run_steps(torch, P, MC_BOX, MC_EDGES, MC_LMAX, mults, prec, limit=MC_LIMIT[prec])
    # one timed harmonic stage per chunk (the FP64 pass's two m-range launches are timed together)
    chunks = launches
    say(f"  chunks {chunks}, pairs {n} (oracle {npairs})")
    assert chunks >= 3
    assert n == npairs
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  multi-chunk rel err vs oracle {err:.3e}")
    assert err < tol
    one, n1, launches1 = run_steps(torch, P, MC_BOX, MC_EDGES, MC_LMAX, mults, prec)
    assert launches1 == 1
    assert n1 == n
    assert np.array_equal(one, got), "multi-chunk run differs from the single-chunk run"


# The explicit-randoms workload at the paper's density: 1e4 clustered points
# and 5e5 randoms (50x) in a 400 Mpc/h box (2.1e-4 and 7.8e-3 (h/Mpc)^3),
# weights 1 and -N_D/N_R, 12 bins of 10 over [30, 150], lmax 4: about 9,000
# weighted records per (primary, bin) list on average.
SS_BOX, SS_EDGES, SS_LMAX = 400.0, np.linspace(30.0, 150.0, 13), 4


@pytest.fixture(scope="module")
def long_lists_case(torch):
    nd, nr = 10_000, 500_000
    D = C.zeldovich(nd, SS_BOX, 5.0, 0.8, C.catalogue_seed(93), grid=64)
    R = C.randoms(nr, SS_BOX, C.randoms_seed(93))
    pos = np.vstack([D, R])
    w = C.dr_weights(nd, nr)
    return pos, w, nd


# The a_lm of a catalogue must be resident (one chunk) to be exported: a box
# of 250 Mpc/h with 1,372 clustered points and 68,600 randoms (50x), 6 bins
# over [20, 120] (the shells cover half the box), lmax 4: about 5,000
# weighted records per (primary, bin) list on average, 2.3e9 in all.
RL_BOX, RL_EDGES, RL_LMAX = 250.0, np.linspace(20.0, 120.0, 7), 4


def test_long_weighted_lists_alm_match_oracle(torch):
    nd, nr = 1_372, 68_600
    D = C.zeldovich(nd, RL_BOX, 5.0, 0.8, C.catalogue_seed(94), grid=64)
    R = C.randoms(nr, RL_BOX, C.randoms_seed(94))
    pos = np.vstack([D, R])
    w = C.dr_weights(nd, nr)
    P, W = torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda()
    h = T.Handle(RL_BOX, RL_EDGES, RL_LMAX, precision=T.PREC_FP32, workspace_limit=200 << 30)
    h.build_grid(P, W, nd)
    h.alm_accumulate()
    n_slice = 32
    mask = np.tril(np.ones((RL_LMAX + 1, RL_LMAX + 1), dtype=bool))
    try:
        for first in (500, 40_000):  # data primaries, random primaries
            got = h.get_alm(first, n_slice).cpu().numpy()
            h.sync()
            res = O.estimate(pos, RL_BOX, RL_EDGES, RL_LMAX, w=w, prim_first=first, prim_count=n_slice,
                             want_alm=True, want_nnn=False)
            ref = res.alm
            per_list = res.npairs / (n_slice * (len(RL_EDGES) - 1))
            err = float(np.abs(got[..., mask] - ref[..., mask]).max() / np.abs(ref[..., mask]).max())
            say(f"  primaries {first}..{first + n_slice}: {per_list:.0f} records per list, "
                f"a_lm rel err {err:.3e}")
            assert per_list >= 5000
            assert err < 1e-5
    finally:
        h.close()


def test_long_weighted_lists_multipoles_vs_fp64(torch, long_lists_case):
    pos, w, nd = long_lists_case
    P, W = torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda()
    mults = O.all_multipoles(SS_LMAX, 2)
    outs, pairs = {}, set()
    for prec in (T.PREC_FP64, T.PREC_FP32, T.PREC_MIXED_BF16X3):
        say(f"  data + 50x randoms, precision {prec}")
        h = T.Handle(SS_BOX, SS_EDGES, SS_LMAX, precision=prec, workspace_limit=200 << 30)
        h.build_grid(P, W, nd)
        h.alm_accumulate()
        h.contract()
        outs[prec] = h.multipoles(mults).cpu().numpy()
        h.sync()
        pairs.add(h.pair_count())
        h.close()
    assert len(pairs) == 1
    ref = outs[T.PREC_FP64]
    for prec in (T.PREC_FP32, T.PREC_MIXED_BF16X3):
        # with weights the split-BF16 request runs the six-product split (FP32-level)
        err = float(np.abs(outs[prec] - ref).max() / np.abs(ref).max())
        say(f"  precision {prec}: rel err vs FP64 path {err:.3e}")
        assert err < 1e-5
