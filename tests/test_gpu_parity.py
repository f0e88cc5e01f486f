"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances, relative to max |zeta| over all multipoles and bins:
FP64 path 1e-12, FP32 path 1e-5, split-BF16 (3 products) 1e-4, split-BF16
(6 products) 1e-5. Pair counts and lmax = 0 integer triplet counts are exact.

The 3-product split keeps x to 2^-16 relative, and the removal of degenerate
triangles on b1 = b2 cancels sum_p |a|^2 against sum_p sum_j |Y|^2, so its
error grows like 2^-16 (2l+1) / nbar_b (nbar_b = neighbours per primary in
bin b). Its 1e-4 bound is checked on the dense configuration it is meant for;
the sparse C1 anchor (0.13 neighbours per primary in its first bin) is
checked with the 6-product split.
"""
import ctypes
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_03036_amd import catalogs as C
from paper_2408_03036_amd import tpcf as T

pytestmark = pytest.mark.gpu

TOL = {T.PREC_FP64: 1e-12, T.PREC_FP32: 1e-5, T.PREC_MIXED_BF16X3: 1e-4,
       T.PREC_MIXED_BF16X6: 1e-5}
PRECS = [T.PREC_FP64, T.PREC_FP32, T.PREC_MIXED_BF16X3, T.PREC_MIXED_BF16X6]
PNAME = {T.PREC_FP64: "fp64", T.PREC_FP32: "fp32", T.PREC_MIXED_BF16X3: "bf16x3",
         T.PREC_MIXED_BF16X6: "bf16x6"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    T.load()
    return _t


def gpu(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run_gpu(torch, pos, box, edges, lmax, mults, prec, w=None, n_data=None, flags=0, refine=0,
            want_alm=False, want_nnn=False):
    say(f"  gpu: n={pos.shape[0]} box={box} nb={len(edges) - 1} lmax={lmax} prec={PNAME[prec]} "
        f"refine={refine} weighted={w is not None}")
    h = T.Handle(box, edges, lmax, precision=prec, flags=flags, grid_refine=refine)
    P = gpu(torch, pos)
    W = gpu(torch, w)
    h.build_grid(P, W, n_data)
    h.alm_accumulate()
    alm = h.get_alm(0, pos.shape[0]).cpu().numpy() if want_alm else None
    nnn = h.contract(export=want_nnn)
    out = h.multipoles(mults)
    h.sync()
    npairs = h.pair_count()
    res = out.cpu().numpy()
    nnn = nnn.cpu().numpy() if nnn is not None else None
    h.close()
    return res, npairs, alm, nnn


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


C1 = dict(n=2000, box=200.0, edges=np.linspace(0.0, 40.0, 9), lmax=4, Lmax=2)


@pytest.fixture(scope="module")
def c1_case():
    pos = C.poisson(C1["n"], C1["box"], C.catalogue_seed(0))
    mults = O.all_multipoles(C1["lmax"], C1["Lmax"])
    re, im, res = O.run(pos, C1["box"], C1["edges"], C1["lmax"], mults)
    return pos, mults, re, res


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32, T.PREC_MIXED_BF16X6])
def test_c1_multipoles_match_oracle(torch, c1_case, prec):
    pos, mults, ref, res = c1_case
    got, npairs, _, _ = run_gpu(torch, pos, C1["box"], C1["edges"], C1["lmax"], mults, prec)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  C1 {PNAME[prec]} rel err {err:.3e}")
    assert err < TOL[prec]


# Dense anchor: 10^4 clustered points in a 400 Mpc/h box (mean density
# 1.56e-4, close to the 400k-in-1500 catalogue), 12 bins over [10, 130],
# lmax = 10, L <= 4.
DENSE = dict(n=10000, box=400.0, edges=np.linspace(10.0, 130.0, 13), lmax=10, Lmax=4)


@pytest.fixture(scope="module")
def dense_case():
    pos = C.zeldovich(DENSE["n"], DENSE["box"], 5.0, 0.8, C.catalogue_seed(3), grid=64)
    mults = O.all_multipoles(DENSE["lmax"], DENSE["Lmax"])
    say("  oracle: dense anchor")
    re, im, res = O.run(pos, DENSE["box"], DENSE["edges"], DENSE["lmax"], mults)
    return pos, mults, re, res


@pytest.mark.parametrize("prec", PRECS)
def test_dense_multipoles_match_oracle(torch, dense_case, prec):
    pos, mults, ref, res = dense_case
    got, npairs, _, _ = run_gpu(torch, pos, DENSE["box"], DENSE["edges"], DENSE["lmax"], mults,
                                prec)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  dense {PNAME[prec]} rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
def test_alm_and_nnn_match_oracle(torch, prec):
    box, edges, lmax = 100.0, np.array([4.0, 9.0, 14.0, 20.0, 25.0]), 6
    pos = C.zeldovich(3000, box, 2.0, 0.8, 77, grid=32)
    res = O.estimate(pos, box, edges, lmax, want_alm=True)
    mults = O.all_multipoles(lmax, 2)
    _, npairs, alm, nnn = run_gpu(torch, pos, box, edges, lmax, mults, prec, want_alm=True,
                                  want_nnn=True)
    assert npairs == res.npairs
    s1 = lmax + 1
    mask = np.tril(np.ones((s1, s1), dtype=bool))  # m <= l
    ea = np.abs(alm[..., mask] - res.alm[..., mask]).max() / np.abs(res.alm).max()
    say(f"  a_lm {PNAME[prec]} rel err {ea:.3e}")
    assert ea < (1e-12 if prec == T.PREC_FP64 else 1e-5)
    ref = res.nnn.real
    en = np.abs(nnn - ref).max() / np.abs(ref).max()
    say(f"  NNN {PNAME[prec]} rel err {en:.3e}")
    assert en < (1e-12 if prec == T.PREC_FP64 else 1e-5)


@pytest.mark.parametrize("prec", PRECS)
def test_weighted_data_minus_randoms(torch, prec):
    box, edges, lmax = 60.0, np.array([2.0, 5.0, 8.0, 12.0]), 3
    nd, nr = 400, 800
    pos = np.vstack([C.zeldovich(nd, box, 1.5, 0.8, 91, grid=16), C.randoms(nr, box, 92)])
    w = C.dr_weights(nd, nr)
    mults = O.all_multipoles(lmax, 3)
    ref, _, res = O.run(pos, box, edges, lmax, mults, w=w, n_data=nd)
    got, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec, w=w, n_data=nd)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  D-R {PNAME[prec]} rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("lmax", [8, 12, 13, 16])
@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32, T.PREC_MIXED_BF16X6])
def test_high_lmax_split_harmonics(torch, prec, lmax, weighted):
    """High orders, where the harmonic pass splits the m range of a list over
    two launches (FP64 from lmax 7 on, FP32 from lmax 11 on) and from lmax 13
    over three (FP32) or four (FP64), with unit weights (the self moments of
    order <= lmax shared with the m = 0 sums) and with data-minus-randoms
    weights. The FP32 pass is the one of every mixed path; the 3-product split
    is left to the dense configuration, since its degenerate-triangle error
    grows with 2l+1 over the few neighbours per bin of this catalogue."""
    box, edges = 60.0, np.array([2.0, 5.0, 8.0, 12.0])
    nd, nr = 300, 600
    pos = np.vstack([C.zeldovich(nd, box, 1.5, 0.8, 93, grid=16), C.randoms(nr, box, 94)])
    w = C.dr_weights(nd, nr) if weighted else None
    n_data = nd if weighted else None
    mults = O.all_multipoles(lmax, 2)
    ref, _, res = O.run(pos, box, edges, lmax, mults, w=w, n_data=n_data)
    got, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec, w=w, n_data=n_data)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  lmax {lmax} weighted={weighted} {PNAME[prec]} rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("lmax", [13, 16])
@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
def test_alm_and_nnn_match_oracle_top_lmax(torch, prec, lmax):
    """Every a_lm and every per-m sum NNN^m at the top of the lmax range, where
    each list is accumulated in three (FP32) or four (FP64) launches over
    parts of the m range, against the oracle element by element."""
    box, edges = 80.0, np.array([3.0, 7.0, 11.0, 15.0])
    pos = C.zeldovich(1200, box, 2.0, 0.8, 171 + lmax, grid=16)
    res = O.estimate(pos, box, edges, lmax, want_alm=True)
    mults = O.all_multipoles(lmax, 2)
    _, npairs, alm, nnn = run_gpu(torch, pos, box, edges, lmax, mults, prec, want_alm=True, want_nnn=True)
    assert npairs == res.npairs
    s1 = lmax + 1
    mask = np.tril(np.ones((s1, s1), dtype=bool))  # m <= l
    ea = np.abs(alm[..., mask] - res.alm[..., mask]).max() / np.abs(res.alm).max()
    ref = res.nnn.real
    en = np.abs(nnn - ref).max() / np.abs(ref).max()
    say(f"  lmax {lmax} {PNAME[prec]}: a_lm rel err {ea:.3e}, NNN rel err {en:.3e}")
    assert ea < (1e-12 if prec == T.PREC_FP64 else 1e-5)
    assert en < (1e-12 if prec == T.PREC_FP64 else 1e-5)


@pytest.mark.parametrize("prec", [T.PREC_MIXED_BF16X3, T.PREC_MIXED_BF16X6])
def test_largest_operand_weighted_mixed(torch, prec):
    """32 bins at lmax 16 with weights: one split-BF16 step cannot stage the
    544 columns, so the contraction runs on FP32 MFMA; the multipoles still
    match the oracle within the requested precision's tolerance."""
    box, edges = 60.0, np.linspace(2.0, 14.0, 33)
    nd, nr = 200, 400
    pos = np.vstack([C.zeldovich(nd, box, 1.5, 0.8, 181, grid=16), C.randoms(nr, box, 182)])
    w = C.dr_weights(nd, nr)
    mults = O.all_multipoles(16, 2)
    ref, _, res = O.run(pos, box, edges, 16, mults, w=w, n_data=nd)
    got, npairs, _, _ = run_gpu(torch, pos, box, edges, 16, mults, prec, w=w, n_data=nd)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  32 bins, lmax 16, weighted {PNAME[prec]} rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_single_cell_box_and_bins_from_zero(torch, prec):
    """rmax close to L/2: one cell with per-pair minimum image; first bin from 0."""
    box, edges, lmax = 10.0, np.array([0.0, 1.5, 3.0, 4.9]), 4
    pos = C.poisson(300, box, 101)
    mults = O.all_multipoles(lmax, 4)
    ref, _, res = O.run(pos, box, edges, lmax, mults)
    got, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  single-cell {PNAME[prec]} rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("refine", [1, 2, 3, 4])
def test_lmax0_exact_counts_every_grid(torch, refine):
    """lmax = 0: integer triplet counts, exact on every precision path and
    every neighbour-grid refinement (pins the pair set and the binning)."""
    box, edges = 120.0, np.linspace(5.0, 30.0, 6)
    pos = C.zeldovich(4000, box, 3.0, 0.8, 111, grid=32)
    ref, _, res = O.run(pos, box, edges, 0, [(0, 0, 0)])
    for prec in PRECS:
        got, npairs, _, _ = run_gpu(torch, pos, box, edges, 0, [(0, 0, 0)], prec, refine=refine)
        assert npairs == res.npairs
        err = rel_err(got, ref)
        assert err < 1e-12, (PNAME[prec], err)


@pytest.mark.parametrize("refine", [1, 2, 3, 4])
def test_lattice_ties_full_items(torch, refine):
    """Half-spaced lattice (8 points per unit volume) with edges at multiples
    of 0.5: most pairs lie exactly on an edge, so nearly every test goes to the
    exact FP64 decision that follows each tile. Cells hold 125 (refine 1) or
    16 (refine 2) points, so work items are full (every primary slot of every
    wavefront) and stencils span many tiles. lmax = 0 integer counts, exact on
    every precision path."""
    g = np.arange(40) * 0.5
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    box, edges = 20.0, np.array([0.5, 1.0, 1.5, 2.0, 2.5])
    ref, _, res = O.run(pos, box, edges, 0, [(0, 0, 0)])
    for prec in PRECS:
        got, npairs, _, _ = run_gpu(torch, pos, box, edges, 0, [(0, 0, 0)], prec, refine=refine)
        assert npairs == res.npairs, PNAME[prec]
        err = rel_err(got, ref)
        assert err < 1e-12, (PNAME[prec], err)


def test_lattice_ties_on_bin_edges(torch):
    """Dyadic lattice: many pairs exactly on bin edges (half-open bins)."""
    box, edges = 16.0, np.array([0.5, 1.0, 1.5, 2.0, 3.0])
    pos = np.unique(C.dyadic_lattice(1500, box, 5, 121), axis=0)
    for lmax in (0, 3):
        mults = O.all_multipoles(lmax, 2)
        ref, _, res = O.run(pos, box, edges, lmax, mults)
        for prec in PRECS:
            got, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec)
            assert npairs == res.npairs, PNAME[prec]
            assert rel_err(got, ref) < TOL[prec], PNAME[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_lattice_directions_alm(torch, prec):
    """Integer lattice at lmax 10: every hit lies along an axis, a face or a
    body diagonal, or another lattice direction, so the FP32 records meet
    the special cases of their direction code (the poles, the equator z = 0,
    the fold of the lower half, zero components of either sign). a_lm of
    every primary against the oracle."""
    g = np.arange(12, dtype=np.float64)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3) + 0.25
    box, edges, lmax = 12.0, np.array([0.5, 1.2, 1.6, 2.1, 3.1]), 10
    res = O.estimate(pos, box, edges, lmax, want_alm=True)
    mults = O.all_multipoles(lmax, 2)
    _, npairs, alm, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec, want_alm=True)
    assert npairs == res.npairs
    s1 = lmax + 1
    mask = np.tril(np.ones((s1, s1), dtype=bool))  # m <= l
    ea = np.abs(alm[..., mask] - res.alm[..., mask]).max() / np.abs(res.alm).max()
    say(f"  lattice a_lm {PNAME[prec]} rel err {ea:.3e}")
    assert ea < (1e-12 if prec == T.PREC_FP64 else 1e-5)


def test_keep_degenerate_and_literal_flags(torch):
    box, edges, lmax = 50.0, np.array([2.0, 6.0, 10.0]), 3
    pos = C.poisson(600, box, 131)
    mults = O.all_multipoles(lmax, 2)
    ref_keep, _, _ = O.run(pos, box, edges, lmax, mults, subtract_self=False)
    got, _, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, T.PREC_FP64,
                           flags=T.F_KEEP_DEGENERATE)
    assert rel_err(got, ref_keep) < 1e-12
    ref_lit, _, _ = O.run(pos, box, edges, lmax, mults, literal=True)
    got, _, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, T.PREC_FP64,
                           flags=T.F_PAPER_LITERAL)
    assert rel_err(got, ref_lit) < 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_batched_equals_single_bitwise(torch, prec):
    box, edges, lmax = 150.0, np.linspace(10.0, 40.0, 4), 4
    sizes = [1500, 700, 2600]
    cats = [C.zeldovich(n, box, 3.0, 0.8, 200 + i, grid=32) for i, n in enumerate(sizes)]
    mults = O.all_multipoles(lmax, 2)
    h = T.Handle(box, edges, lmax, precision=prec)
    say(f"  batched {PNAME[prec]}")
    P = gpu(torch, np.vstack(cats))
    out = h.run_catalogs(sizes, sizes, P, None, mults)
    h.sync()
    out2 = h.run_catalogs(sizes, sizes, P, None, mults)
    h.sync()
    batched = out.cpu().numpy()
    assert np.array_equal(batched, out2.cpu().numpy()), "run-to-run difference"
    for i, cat in enumerate(cats):
        single, _, _, _ = run_gpu(torch, cat, box, edges, lmax, mults, prec)
        assert np.array_equal(batched[i], single), i
        ref, _, _ = O.run(cat, box, edges, lmax, mults)
        assert rel_err(single, ref) < TOL[prec]
    h.close()


@pytest.mark.parametrize("prec", [T.PREC_MIXED_BF16X3, T.PREC_MIXED_BF16X6])
@pytest.mark.parametrize("Lmax", [0, 2, 4])
def test_coupled_tiles_only_batched_equals_steps(torch, prec, Lmax):
    """lmax 10 with 10 bins: 110 columns at m = 0, four 32-column tiles a
    side. A batched run whose multipoles have L <= Lmax forms only the tiles
    that couple some |l1 - l2| <= Lmax (3 of the 10 of m = 0 skipped at Lmax
    2); its multipoles equal those of the step calls, which form every tile,
    bit for bit, and the oracle's within the tolerance."""
    box, edges, lmax = 220.0, np.linspace(8.0, 48.0, 11), 10
    pos = C.zeldovich(2500, box, 3.0, 0.8, 331 + Lmax, grid=32)
    mults = O.all_multipoles(lmax, Lmax)
    n = pos.shape[0]
    h = T.Handle(box, edges, lmax, precision=prec)
    batched = h.run_catalogs([n], [n], gpu(torch, pos), None, mults).cpu().numpy()[0]
    h.sync()
    h.close()
    steps, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec)
    assert np.array_equal(batched, steps)
    ref, _, res = O.run(pos, box, edges, lmax, mults)
    assert npairs == res.npairs
    err = rel_err(batched, ref)
    say(f"  coupled tiles {PNAME[prec]} Lmax {Lmax}: {len(mults)} multipoles, rel err {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
def test_list_room_exhausted_pass_redone(torch, prec):
    """Half of the points in one tight clump: their pairs exceed the list room
    sized from the mean density several times over, so the pair pass runs out
    of room, which it learns only after its last chunk, and is run again with
    more room. The result still matches the oracle, and the pair count is
    exact."""
    box, edges, lmax = 100.0, np.array([1.0, 4.0, 7.0, 10.0]), 2
    rng = np.random.default_rng(C.catalogue_seed(11))
    clump = np.mod(50.0 + rng.normal(0.0, 1.2, size=(2000, 3)), box)
    pos = np.vstack([C.poisson(2000, box, C.catalogue_seed(12)), clump])
    mults = O.all_multipoles(lmax, 2)
    ref, _, res = O.run(pos, box, edges, lmax, mults)
    # the list room of the first pass: 1.15 (64 + sum_b 1.15 pred_b + 4 sqrt(pred_b) + 9)
    # entries per primary (pred_b the mean-density count of bin b), at least 1e6
    n = pos.shape[0]
    pred = n / box ** 3 * 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    room = max(1e6, 1.15 * n * (64.0 + np.sum(1.15 * pred + 4.0 * np.sqrt(pred) + 9.0)))
    assert res.npairs > 2.0 * room
    got, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, mults, prec)
    say(f"  lists exhausted {PNAME[prec]}: {npairs} pairs against room for {room:.0f}, "
        f"rel err {rel_err(got, ref):.3e}")
    assert npairs == res.npairs
    assert rel_err(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
def test_crowded_cluster_exact_rebinning(torch, prec):
    """A dense clump inside a sparse box: its members see far more close
    neighbours than their cell's stencil predicts, so they take the exact
    rebinning path; the result must still match the oracle."""
    box, edges, lmax = 120.0, np.linspace(2.0, 30.0, 8), 4
    rng = np.random.default_rng(C.catalogue_seed(9))
    clump = 40.0 + rng.normal(0.0, 1.5, size=(600, 3))
    pos = np.vstack([C.poisson(1400, box, C.catalogue_seed(8)), np.mod(clump, box)])
    mults = O.all_multipoles(lmax, 2)
    ref, _, res = O.run(pos, box, edges, lmax, mults)
    h = T.Handle(box, edges, lmax, precision=prec)
    h.build_grid(gpu(torch, pos))
    h.alm_accumulate()
    h.contract()
    out = h.multipoles(mults)
    h.sync()
    npairs, nfix = h.pair_count(), h.rebinned_count()
    h.close()
    say(f"  crowded {PNAME[prec]}: rebinned primaries {nfix}")
    assert nfix > 0
    assert npairs == res.npairs
    assert rel_err(out.cpu().numpy(), ref) < TOL[prec]


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("prec", [T.PREC_FP32, T.PREC_MIXED_BF16X3])
def test_run_catalogs_self_orders(torch, prec, weighted):
    """A batched run whose multipoles all have L <= lmax stops the self
    moments at order lmax (the others cancel from every such multipole), and
    its contraction skips the blocks of |l1 - l2| above its multipoles'. Its
    result equals that of the step calls, which keep every order and block,
    bit for bit; afterwards the per-m export, multipoles of L > lmax and
    multipoles needing the skipped blocks are refused."""
    box, edges, lmax, n = 150.0, np.linspace(10.0, 40.0, 4), 4, 3000
    cats = [C.zeldovich(n, box, 3.0, 0.8, 151 + i, grid=32) for i in range(2)]
    ws = [np.random.default_rng(161 + i).uniform(0.5, 1.5, n) for i in range(2)] if weighted else [None, None]
    mults = O.all_multipoles(lmax, 2)
    h = T.Handle(box, edges, lmax, precision=prec)
    out = h.run_catalogs([n, n], [n, n], gpu(torch, np.vstack(cats)),
                         gpu(torch, np.concatenate(ws)) if weighted else None, mults)
    h.sync()
    batched = out.cpu().numpy()
    with pytest.raises(T.TpcfError) as e:
        h.contract(export=True)
    assert e.value.status == T.TPCF_ERR_STATE
    with pytest.raises(T.TpcfError) as e:
        h.multipoles([(4, 4, 6)])
    assert e.value.status == T.TPCF_ERR_STATE
    # the handle holds two catalogues' sums: the one-catalogue multipole call
    # is refused (its output has room for one)
    with pytest.raises(T.TpcfError) as e:
        h.multipoles(mults[:3])
    assert e.value.status == T.TPCF_ERR_STATE
    # A one-catalogue run: its contraction summed only the blocks with
    # |l1 - l2| <= 2 (the largest of its multipoles). A triple needing
    # |l1 - l2| = 4 is refused; one within the run's blocks is given, equal to
    # the run's own result.
    one = h.run_catalogs([n], [n], gpu(torch, cats[0]), gpu(torch, ws[0]) if weighted else None, mults)
    h.sync()
    assert np.array_equal(one.cpu().numpy()[0], batched[0])
    with pytest.raises(T.TpcfError) as e:
        h.multipoles([(0, 4, 4)])
    assert e.value.status == T.TPCF_ERR_STATE
    again = h.multipoles(mults[:3]).cpu().numpy()
    h.sync()
    assert np.array_equal(again, batched[0][:3])
    h.close()
    for i in range(2):
        h = T.Handle(box, edges, lmax, precision=prec)
        h.build_grid(gpu(torch, cats[i]), gpu(torch, ws[i]))
        h.alm_accumulate()
        h.contract()
        single = h.multipoles(mults).cpu().numpy()
        h.sync()
        h.close()
        assert np.array_equal(single, batched[i]), i
    ref, _, _ = O.run(cats[0], box, edges, lmax, mults, w=ws[0])
    err = rel_err(batched[0], ref)
    say(f"  batched self orders {PNAME[prec]} weighted={weighted} rel err {err:.3e}")
    assert err < TOL[prec]


def test_nonfinite_positions_reported(torch):
    pos = C.poisson(500, 50.0, 141)
    pos[17, 1] = np.nan
    h = T.Handle(50.0, np.array([1.0, 5.0]), 2, precision=T.PREC_FP32)
    h.build_grid(gpu(torch, pos))
    with pytest.raises(T.TpcfError) as e:
        h.alm_accumulate()
    assert e.value.status == T.TPCF_ERR_DEVICE
    h.close()


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_MIXED_BF16X3])
def test_bad_catalogue_isolated_in_batch(torch, prec):
    """A batch of five catalogues, the second and the last with a non-finite
    coordinate: run_catalogs reports those two (TPCF_ERR_DEVICE, status per
    catalogue), their results are NaN, and the other three equal, bit for bit,
    those of a batch of only the good catalogues."""
    box, edges, lmax = 150.0, np.linspace(10.0, 40.0, 4), 4
    sizes = [1500, 700, 2600, 900, 1100]
    cats = [C.zeldovich(n, box, 3.0, 0.8, 300 + i, grid=32) for i, n in enumerate(sizes)]
    cats[1][333, 2] = np.nan
    cats[4][0, 0] = np.inf
    mults = O.all_multipoles(lmax, 2)
    h = T.Handle(box, edges, lmax, precision=prec)
    out = torch.zeros((5, len(mults), 3, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(T.TpcfError) as e:
        h.run_catalogs(sizes, sizes, gpu(torch, np.vstack(cats)), None, mults, out=out)
    assert e.value.status == T.TPCF_ERR_DEVICE
    assert "(1, 4)" in str(e.value)
    st = h.catalog_status(5)
    assert st.tolist() == [0, T.TPCF_ERR_DEVICE, 0, 0, T.TPCF_ERR_DEVICE]
    h.sync()
    got = out.cpu().numpy()
    assert np.isnan(got[[1, 4]]).all()
    good = [0, 2, 3]
    ref = h.run_catalogs([sizes[i] for i in good], [sizes[i] for i in good],
                         gpu(torch, np.vstack([cats[i] for i in good])), None, mults)
    h.sync()
    assert h.catalog_status(3).tolist() == [0, 0, 0]
    with pytest.raises(T.TpcfError) as e:
        h.catalog_status(5)
    assert e.value.status == T.TPCF_ERR_ARG
    ref = ref.cpu().numpy()
    for k, i in enumerate(good):
        assert np.array_equal(got[i], ref[k]), i
    say(f"  bad catalogues isolated ({PNAME[prec]}): statuses {st.tolist()}")
    h.close()


@pytest.mark.parametrize("prec", PRECS)
def test_degenerate_catalogues_alone_and_batched(torch, prec):
    """Catalogues at the edge of the method: one point (no pair), points
    farther apart than the last edge (no pair in any shell), and an
    equilateral triangle inside one bin (every ordered distinct triplet in
    that bin, 6 of them), each alone and together with a normal catalogue in
    one ragged batch. Pair counts are exact, the multipoles equal the oracle's
    (zero where there is no pair), and the batched results equal the single
    runs bit for bit."""
    box, edges, lmax = 100.0, np.array([2.0, 4.0, 6.0, 8.0]), 2
    mults = O.all_multipoles(lmax, 2)
    one = np.array([[10.0, 20.0, 30.0]])
    apart = np.array([[5.0, 5.0, 5.0], [30.0, 5.0, 5.0], [5.0, 60.0, 5.0], [70.0, 70.0, 70.0]])
    tri = 50.0 + np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0], [2.5, 5.0 * np.sqrt(3.0) / 2.0, 1.0]])
    normal = C.zeldovich(800, box, 2.0, 0.8, 191, grid=16)
    cats = [one, apart, tri, normal]
    nd = [3, 4, 3, 800]  # n_data >= 3 for RRR
    singles, counts = [], []
    for cat, n_data in zip(cats, nd):
        ref, _, res = O.run(cat, box, edges, lmax, mults, n_data=n_data)
        got, npairs, _, _ = run_gpu(torch, cat, box, edges, lmax, mults, prec, n_data=n_data)
        assert npairs == res.npairs
        counts.append(npairs)
        if res.npairs == 0:
            assert not np.any(got) and not np.any(ref)
        else:
            assert rel_err(got, ref) < TOL[prec]
        singles.append(got)
    # the triangle: 3 x 2 ordered distinct pairs, all in the middle bin
    assert O.estimate(tri, box, edges, 0).npairs == 6
    h = T.Handle(box, edges, lmax, precision=prec)
    out = h.run_catalogs([c.shape[0] for c in cats], nd, gpu(torch, np.vstack(cats)), None, mults)
    h.sync()
    h.close()
    batched = out.cpu().numpy()
    for i in range(len(cats)):
        assert np.array_equal(batched[i], singles[i]), i
    say(f"  degenerate catalogues {PNAME[prec]}: pairs {counts}, batched == single")


def test_out_of_order_calls(torch):
    h = T.Handle(50.0, np.array([1.0, 5.0]), 2)
    with pytest.raises(T.TpcfError) as e:
        h.alm_accumulate()
    assert e.value.status == T.TPCF_ERR_STATE
    with pytest.raises(T.TpcfError) as e:
        h.multipoles([(0, 0, 0)])
    assert e.value.status == T.TPCF_ERR_STATE
    with pytest.raises(T.TpcfError) as e:
        h.multipoles([(1, 0, 0)])
    assert e.value.status == T.TPCF_ERR_ARG
    h.close()


def test_double_destroy_and_use_after_destroy(torch):
    """A destroyed handle is refused by every call (looked up in the library's
    set of live handles, not read), and destroying it again is a no-op."""
    h = T.Handle(50.0, np.array([1.0, 5.0]), 2)
    raw = ctypes.c_void_p(h.h.value)
    lib = h.lib
    assert lib.tpcf_sync(raw) == T.TPCF_OK
    lib.tpcf_destroy(raw)
    h.h = None
    lib.tpcf_destroy(raw)
    assert lib.tpcf_sync(raw) == T.TPCF_ERR_ARG
    assert lib.tpcf_alm_accumulate(raw) == T.TPCF_ERR_ARG
    assert b"invalid or destroyed" in lib.tpcf_last_error(raw)
    # a new handle works after the dead one
    h2 = T.Handle(50.0, np.array([1.0, 5.0]), 2)
    h2.sync()
    h2.close()


def test_workspace_limit_enforced(torch):
    pos = C.poisson(20000, 100.0, 151)
    h = T.Handle(100.0, np.linspace(2.0, 20.0, 10), 10, workspace_limit=1 << 20)
    with pytest.raises(T.TpcfError) as e:
        h.build_grid(gpu(torch, pos))
        h.alm_accumulate()
    assert e.value.status == T.TPCF_ERR_ALLOC
    h.close()


# ------------------------------------------------------------------ isotropic schedule


def iso_rows(mults, lmax):
    """Indices of the (l, l, 0) triples in mults, l = 0..lmax."""
    idx = {tuple(t): i for i, t in enumerate(mults)}
    return [idx[(l, l, 0)] for l in range(lmax + 1)]


@pytest.mark.parametrize("prec", PRECS)
def test_isotropic_matches_oracle(torch, dense_case, prec):
    """TPCF_F_ISOTROPIC forms only the l1 = l2 blocks (FP64 MFMA); its (l, l, 0)
    outputs, the Legendre coefficients zeta_l(r1, r2), match the oracle within
    1e-12 (FP64 pair pass) or 1e-5 (FP32 pair pass)."""
    pos, mults, ref, res = dense_case
    lmax = DENSE["lmax"]
    iso = [(l, l, 0) for l in range(lmax + 1)]
    got, npairs, _, nnn = run_gpu(torch, pos, DENSE["box"], DENSE["edges"], lmax, iso, prec,
                                  flags=T.F_ISOTROPIC, want_nnn=True)
    assert npairs == res.npairs
    r = ref[iso_rows(mults, lmax)]
    err = rel_err(got, r)
    say(f"  isotropic {PNAME[prec]} rel err {err:.3e}")
    assert err < (1e-12 if prec == T.PREC_FP64 else 1e-5)
    # exported NNN^m: zero off the l1 = l2 blocks, the oracle's on them
    s1 = lmax + 1
    off = np.ones((s1, s1), dtype=bool)
    np.fill_diagonal(off, False)
    assert np.all(nnn[:, off] == 0.0)
    diag = np.array([nnn[m, l, l] for m in range(s1) for l in range(m, s1)])
    rdiag = np.array([res.nnn[m, l, l].real for m in range(s1) for l in range(m, s1)])
    derr = float(np.abs(diag - rdiag).max() / np.abs(rdiag).max())
    assert derr < (1e-12 if prec == T.PREC_FP64 else 1e-5), derr


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
def test_isotropic_weighted_and_wide(torch, prec):
    """Data minus randoms weights, and 20 bins (two 16-bin tiles of the block)."""
    box, nd = 300.0, 3000
    edges = np.linspace(4.0, 64.0, 21)
    lmax = 4
    D = C.zeldovich(nd, box, 4.0, 0.8, C.catalogue_seed(70), grid=64)
    pos = np.vstack([D, C.randoms(2 * nd, box, C.randoms_seed(70))])
    w = C.dr_weights(nd, 2 * nd)
    iso = [(l, l, 0) for l in range(lmax + 1)]
    say("  oracle: weighted isotropic case")
    ref, _, res = O.run(pos, box, edges, lmax, iso, w=w, n_data=nd)
    got, npairs, _, _ = run_gpu(torch, pos, box, edges, lmax, iso, prec, w=w, n_data=nd,
                                flags=T.F_ISOTROPIC)
    assert npairs == res.npairs
    err = rel_err(got, ref)
    say(f"  isotropic weighted {PNAME[prec]} rel err {err:.3e}")
    assert err < (1e-12 if prec == T.PREC_FP64 else 1e-5)


def test_isotropic_rejects_anisotropic_triples(torch):
    h = T.Handle(200.0, np.linspace(0.0, 40.0, 9), 4, flags=T.F_ISOTROPIC)
    h.build_grid(gpu(torch, C.poisson(500, 200.0, 3)))
    h.alm_accumulate()
    h.contract()
    with pytest.raises(T.TpcfError) as e:
        h.multipoles([(2, 0, 2)])
    assert e.value.status == T.TPCF_ERR_ARG
    h.close()


# ------------------------------------------------------------------ autotuner


def test_autotune_keeps_results(torch, dense_case):
    """The autotuner picks an admissible grid refinement by timing; the pair
    count is unchanged and the FP64 multipoles agree to rounding."""
    pos, mults, ref, res = dense_case
    h = T.Handle(DENSE["box"], DENSE["edges"], DENSE["lmax"], precision=T.PREC_FP64)
    P = gpu(torch, pos)
    k, ms = h.autotune(P)
    say(f"  autotune: refinement {k}, ms per refinement {np.round(ms, 2).tolist()}")
    assert 1 <= k <= 4 and ms[k - 1] > 0 and ms[k - 1] == ms[ms > 0].min()
    h.build_grid(P)
    h.alm_accumulate()
    h.contract()
    out = h.multipoles(mults).cpu().numpy()
    h.sync()
    assert h.pair_count() == res.npairs
    h.close()
    assert rel_err(out, ref) < 1e-12
    # the 2PCF counts tuned the same way
    h = T.Handle(400.0, np.linspace(0.0, 60.0, 13), 0)
    k2, ms2 = h.autotune(P, nmu=40)
    assert 1 <= k2 <= 4 and ms2[k2 - 1] == ms2[ms2 > 0].min()
    h.build_grid(P)
    dd = h.xi_count(40).cpu().numpy()
    h.close()
    assert np.array_equal(dd, O.xi_counts(pos, 400.0, np.linspace(0.0, 60.0, 13), 40))


def test_autotune_plan_keeps_results(torch, tmp_path):
    """The plan autotuner times refinements, list modes and contraction steps
    on a sample and keeps the fastest; the plan cache returns it without
    timing. Across every plan, lmax = 0 triplet counts are bit-exact (the pair
    set does not depend on the plan) and the lmax = 4 multipoles of the FP32
    pair pass stay within the FP32 tolerance of the oracle."""
    box, edges = 120.0, np.linspace(5.0, 30.0, 6)
    pos = C.zeldovich(4000, box, 3.0, 0.8, 112, grid=32)
    P = gpu(torch, pos)
    ref0, _, res = O.run(pos, box, edges, 0, [(0, 0, 0)])
    mults = O.all_multipoles(4, 2)
    ref4, _, _ = O.run(pos, box, edges, 4, mults)
    cache = str(tmp_path / "plans.json")
    for prec in (T.PREC_FP32, T.PREC_MIXED_BF16X6):
        h = T.Handle(box, edges, 4, precision=prec)
        plan = h.autotune_plan(P, cache=cache)
        say(f"  {PNAME[prec]}: tuned plan {plan}")
        assert not plan["cached"] and plan["ms"] > 0
        assert 1 <= plan["grid_refine"] <= 4 and plan["list_mode"] in (0, 1)
        cur = h.get_plan()
        assert (cur["grid_refine"], cur["list_mode"], cur["contract_step"]) == \
            (plan["grid_refine"], plan["list_mode"], plan["contract_step"])
        again = h.autotune_plan(P, cache=cache)
        assert again["cached"] and again["grid_refine"] == plan["grid_refine"]
        assert again["list_mode"] == plan["list_mode"] and again["contract_step"] == plan["contract_step"]
        h.close()
        for k in (1, 2, 3):
            for mode in (0, 1):
                for step in (0, 32):
                    h0 = T.Handle(box, edges, 0, precision=prec)
                    h0.set_plan(k, mode, step)
                    h0.build_grid(P)
                    h0.alm_accumulate()
                    h0.contract()
                    c0 = h0.multipoles([(0, 0, 0)]).cpu().numpy()
                    h0.sync()
                    assert h0.pair_count() == res.npairs
                    h0.close()
                    assert rel_err(c0, ref0) < 1e-12, (k, mode, step)
                    h4 = T.Handle(box, edges, 4, precision=prec)
                    h4.set_plan(k, mode, step)
                    h4.build_grid(P)
                    h4.alm_accumulate()
                    h4.contract()
                    c4 = h4.multipoles(mults).cpu().numpy()
                    h4.sync()
                    h4.close()
                    assert rel_err(c4, ref4) < 1e-5, (PNAME[prec], k, mode, step, rel_err(c4, ref4))


# ------------------------------------------------------------------ long lists


@pytest.mark.parametrize("weighted", [False, True])
def test_long_lists_wave_kernel(torch, weighted):
    """Hundreds of neighbours per (primary, bin) at lmax 4 (the wavefront-per-list
    harmonic kernel): a_lm of a slice of primaries against the oracle (FP32
    tolerance), and the multipoles against the FP64 path."""
    box, edges, lmax = 100.0, np.linspace(2.0, 20.0, 5), 4
    n = 40000
    pos = C.zeldovich(n, box, 2.0, 0.8, C.catalogue_seed(95), grid=64)
    w = None
    if weighted:
        w = np.random.default_rng(95).uniform(0.5, 1.5, n)
    mults = O.all_multipoles(lmax, 4)
    outs = {}
    for prec in (T.PREC_FP32, T.PREC_FP64):
        h = T.Handle(box, edges, lmax, precision=prec)
        h.build_grid(gpu(torch, pos), gpu(torch, w))
        h.alm_accumulate()
        alm = h.get_alm(12345, 32).cpu().numpy()
        h.contract()
        outs[prec] = h.multipoles(mults).cpu().numpy()
        h.sync()
        h.close()
        if prec == T.PREC_FP32:
            ref = O.estimate(pos, box, edges, lmax, w=w, prim_first=12345, prim_count=32, want_alm=True,
                             want_nnn=False).alm
            mask = np.tril(np.ones((lmax + 1, lmax + 1), dtype=bool))
            err = float(np.abs(alm[..., mask] - ref[..., mask]).max() / np.abs(ref[..., mask]).max())
            say(f"  long lists a_lm slice rel err {err:.2e} (weighted={weighted})")
            assert err < 1e-5
            # a_00 = count / sqrt(4 pi) for unit weights: lists average several hundred
            if not weighted:
                assert np.mean(ref[:, :, 0, 0].real) * math.sqrt(4 * math.pi) > 256
    err = rel_err(outs[T.PREC_FP32], outs[T.PREC_FP64])
    say(f"  long lists FP32 vs FP64 rel err {err:.2e}")
    assert err < 1e-5
    # the batched call runs the same kernel with the self moments stopped at
    # lmax (every L here is <= lmax): bit for bit the step calls' result
    h = T.Handle(box, edges, lmax, precision=T.PREC_FP32)
    batched = h.run_catalogs([n], [n], gpu(torch, pos), gpu(torch, w), mults).cpu().numpy()
    h.sync()
    h.close()
    assert np.array_equal(batched[0], outs[T.PREC_FP32])
