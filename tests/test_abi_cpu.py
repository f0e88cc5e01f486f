"""C-ABI checks that need no GPU: the library builds/loads, exports every
symbol include/tpcf.h declares, and rejects invalid configurations before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2408_03036_amd import tpcf as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tpcf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpcf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        from paper_2408_03036_amd import build
        build.build()
    return T.load()


def test_header_and_binding_agree():
    assert _declared() == sorted(T.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def _create(lib, **kw):
    args = dict(box=200.0, edges=np.linspace(0.0, 40.0, 9), lmax=4)
    args.update(kw)
    cfg, keep = T.make_config(**args)
    h = ctypes.c_void_p()
    rc = lib.tpcf_create(ctypes.byref(cfg), 0, None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw,expect", [
    (dict(box=0.0), T.TPCF_ERR_ARG),
    (dict(box=float("nan")), T.TPCF_ERR_ARG),
    (dict(box=-5.0), T.TPCF_ERR_ARG),
    (dict(edges=[0.0, 10.0, 10.0]), T.TPCF_ERR_RANGE),
    (dict(edges=[5.0, 4.0, 10.0]), T.TPCF_ERR_RANGE),
    (dict(edges=[-1.0, 10.0]), T.TPCF_ERR_RANGE),
    (dict(edges=[0.0, 101.0]), T.TPCF_ERR_RANGE),
    (dict(lmax=17), T.TPCF_ERR_RANGE),
    (dict(lmax=-1), T.TPCF_ERR_RANGE),
    (dict(precision=4), T.TPCF_ERR_ARG),
    (dict(grid_refine=5), T.TPCF_ERR_RANGE),
    (dict(flags=8), T.TPCF_ERR_ARG),
    (dict(edges=np.linspace(0, 40, 34)), T.TPCF_ERR_RANGE),
])
def test_invalid_configs_rejected_before_device(lib, kw, expect):
    rc, h = _create(lib, **kw)
    assert rc == expect
    assert not h.value


def test_largest_config_fits_every_precision(lib):
    # 32 bins at lmax 16 is the largest operand: every precision plans its
    # contraction within LDS (the split-BF16 ones by running FP32 MFMA where a
    # weighted step would not fit the threads' registers), so creation fails
    # only for want of a device
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    for lmax in (12, 13, 16):
        for prec in range(4):
            rc, h = _create(lib, lmax=lmax, edges=np.linspace(0, 40, 33), precision=prec)
            assert rc == T.TPCF_ERR_DEVICE, (lmax, prec)


def test_null_arguments(lib):
    cfg, keep = T.make_config(200.0, np.linspace(0, 40, 9), 4)
    assert lib.tpcf_create(ctypes.byref(cfg), 0, None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_create(None, 0, None, ctypes.byref(ctypes.c_void_p())) == T.TPCF_ERR_ARG
    # calls on a NULL handle fail cleanly
    assert lib.tpcf_build_grid(None, None, None, 10, 10) == T.TPCF_ERR_ARG
    assert lib.tpcf_alm_accumulate(None) == T.TPCF_ERR_ARG
    assert lib.tpcf_sync(None) == T.TPCF_ERR_ARG
    assert lib.tpcf_rebinned_count(None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_xi_count(None, 10, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_xi_multipoles(None, 10, None, 10, 1, None, None) == T.TPCF_ERR_ARG
    assert b"invalid" in lib.tpcf_last_error(None)
    lib.tpcf_destroy(None)


def test_valid_config_without_gpu_reports_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _create(lib)
    assert rc == T.TPCF_ERR_DEVICE


def test_host_helpers_match_oracle(lib):
    """tpcf_triangle_index and tpcf_percival_m1 need no device: compare with the
    covariance oracle."""
    from oracle import cov_oracle as V
    edges = np.linspace(30.0, 150.0, 13)
    for eta, rmin in [(1, 0.0), (3, 0.0), (1, 40.0), (2, 55.0)]:
        sel = V.select_triangles(edges, eta, rmin)
        off = T.triangle_index(edges, eta, rmin, [0, 4])
        nb = 12
        ref = [(t * nb + b1) * nb + b2 for t in (0, 4) for (b1, b2) in sel]
        assert off.tolist() == ref, (eta, rmin)
    for nm, nd, npar in [(3000, 336, 6), (298, 48, 4), (100, 90, 3)]:
        assert abs(T.percival_m1(nm, nd, npar) - V.percival_m1(nm, nd, npar)) < 1e-14
    # and with the exact fractions evaluated by hand (tests/golden/percival_m1.json)
    import json
    import os
    from fractions import Fraction
    with open(os.path.join(os.path.dirname(__file__), "golden", "percival_m1.json")) as f:
        for g in json.load(f)["values"]:
            m1 = float(Fraction(*g["m1"]))
            assert abs(T.percival_m1(g["n_mocks"], g["n_d"], g["n_params"]) - m1) <= 4 * np.spacing(m1)
    with pytest.raises(T.TpcfError):
        T.triangle_index([0.0, 1.0, 3.0], 1, 0.0, [0])  # unequal bins
    with pytest.raises(T.TpcfError):
        T.percival_m1(10, 8, 2)  # too few mocks
    assert lib.tpcf_covariance(None, 10, 10, None, 5, None, None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_covariance_noalloc(None, 10, 10, None, 5, None, None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_precision_matrix(None, 5, None, 10, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_autotune(None, None, None, 10, 10, 0, None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_autotune_plan(None, 1, None, None, None, None, None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_set_plan(None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_get_plan(None, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_catalog_status(None, 1, None) == T.TPCF_ERR_ARG
    assert lib.tpcf_edge_correct_isotropic(None, 3, None, None, None) == T.TPCF_ERR_ARG


def test_foreign_and_dead_handles_are_refused_unread(lib):
    """Handles are checked against the library's set of live handles, never by
    reading through the pointer: a pointer that was never a handle (here the
    address of a host buffer filled with garbage) is refused by every call, and
    destroying it is a no-op. (A double destroy and a use after destroy of a
    real handle are tested on the GPU.)"""
    junk = (ctypes.c_ubyte * 4096)(*([0xAB] * 4096))
    bogus = ctypes.c_void_p(ctypes.addressof(junk))
    assert lib.tpcf_sync(bogus) == T.TPCF_ERR_ARG
    assert lib.tpcf_alm_accumulate(bogus) == T.TPCF_ERR_ARG
    assert lib.tpcf_contract(bogus, None) == T.TPCF_ERR_ARG
    st = (ctypes.c_int32 * 4)()
    assert lib.tpcf_catalog_status(bogus, 4, st) == T.TPCF_ERR_ARG
    assert b"invalid or destroyed" in lib.tpcf_last_error(bogus)
    lib.tpcf_destroy(bogus)
    lib.tpcf_destroy(bogus)
    assert bytes(junk) == bytes([0xAB] * 4096)  # nothing was written through it
