"""Python binding of libtpcf.so (include/tpcf.h): argument marshalling only.

Every step of the estimator runs in the library's HIP kernels; PyTorch only
provides device memory (tensors) and the stream. There is no fallback: if the
library is missing this module raises.

    h = Handle(box=1000.0, edges=np.linspace(20, 120, 11), lmax=10,
               precision=PREC_MIXED_BF16X3)
    out = h.run_catalogs(sizes, n_data, pos, None, mults)   # cuda tensors
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TPCF_LIBRARY selects another build of the library (for example the
# host-sanitized _build_san/libtpcf_san.so of build.py); default: the in-tree libtpcf.so
LIB_PATH = os.environ.get("TPCF_LIBRARY") or os.path.join(HERE, "libtpcf.so")

TPCF_OK = 0
TPCF_ERR_ARG = -1
TPCF_ERR_RANGE = -2
TPCF_ERR_ALLOC = -3
TPCF_ERR_DEVICE = -4
TPCF_ERR_STATE = -5
PREC_FP64 = 0
PREC_FP32 = 1
PREC_MIXED_BF16X3 = 2
PREC_MIXED_BF16X6 = 3
F_KEEP_DEGENERATE = 1
F_PAPER_LITERAL = 2
F_ISOTROPIC = 4

EXPORTS = ["tpcf_create", "tpcf_destroy", "tpcf_last_error", "tpcf_build_grid",
           "tpcf_alm_accumulate", "tpcf_get_alm", "tpcf_contract", "tpcf_multipoles",
           "tpcf_run_catalogs", "tpcf_sync", "tpcf_pair_count", "tpcf_rebinned_count", "tpcf_set_timing",
           "tpcf_stage_times", "tpcf_xi_count", "tpcf_xi_multipoles", "tpcf_triangle_index",
           "tpcf_covariance", "tpcf_covariance_noalloc", "tpcf_precision_matrix", "tpcf_percival_m1", "tpcf_edge_correct_isotropic", "tpcf_edge_correct",
           "tpcf_autotune", "tpcf_autotune_plan", "tpcf_set_plan", "tpcf_get_plan", "tpcf_catalog_status"]


class TpcfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tpcf status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double), ("nbins", ctypes.c_int32),
                ("h_edges", ctypes.POINTER(ctypes.c_double)), ("lmax", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("grid_refine", ctypes.c_int32), ("workspace_limit", ctypes.c_int64)]


class Plan(ctypes.Structure):
    _fields_ = [("grid_refine", ctypes.c_int32), ("list_mode", ctypes.c_int32),
                ("contract_step", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {"grid_refine": self.grid_refine, "list_mode": self.list_mode,
                "contract_step": self.contract_step, "ms": self.ms}


_lib = None


def load():
    """Loads libtpcf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run python -m paper_2408_03036_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    lib.tpcf_create.argtypes = [ctypes.POINTER(Config), ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.tpcf_create.restype = st
    lib.tpcf_destroy.argtypes = [vp]
    lib.tpcf_destroy.restype = None
    lib.tpcf_last_error.argtypes = [vp]
    lib.tpcf_last_error.restype = ctypes.c_char_p
    lib.tpcf_build_grid.argtypes = [vp, vp, vp, i64, i64]
    lib.tpcf_build_grid.restype = st
    lib.tpcf_alm_accumulate.argtypes = [vp]
    lib.tpcf_alm_accumulate.restype = st
    lib.tpcf_get_alm.argtypes = [vp, i64, i64, vp]
    lib.tpcf_get_alm.restype = st
    lib.tpcf_contract.argtypes = [vp, vp]
    lib.tpcf_contract.restype = st
    lib.tpcf_multipoles.argtypes = [vp, i32, vp, vp]
    lib.tpcf_multipoles.restype = st
    lib.tpcf_run_catalogs.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp]
    lib.tpcf_run_catalogs.restype = st
    lib.tpcf_catalog_status.argtypes = [vp, i32, vp]
    lib.tpcf_catalog_status.restype = st
    lib.tpcf_sync.argtypes = [vp]
    lib.tpcf_sync.restype = st
    lib.tpcf_pair_count.argtypes = [vp, ctypes.POINTER(i64)]
    lib.tpcf_pair_count.restype = st
    lib.tpcf_rebinned_count.argtypes = [vp, ctypes.POINTER(i64)]
    lib.tpcf_rebinned_count.restype = st
    lib.tpcf_set_timing.argtypes = [vp, ctypes.c_int]
    lib.tpcf_set_timing.restype = st
    lib.tpcf_stage_times.argtypes = [vp, i32, vp, vp]
    lib.tpcf_stage_times.restype = st
    lib.tpcf_xi_count.argtypes = [vp, i32, vp]
    lib.tpcf_xi_count.restype = st
    lib.tpcf_xi_multipoles.argtypes = [vp, i32, vp, i64, i32, vp, vp]
    lib.tpcf_xi_multipoles.restype = st
    lib.tpcf_triangle_index.argtypes = [i32, vp, dbl, dbl, i32, vp, i64, vp, ctypes.POINTER(i64)]
    lib.tpcf_triangle_index.restype = st
    lib.tpcf_covariance.argtypes = [vp, i32, i64, vp, i32, vp, vp, vp]
    lib.tpcf_covariance.restype = st
    lib.tpcf_covariance_noalloc.argtypes = [vp, i32, i64, vp, i32, vp, vp, vp]
    lib.tpcf_covariance_noalloc.restype = st
    lib.tpcf_precision_matrix.argtypes = [vp, i32, vp, i32, vp]
    lib.tpcf_precision_matrix.restype = st
    lib.tpcf_percival_m1.argtypes = [i32, i32, i32, ctypes.POINTER(dbl)]
    lib.tpcf_percival_m1.restype = st
    lib.tpcf_edge_correct_isotropic.argtypes = [vp, i32, vp, vp, vp]
    lib.tpcf_edge_correct_isotropic.restype = st
    lib.tpcf_edge_correct.argtypes = [vp, vp, i64, vp, i64, i32, vp, vp, vp]
    lib.tpcf_edge_correct.restype = st
    lib.tpcf_autotune.argtypes = [vp, vp, vp, i64, i64, i32, ctypes.POINTER(i32), vp]
    lib.tpcf_autotune.restype = st
    lib.tpcf_autotune_plan.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.POINTER(Plan), vp]
    lib.tpcf_autotune_plan.restype = st
    lib.tpcf_set_plan.argtypes = [vp, ctypes.POINTER(Plan)]
    lib.tpcf_set_plan.restype = st
    lib.tpcf_get_plan.argtypes = [vp, ctypes.POINTER(Plan)]
    lib.tpcf_get_plan.restype = st
    _lib = lib
    return lib


def make_config(box, edges, lmax, precision=PREC_MIXED_BF16X3, flags=0, grid_refine=0,
                workspace_limit=0):
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    cfg = Config(float(box), int(edges.shape[0] - 1),
                 edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(lmax),
                 int(precision), int(flags), int(grid_refine), int(workspace_limit))
    return cfg, edges


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_dev(t, dtype, name):
    import torch
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")


class Handle:
    """Owns one tpcf_handle on a device and a stream."""

    def __init__(self, box, edges, lmax, precision=PREC_MIXED_BF16X3, flags=0, grid_refine=0,
                 workspace_limit=0, device=0, stream=None):
        import torch
        self.lib = load()
        self.edges = np.ascontiguousarray(edges, dtype=np.float64)
        self.nbins = self.edges.shape[0] - 1
        self.lmax = int(lmax)
        self.box = float(box)
        self.prec = int(precision)
        self.flags = int(flags)
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        cfg, _keep = make_config(box, self.edges, lmax, precision, flags, grid_refine,
                                 workspace_limit)
        h = ctypes.c_void_p()
        rc = self.lib.tpcf_create(ctypes.byref(cfg), self.device,
                                  ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != TPCF_OK:
            raise TpcfError(rc, "tpcf_create failed")
        self.h = h

    def _chk(self, rc):
        if rc != TPCF_OK:
            raise TpcfError(rc, self.lib.tpcf_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpcf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- steps ---------------------------------------------------------
    def build_grid(self, pos, w=None, n_data=None):
        import torch
        _check_dev(pos, torch.float64, "pos")
        _check_dev(w, torch.float64, "w")
        n = pos.shape[0]
        self._keep = (pos, w)
        self._chk(self.lib.tpcf_build_grid(self.h, _ptr(pos), _ptr(w), n,
                                           n if n_data is None else int(n_data)))

    def autotune(self, pos, w=None, n_data=None, nmu=0):
        """Times every admissible grid refinement on the sample catalogue and keeps
        the fastest; returns (refinement, ms per refinement 1..4, -1 if not admissible)."""
        import torch
        _check_dev(pos, torch.float64, "pos")
        _check_dev(w, torch.float64, "w")
        n = pos.shape[0]
        k = ctypes.c_int32(0)
        ms = np.zeros(4)
        self._chk(self.lib.tpcf_autotune(self.h, _ptr(pos), _ptr(w), n, n if n_data is None else int(n_data),
                                         int(nmu), ctypes.byref(k), ctypes.c_void_p(ms.ctypes.data)))
        return int(k.value), ms

    def plan_key(self, sizes):
        """Key of a plan cache entry: the device's architecture, the handle's
        precision, flags, bins, lmax and box, and the sample's number of
        catalogues, mean size and mean density (points per r_max^3) in
        factor-of-two buckets."""
        import hashlib
        import math
        import torch
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        sizes = np.asarray(sizes, dtype=np.float64)
        mean = float(sizes.mean())
        dens = mean / self.box ** 3 * float(self.edges[-1]) ** 3
        eh = hashlib.sha1(self.edges.tobytes()).hexdigest()[:10]
        b = lambda x: int(round(math.log2(max(x, 1e-9))))
        return (f"{arch}|prec{self.prec}|flags{self.flags}|lmax{self.lmax}|nb{self.nbins}|edges{eh}|"
                f"box{self.box:g}|ncat2^{b(len(sizes))}|n2^{b(mean)}|nr3_2^{b(dens)}")

    def autotune_plan(self, pos, w=None, sizes=None, n_data=None, cache=None):
        """Chooses the launch plan (grid refinement, list mode, contraction
        step) by timing steps 1-3 of the sample (one catalogue, or a batch
        given by `sizes` as for run_catalogs), or takes it from the JSON plan
        cache at `cache` when it holds this key; returns the plan as a dict
        with the time of every candidate (ms, -1 where not run)."""
        import json
        import torch
        _check_dev(pos, torch.float64, "pos")
        _check_dev(w, torch.float64, "w")
        sizes = np.ascontiguousarray(np.asarray([pos.shape[0]] if sizes is None else sizes, dtype=np.int64))
        nd = np.ascontiguousarray(np.asarray(sizes if n_data is None else n_data, dtype=np.int64).reshape(-1))
        key = self.plan_key(sizes)
        entries = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                entries = json.load(f)
            if key in entries:
                e = entries[key]
                plan = Plan(int(e["grid_refine"]), int(e["list_mode"]), int(e["contract_step"]), 0, 0.0)
                self._chk(self.lib.tpcf_set_plan(self.h, ctypes.byref(plan)))
                return dict(e, cached=True)
        plan = Plan()
        ms = np.full(16, -1.0)
        self._chk(self.lib.tpcf_autotune_plan(self.h, sizes.shape[0], ctypes.c_void_p(sizes.ctypes.data),
                                              ctypes.c_void_p(nd.ctypes.data), _ptr(pos), _ptr(w),
                                              ctypes.byref(plan), ctypes.c_void_p(ms.ctypes.data)))
        out = plan.as_dict()
        out["candidates_ms"] = [round(float(v), 3) for v in ms]
        if cache:
            entries[key] = out
            tmp = cache + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(entries, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(out, cached=False)

    def set_plan(self, grid_refine=0, list_mode=-1, contract_step=0):
        plan = Plan(int(grid_refine), int(list_mode), int(contract_step), 0, 0.0)
        self._chk(self.lib.tpcf_set_plan(self.h, ctypes.byref(plan)))

    def get_plan(self):
        plan = Plan()
        self._chk(self.lib.tpcf_get_plan(self.h, ctypes.byref(plan)))
        return plan.as_dict()

    def alm_accumulate(self):
        self._chk(self.lib.tpcf_alm_accumulate(self.h))

    def get_alm(self, first, count):
        import torch
        s1 = self.lmax + 1
        out = torch.empty((count, self.nbins, s1, s1, 2), dtype=torch.float64,
                          device=f"cuda:{self.device}")
        self._chk(self.lib.tpcf_get_alm(self.h, int(first), int(count), _ptr(out)))
        return torch.view_as_complex(out)

    def contract(self, export=False):
        import torch
        out = None
        if export:
            s1 = self.lmax + 1
            out = torch.empty((s1, s1, s1, self.nbins, self.nbins), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        self._chk(self.lib.tpcf_contract(self.h, _ptr(out)))
        return out

    def multipoles(self, mults):
        import torch
        tr = np.ascontiguousarray(np.array(mults, dtype=np.int32).reshape(-1, 3))
        out = torch.empty((tr.shape[0], self.nbins, self.nbins), dtype=torch.float64,
                          device=f"cuda:{self.device}")
        self._chk(self.lib.tpcf_multipoles(self.h, tr.shape[0], ctypes.c_void_p(tr.ctypes.data),
                                           _ptr(out)))
        return out

    def run_catalogs(self, sizes, n_data, pos, w, mults, out=None):
        import torch
        _check_dev(pos, torch.float64, "pos")
        _check_dev(w, torch.float64, "w")
        sizes = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
        nd = np.ascontiguousarray(np.asarray(n_data, dtype=np.int64))
        tr = np.ascontiguousarray(np.array(mults, dtype=np.int32).reshape(-1, 3))
        ncat = sizes.shape[0]
        if out is None:
            out = torch.empty((ncat, tr.shape[0], self.nbins, self.nbins), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        self._chk(self.lib.tpcf_run_catalogs(self.h, ncat, ctypes.c_void_p(sizes.ctypes.data),
                                             ctypes.c_void_p(nd.ctypes.data), _ptr(pos), _ptr(w),
                                             tr.shape[0], ctypes.c_void_p(tr.ctypes.data),
                                             _ptr(out)))
        return out

    def catalog_status(self, ncat):
        """Per-catalogue status (int32, 0 = ok) of the last run_catalogs; a
        catalogue with non-finite positions has TPCF_ERR_DEVICE and NaN
        results while the others complete (run_catalogs itself raises)."""
        out = np.zeros(int(ncat), dtype=np.int32)
        self._chk(self.lib.tpcf_catalog_status(self.h, int(ncat), ctypes.c_void_p(out.ctypes.data)))
        return out

    # -- anisotropic 2PCF (Sec. 4.1) ----------------------------------
    def xi_count(self, nmu, out=None):
        """DD(r, mu) of the catalogue given to build_grid: int64 [nbins][nmu]."""
        import torch
        if out is None:
            out = torch.empty((self.nbins, int(nmu)), dtype=torch.int64, device=f"cuda:{self.device}")
        _check_dev(out, torch.int64, "out")
        self._chk(self.lib.tpcf_xi_count(self.h, int(nmu), _ptr(out)))
        return out

    def xi_multipoles(self, counts, n_data, ells):
        """xi_l(r_b) of the natural estimator from DD(r, mu): float64 [len(ells)][nbins]."""
        import torch
        _check_dev(counts, torch.int64, "counts")
        el = np.ascontiguousarray(np.array(ells, dtype=np.int32).reshape(-1))
        out = torch.empty((el.shape[0], self.nbins), dtype=torch.float64, device=f"cuda:{self.device}")
        self._chk(self.lib.tpcf_xi_multipoles(self.h, int(counts.shape[1]), _ptr(counts), int(n_data),
                                              el.shape[0], ctypes.c_void_p(el.ctypes.data), _ptr(out)))
        return out

    # -- Szapudi-Szalay estimator with explicit randoms -------------------
    def edge_correct_isotropic(self, N, R):
        """zeta_l(b1, b2) from the (l, l, 0) multipoles N of a data-minus-randoms
        run and R of a randoms run ([n_ell][nb][nb] float64 on the GPU)."""
        import torch
        _check_dev(N, torch.float64, "N")
        _check_dev(R, torch.float64, "R")
        if N.shape != R.shape or N.shape[1:] != (self.nbins, self.nbins):
            raise ValueError("N and R must both be [n_ell][nbins][nbins]")
        out = torch.empty_like(N)
        self._chk(self.lib.tpcf_edge_correct_isotropic(self.h, N.shape[0], _ptr(N), _ptr(R), _ptr(out)))
        return out

    def edge_correct(self, nnn_N, n_data_N, nnn_R, n_data_R, mults=None, want_zeta=False):
        """Anisotropic edge correction from the NNN^m exports of a data-minus-
        randoms run and of a randoms run ([m][l1][l2][b1][b2] float64 on the
        GPU, from contract(export=True)); returns (multipoles or None, zeta^m
        or None)."""
        import torch
        _check_dev(nnn_N, torch.float64, "nnn_N")
        _check_dev(nnn_R, torch.float64, "nnn_R")
        s1 = self.lmax + 1
        shape = (s1, s1, s1, self.nbins, self.nbins)
        if tuple(nnn_N.shape) != shape or tuple(nnn_R.shape) != shape:
            raise ValueError(f"the exports must be {shape}")
        out = zeta = None
        tr = None
        if mults is not None:
            tr = np.ascontiguousarray(np.array(mults, dtype=np.int32).reshape(-1, 3))
            out = torch.empty((tr.shape[0], self.nbins, self.nbins), dtype=torch.float64, device=nnn_N.device)
        if want_zeta:
            zeta = torch.empty(shape, dtype=torch.float64, device=nnn_N.device)
        self._chk(self.lib.tpcf_edge_correct(self.h, _ptr(nnn_N), int(n_data_N), _ptr(nnn_R), int(n_data_R),
                                             0 if tr is None else tr.shape[0],
                                             None if tr is None else ctypes.c_void_p(tr.ctypes.data),
                                             _ptr(out), _ptr(zeta)))
        return out, zeta

    # -- covariance over mock catalogues (Sec. 4.3) -----------------------
    def covariance(self, src, n_d=None, offsets=None):
        """Mean and covariance of the rows of src (n_mocks x stride, float64 on the
        GPU), over entries `offsets` (host int64) or the first n_d."""
        import torch
        _check_dev(src, torch.float64, "src")
        nm, stride = src.shape
        off = None if offsets is None else np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        nd = int(off.shape[0]) if off is not None else int(stride if n_d is None else n_d)
        mean = torch.empty(nd, dtype=torch.float64, device=src.device)
        cov = torch.empty((nd, nd), dtype=torch.float64, device=src.device)
        self._chk(self.lib.tpcf_covariance(self.h, nm, stride, _ptr(src), nd,
                                           None if off is None else ctypes.c_void_p(off.ctypes.data),
                                           _ptr(mean), _ptr(cov)))
        self._keep_off = off
        return mean, cov

    def covariance_noalloc(self, src, n_d=None, offsets=None, mean=None, cov=None):
        """covariance() through the allocation-free entry point: offsets (int64)
        and the outputs are device tensors given by the caller (allocated here
        only when not given)."""
        import torch
        _check_dev(src, torch.float64, "src")
        _check_dev(offsets, torch.int64, "offsets")
        nm, stride = src.shape
        nd = int(offsets.shape[0]) if offsets is not None else int(stride if n_d is None else n_d)
        if mean is None:
            mean = torch.empty(nd, dtype=torch.float64, device=src.device)
        if cov is None:
            cov = torch.empty((nd, nd), dtype=torch.float64, device=src.device)
        _check_dev(mean, torch.float64, "mean")
        _check_dev(cov, torch.float64, "cov")
        self._chk(self.lib.tpcf_covariance_noalloc(self.h, nm, stride, _ptr(src), nd, _ptr(offsets),
                                                   _ptr(mean), _ptr(cov)))
        return mean, cov

    def precision(self, cov, n_mocks, out=None):
        """Hartlap-corrected inverse of cov (eq. (Hartlap))."""
        import torch
        _check_dev(cov, torch.float64, "cov")
        if out is None:
            out = torch.empty_like(cov)
        self._chk(self.lib.tpcf_precision_matrix(self.h, cov.shape[0], _ptr(cov), int(n_mocks), _ptr(out)))
        return out

    def sync(self):
        self._chk(self.lib.tpcf_sync(self.h))

    def pair_count(self):
        v = ctypes.c_int64(0)
        self._chk(self.lib.tpcf_pair_count(self.h, ctypes.byref(v)))
        return int(v.value)

    def rebinned_count(self):
        v = ctypes.c_int64(0)
        self._chk(self.lib.tpcf_rebinned_count(self.h, ctypes.byref(v)))
        return int(v.value)

    def set_timing(self, enable=True):
        self._chk(self.lib.tpcf_set_timing(self.h, 1 if enable else 0))

    def stage_times(self):
        """Milliseconds and launches per stage: grid, binning, harmonics,
        contraction, finalisation, 2PCF counts."""
        ms = np.zeros(6)
        nl = np.zeros(6, dtype=np.int64)
        self._chk(self.lib.tpcf_stage_times(self.h, 6, ctypes.c_void_p(ms.ctypes.data),
                                            ctypes.c_void_p(nl.ctypes.data)))
        return ms, nl


def estimate(pos, box, edges, lmax, mults, w=None, n_data=None, precision=PREC_MIXED_BF16X3,
             flags=0, grid_refine=0):
    """One catalogue through the four steps; returns the multipoles tensor."""
    h = Handle(box, edges, lmax, precision=precision, flags=flags, grid_refine=grid_refine,
               device=pos.device.index or 0)
    h.build_grid(pos, w, n_data)
    h.alm_accumulate()
    h.contract()
    out = h.multipoles(mults)
    h.sync()
    h.close()
    return out


def triangle_index(edges, eta, r_min, rows):
    """Offsets of the 3PCF data vector in an n_mult x nbins x nbins block: for
    each multipole row, configurations r1 < r2 with r2 - r1 >= eta dr and
    r1 >= r_min (Sec. 4.3)."""
    lib = load()
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1))
    nb = edges.shape[0] - 1
    cnt = ctypes.c_int64(0)
    rc = lib.tpcf_triangle_index(nb, ctypes.c_void_p(edges.ctypes.data), float(eta), float(r_min), rows.shape[0],
                                 ctypes.c_void_p(rows.ctypes.data), 0, None, ctypes.byref(cnt))
    if rc != TPCF_OK:
        raise TpcfError(rc, "tpcf_triangle_index rejected its arguments")
    out = np.zeros(max(cnt.value, 1), dtype=np.int64)
    rc = lib.tpcf_triangle_index(nb, ctypes.c_void_p(edges.ctypes.data), float(eta), float(r_min), rows.shape[0],
                                 ctypes.c_void_p(rows.ctypes.data), out.shape[0], ctypes.c_void_p(out.ctypes.data),
                                 ctypes.byref(cnt))
    if rc != TPCF_OK:
        raise TpcfError(rc, "tpcf_triangle_index failed")
    return out[:cnt.value]


def percival_m1(n_mocks, n_d, n_params):
    """Percival factor m1 of eqs. (Perc1), (Perc)."""
    v = ctypes.c_double(0.0)
    rc = load().tpcf_percival_m1(int(n_mocks), int(n_d), int(n_params), ctypes.byref(v))
    if rc != TPCF_OK:
        raise TpcfError(rc, "tpcf_percival_m1 rejected its arguments")
    return v.value
