"""Benchmark of the anisotropic 3PCF estimator on one MI355X.

Workload (default): the batched covariance run -- 64 clustered catalogues
(Zel'dovich + RSD, sizes log-uniform in [5e4, 3e5], 1000 Mpc/h periodic boxes,
per-catalogue seeds), 10 radial bins over [20, 120] Mpc/h, lmax = 10, every
multipole with L <= 2, processed by one tpcf_run_catalogs call per step with
the positions already resident in HBM. The same step is timed for the mixed
path (FP32 pair pass + split-BF16 contraction) and for the plain FP64 path.

Prints ONE JSON line. `value` is pairs/s into a_lm(r) (ordered in-shell pairs
of all catalogues per step / seconds per step) for the mixed path.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

With --workload xi it times instead the anisotropic 2PCF of Sec. 4.1 on one
catalogue of the paper's halo density (7.2e5 clustered points, 1500 Mpc/h
box): DD(r, mu) in 30 x 5 Mpc/h radial bins and mu bins of 0.01, then the
Legendre multipoles l = 0, 2, 4; `value` is ordered pairs counted per second.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pairs/s into a_lm(r) + catalogs/hour, batched mixed vs plain FP64, 1 GPU"
PEAK_FP32_VALU = 157.3e12   # MI355X published FP32 vector peak (packed)
PEAK_BF16_MFMA = 2.5e15     # dense
PEAK_HBM = 8.0e12


def flop_per_pair(lmax: int) -> int:
    """Algorithmic FP32 work per in-shell pair of the harmonic pass:
    F(lmax) = 7 N_lm + 6 lmax + 40 with N_lm = (lmax+1)(lmax+2)/2 (three flops
    of recurrence, two of phase scaling and two of accumulation per
    coefficient, plus separation, normalisation, bin and powers)."""
    nlm = (lmax + 1) * (lmax + 2) // 2
    return 7 * nlm + 6 * lmax + 40


def contraction_flop(sizes, nb, lmax):
    """Dense MFMA work of the contraction, sum over catalogues and m of
    2 K_rows K_m^2 (K_rows = P for m = 0, 2P for m >= 1, K_m = nb (lmax-m+1))."""
    tot = 0.0
    for P in sizes:
        for m in range(lmax + 1):
            K = nb * (lmax - m + 1)
            tot += 2.0 * (P if m == 0 else 2 * P) * K * K
    return tot


def needed_contraction_flop(sizes, nb, lmax, Lmax):
    """The part of the dense contraction work that multipoles with L <= Lmax
    read: the (l1, l2, m) blocks with |l1 - l2| <= Lmax, each 2 K_rows nb^2."""
    per_p = 0.0
    for m in range(lmax + 1):
        rows = 1 if m == 0 else 2
        for l1 in range(m, lmax + 1):
            for l2 in range(m, lmax + 1):
                if abs(l1 - l2) <= Lmax:
                    per_p += 2.0 * rows * nb * nb
    return per_p * float(sum(int(p) for p in sizes))


def all_multipoles(lmax, Lmax):
    out = []
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for L in range(abs(l1 - l2), min(l1 + l2, Lmax) + 1):
                if (l1 + l2 + L) % 2 == 0:
                    out.append((l1, l2, L))
    return out


def make_batch(torch, ncat, lo, hi, box, sigma, f, grid, device):
    from paper_2408_03036_amd import catalogs as C
    sizes = C.log_uniform_sizes(ncat, lo, hi, C.BASE_SEED + 777)
    cats = [C.zeldovich_torch(int(n), box, sigma, f, C.catalogue_seed(i), grid=grid, device=device)
            for i, n in enumerate(sizes)]
    pos = torch.cat(cats, dim=0).contiguous()
    torch.cuda.synchronize()
    return sizes, pos


def tune(h, sizes, pos, w, n_data, args):
    """Launch plan for the handle, tuned on the whole batch (outside the timed
    steps), or read from --plan-cache; None with --no-tune or a fixed --refine."""
    if args.no_tune or args.refine:
        return None
    print(f"[bench] tuning the plan on the batch ({len(sizes)} catalogues)", file=sys.stderr, flush=True)
    return h.autotune_plan(pos, w, sizes=sizes, n_data=n_data, cache=args.plan_cache)


def time_steps(torch, h, sizes, pos, mults, steps, warmup):
    for _ in range(warmup):
        h.run_catalogs(sizes, sizes, pos, None, mults)
    h.sync()
    h.stage_times()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = h.run_catalogs(sizes, sizes, pos, None, mults)
    h.sync()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms, nl = h.stage_times()
    npairs = h.pair_count()
    return dt, ms, nl, npairs, out


def measured_traffic(kernel_sources):
    """HBM bytes per launch of the dominant kernel, from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes summarised in profiles/ (scaled by the copy-kernel
    calibration recorded there). None once the kernel's sources, or the host
    code that sizes its launches, differ from the ones the counters were taken
    on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_pair_alm_batched64_lmax10_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", kernel_sources):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def host_info():
    """The host the CPU baseline runs on: logical CPUs, CPUs this process may
    run on, the OpenMP thread setting and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except Exception:
        aff = None
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "cpu_model": model}


def oracle_threads():
    """Threads for the oracle: OMP_NUM_THREADS when it is set (the CPU share
    the host gives this job), else every CPU this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env), "OMP_NUM_THREADS"
    try:
        return len(os.sched_getaffinity(0)), "affinity"
    except Exception:
        return os.cpu_count() or 1, "cpu_count"


def _oracle_sample(O, pos_np, box, edges, lmax, nthr, target_s, w=None):
    """Times the oracle on the first primaries of a catalogue, sized for about
    target_s seconds; returns (pairs/s, primaries, pairs, seconds)."""
    n = pos_np.shape[0]
    probe = min(n, max(16, 16 * nthr))
    t0 = time.perf_counter()
    r = O.estimate(pos_np, box, edges, lmax, w=w, prim_first=0, prim_count=probe, nthreads=nthr)
    t1 = time.perf_counter() - t0
    rate = r.npairs / max(t1, 1e-9)
    per_prim = r.npairs / probe
    count = int(min(n, max(probe, target_s * rate / max(per_prim, 1.0))))
    t0 = time.perf_counter()
    r = O.estimate(pos_np, box, edges, lmax, w=w, prim_first=0, prim_count=count, nthreads=nthr)
    t1 = time.perf_counter() - t0
    return r.npairs / t1, count, r.npairs, t1


def executed_flop(kernel_sources):
    """FP32 FLOP the harmonic kernel executes per pair, from the
    SQ_INSTS_VALU_FLOPS_FP32 counter summarised in profiles/ (None once the
    sources differ from the ones it was taken on)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_pair_alm_batched64_lmax10_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if "executed_fp32_flop_per_pair" not in rec:
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", kernel_sources):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return {"per_pair": rec["executed_fp32_flop_per_pair"], "summary": rec.get("counters_summary")}


def build_info():
    """Identifies the build that ran: the git commit where the tree has one,
    and a hash of the library's sources (present on every copy of the tree)."""
    import hashlib
    import subprocess
    sha = None
    try:
        sha = subprocess.run(["git", "rev-parse", "--short=12", "HEAD"], cwd=ROOT, capture_output=True,
                             text=True, timeout=10).stdout.strip() or None
    except Exception:
        pass
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2408_03036_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return {"git_sha": sha, "csrc_sha256": h.hexdigest()[:16]}


def cpu_baseline(pos_np, box, edges, lmax, target_s=15.0, target_1t=5.0, w=None, what="catalogue 0"):
    """Times the FP64 CPU oracle (the full estimator including the NNN
    accumulation) on a bounded sample of primaries of one catalogue: with the
    host's threads, and with one thread for the per-core rate; pairs/s."""
    from oracle import oracle as O
    nthr, src = oracle_threads()
    rate, count, npairs, t1 = _oracle_sample(O, pos_np, box, edges, lmax, nthr, target_s, w)
    rate1, count1, npairs1, t11 = _oracle_sample(O, pos_np, box, edges, lmax, 1, target_1t, w)
    return {"value": rate, "unit": "pairs/s", "cores": nthr, "kind": "oracle",
            "sample": f"{count} primaries of {what} ({npairs} pairs, full estimator incl. "
                      f"NNN accumulation) in {t1:.1f} s on {nthr} threads ({src})",
            "value_1thread": rate1,
            "sample_1thread": f"{count1} primaries ({npairs1} pairs) in {t11:.1f} s on 1 thread",
            "host": host_info()}


# Algorithmic FP32 work per counted pair: separation (3), r^2 (5), r (1),
# radial bin (2), mu and its bin (3).
XI_FLOP_PER_PAIR = 14


def xi_cpu_baseline(pos_np, box, edges, nmu, target_s=15.0):
    """Times the CPU oracle's DD(r, mu) on a subsample of the catalogue (the
    points are in random order, so the first n are a uniform subsample),
    sized for about target_s seconds; pairs/s."""
    from oracle import oracle as O
    nthr, src = oracle_threads()
    n = min(pos_np.shape[0], 50_000)
    t0 = time.perf_counter()
    npairs = int(O.xi_counts(pos_np[:n], box, edges, nmu, nthreads=nthr).sum())
    t1 = time.perf_counter() - t0
    # pairs grow as n^2: pick n for about target_s seconds
    n2 = int(min(pos_np.shape[0], n * math.sqrt(max(target_s / max(t1, 1e-3), 1.0))))
    t0 = time.perf_counter()
    npairs = int(O.xi_counts(pos_np[:n2], box, edges, nmu, nthreads=nthr).sum())
    t1 = time.perf_counter() - t0
    return {"value": npairs / t1, "unit": "pairs/s", "cores": nthr, "kind": "oracle",
            "sample": f"DD(r, mu) of the first {n2} points of the catalogue ({npairs} pairs) in {t1:.1f} s "
                      f"on {nthr} threads ({src})",
            "host": host_info()}


def bench_xi(args):
    """The anisotropic 2PCF (Sec. 4.1): grid build, DD(r, mu) and multipoles per step."""
    import torch
    from paper_2408_03036_amd import catalogs as C
    from paper_2408_03036_amd import tpcf as T

    box, n, sigma, fgrowth = 1500.0, 720_000, 5.0, 0.8
    edges = np.linspace(0.0, 150.0, 31)
    nmu, ells = 200, [0, 2, 4]
    print("[bench] generating the 2PCF catalogue on the GPU", file=sys.stderr, flush=True)
    pos = C.zeldovich_torch(n, box, sigma, fgrowth, C.catalogue_seed(60), grid=256, device="cuda:0")
    torch.cuda.synchronize()
    h = T.Handle(box, edges, 0, precision=T.PREC_FP32, grid_refine=args.refine)
    h.set_timing(True)

    def step():
        h.build_grid(pos)
        dd = h.xi_count(nmu)
        return dd, h.xi_multipoles(dd, n, ells)

    print(f"[bench] 2PCF: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    h.sync()
    h.stage_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dd, xi = step()
    h.sync()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ms, nl = h.stage_times()
    h.close()
    npairs = int(dd.sum().item())
    t_cnt = ms[5] / max(nl[5], 1) / 1e3
    achieved = npairs * XI_FLOP_PER_PAIR / t_cnt
    roof = {"kernel": "k_xi_count (DD(r, mu) pair counts)", "bound": "alu",
            "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU, "traffic": None,
            "flop_per_pair": XI_FLOP_PER_PAIR, "avg_launch_ms": t_cnt * 1e3, "launches_per_step": nl[5] / args.steps}
    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = xi_cpu_baseline(pos.cpu().numpy(), box, edges, nmu)
    line = {
        "metric": "pairs/s into DD(r, mu) (anisotropic 2PCF, Sec. 4.1), 1 GPU",
        "value": npairs / dt, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"2PCF of one Zel'dovich+RSD catalogue: {n} points in a {box:.0f} Mpc/h box, "
                               f"30 radial bins [0,150] Mpc/h, {nmu} mu bins over [-1,1], l = 0, 2, 4",
                   "points": n, "pairs_per_step": npairs, "parallelism": "single GPU"},
        "stages_ms": {"grid_ms": ms[0] / args.steps, "xi_count_ms": ms[5] / args.steps,
                      "xi_multipoles_ms": ms[4] / args.steps},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def bench_ss(args):
    """Szapudi-Szalay estimator with explicit randoms at 50x (the paper's ratio):
    a data-minus-randoms run and a randoms run, then the edge correction, on
    1e4 clustered points with 5e5 randoms in a 400 Mpc/h box (the paper's halo
    density), 12 bins over [30, 150], l <= 4. By default the isotropic
    schedule and its correction; with --aniso the full anisotropic pass, the
    per-m sums of both runs and the tripolar correction of every multipole
    with L <= 2."""
    import torch
    from paper_2408_03036_amd import catalogs as C
    from paper_2408_03036_amd import tpcf as T

    box, nd = 400.0, 10_000
    nr = 50 * nd
    edges = np.linspace(30.0, 150.0, 13)
    lmax = 4
    iso = [(l, l, 0) for l in range(lmax + 1)]
    print("[bench] generating data and randoms on the GPU", file=sys.stderr, flush=True)
    D = C.zeldovich_torch(nd, box, 5.0, 0.8, C.catalogue_seed(90), grid=128, device="cuda:0")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(C.randoms_seed(90))
    Rp = (torch.rand((nr, 3), generator=g, device="cuda:0", dtype=torch.float64) * box).contiguous()
    pos = torch.cat([D, Rp], dim=0).contiguous()
    w = torch.from_numpy(C.dr_weights(nd, nr)).cuda()
    prec = {"bf16x3": T.PREC_MIXED_BF16X3, "bf16x6": T.PREC_MIXED_BF16X6, "fp32": T.PREC_FP32,
            "fp64": T.PREC_FP64}[args.precision]
    aniso = bool(getattr(args, "aniso", False))
    flags = 0 if aniso else T.F_ISOTROPIC
    mults = all_multipoles(lmax, 2) if aniso else iso

    def handles(p):
        # the neighbour lists of 1e5 randoms per primary need room: 200 GiB of the 288 GB
        return (T.Handle(box, edges, lmax, precision=p, flags=flags, workspace_limit=200 << 30),
                T.Handle(box, edges, lmax, precision=p, flags=flags, workspace_limit=200 << 30))

    def make_step(hN, hR):
        if not aniso:
            def step():
                Nm = hN.run_catalogs([nd + nr], [nd], pos, w, iso)
                Rm = hR.run_catalogs([nr], [nr], Rp, None, iso)
                return hN.edge_correct_isotropic(Nm[0], Rm[0])
            return step

        def step():
            # the per-m sums NNN^m of both runs, then the tripolar edge correction
            hN.build_grid(pos, w, nd)
            hN.alm_accumulate()
            nnnN = hN.contract(export=True)
            hR.build_grid(Rp, None, nr)
            hR.alm_accumulate()
            nnnR = hR.contract(export=True)
            return hN.edge_correct(nnnN, nd, nnnR, nr, mults)[0]
        return step

    hN, hR = handles(prec)
    plans = {"data_minus_randoms": tune(hN, np.array([nd + nr]), pos, w, [nd], args),
             "randoms": tune(hR, np.array([nr]), Rp, None, [nr], args)}
    hN.set_timing(True)
    hR.set_timing(True)
    step = make_step(hN, hR)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hN.stage_times()
    hR.stage_times()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        z = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    pairs = hN.pair_count() + hR.pair_count()
    msN, nlN = hN.stage_times()
    msR, nlR = hR.stage_times()
    hN.close()
    hR.close()
    t_alm = (msN[2] + msR[2]) / max(nlN[2] + nlR[2], 1) / 1e3
    launches = (nlN[2] + nlR[2]) / args.steps
    achieved = pairs * flop_per_pair(lmax) / launches / t_alm
    fp64 = None
    if not args.no_fp64 and prec != T.PREC_FP64:
        # the same step on the plain FP64 path: time and the accuracy of this precision
        print("[bench] ss fp64 comparison", file=sys.stderr, flush=True)
        hN, hR = handles(T.PREC_FP64)
        tune(hN, np.array([nd + nr]), pos, w, [nd], args)
        tune(hR, np.array([nr]), Rp, None, [nr], args)
        step64 = make_step(hN, hR)
        step64()  # the first step allocates the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z64 = step64()
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        hN.close()
        hR.close()
        fp64 = {"ms_per_step": dt64 * 1e3, "speedup_vs_fp64": dt64 / dt,
                "rel_err_vs_fp64_path": (z - z64).abs().max().item() / z64.abs().max().item()}
    line = {
        "metric": "pairs/s into a_lm(r), Szapudi-Szalay estimator with 50x explicit randoms, 1 GPU",
        "value": pairs / dt, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec != T.PREC_FP64 else "f64", "data": "synthetic",
        "config": {"workload": f"{nd} Zel'dovich+RSD points + {nr} randoms (50x), {box:.0f} Mpc/h box, 12 bins "
                               f"[30,150] Mpc/h, " + (f"anisotropic lmax {lmax}, {len(mults)} multipoles L <= 2, tripolar "
                               "edge correction" if aniso else f"isotropic l <= {lmax}, edge-corrected"),
                   "precision": args.precision, "pairs_per_step": int(pairs), "parallelism": "single GPU"},
        "stages_ms": {k: (msN[i] + msR[i]) / args.steps for i, k in
                      enumerate(["grid_ms", "pair_bin_ms", "pair_alm_ms", "contract_ms", "finalize_ms"])},
        "roofline": {"kernel": f"k_pair_alm<float,{lmax}> (harmonic pass)", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU, "traffic": None, "flop_per_pair": flop_per_pair(lmax),
                     "avg_launch_ms": t_alm * 1e3, "launches_per_step": launches},
        "fp64_path": fp64,
        "plan": plans,
        "cpu_baseline": None,
        "build": build_info(),
    }
    print(json.dumps(line))


def bench_c5(args):
    """Large batched sweep with randoms: catalogues of N_D ~ logU[1e5, 4e5]
    clustered points (Zel'dovich + RSD, sigma_Psi = 5, f = 0.8) each with 5 N_D
    uniform randoms in a 1500 Mpc/h box, weights 1 and -N_D/N_R (the
    data-minus-randoms numerator of eq. (ssest)), 12 bins over [10, 130],
    lmax 10, every multipole with L <= 4. The full sweep is 512 catalogues;
    a step times the first --ncat of them (16 by default) in one
    tpcf_run_catalogs call, and catalogues/hour of the sweep is extrapolated
    from it."""
    import torch
    from paper_2408_03036_amd import catalogs as C
    from paper_2408_03036_amd import tpcf as T

    box, sigma, fgrowth = 1500.0, 5.0, 0.8
    edges = np.linspace(10.0, 130.0, 13)
    lmax, Lmax = 10, 4
    mults = all_multipoles(lmax, Lmax)
    ncat_sweep = 512
    ncat = min(args.ncat if args.ncat != 64 else 16, ncat_sweep)
    nd_all = C.log_uniform_sizes(ncat_sweep, 100_000, 400_000, C.BASE_SEED + 555)
    nd = nd_all[:ncat]
    print(f"[bench] generating {ncat} of the {ncat_sweep} data + 5x randoms catalogues on the GPU",
          file=sys.stderr, flush=True)
    parts, wparts, sizes = [], [], []
    for i, n in enumerate(nd):
        D = C.zeldovich_torch(int(n), box, sigma, fgrowth, C.catalogue_seed(1000 + i), grid=256, device="cuda:0")
        g = torch.Generator(device="cuda:0")
        g.manual_seed(C.randoms_seed(1000 + i))
        R = torch.rand((5 * int(n), 3), generator=g, device="cuda:0", dtype=torch.float64) * box
        parts += [D, R]
        wparts.append(torch.from_numpy(C.dr_weights(int(n), 5 * int(n))).cuda())
        sizes.append(6 * int(n))
    pos = torch.cat(parts, dim=0).contiguous()
    w = torch.cat(wparts, dim=0).contiguous()
    del parts, wparts
    sizes = np.array(sizes, dtype=np.int64)
    torch.cuda.synchronize()
    prec_id = {"bf16x3": T.PREC_MIXED_BF16X3, "bf16x6": T.PREC_MIXED_BF16X6,
               "fp32": T.PREC_FP32, "fp64": T.PREC_FP64}[args.precision]

    plans = {}

    def run(prec, steps, warmup):
        # 240 GiB of the 288 GB (one handle at a time): fewer, larger chunks
        h = T.Handle(box, edges, lmax, precision=prec, grid_refine=args.refine, workspace_limit=240 << 30)
        plans[prec] = tune(h, sizes, pos, w, nd, args)
        h.set_timing(True)
        for _ in range(warmup):
            h.run_catalogs(sizes, nd, pos, w, mults)
        h.sync()
        h.stage_times()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = h.run_catalogs(sizes, nd, pos, w, mults)
        h.sync()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ms, nl = h.stage_times()
        npairs = h.pair_count()
        h.close()
        return dt, ms, nl, npairs, out

    print(f"[bench] c5 {args.precision}: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    dt, ms, nl, npairs, out = run(prec_id, args.steps, args.warmup)
    t_alm = ms[2] / max(nl[2], 1) / 1e3
    launches = nl[2] / args.steps
    achieved = npairs / launches * flop_per_pair(lmax) / t_alm
    t_pair = (ms[1] + ms[2]) / args.steps / 1e3
    roof = {"kernel": "k_pair_alm<float,10> (harmonic pass)", "bound": "alu",
            "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU, "traffic": None, "flop_per_pair": flop_per_pair(lmax),
            "avg_launch_ms": t_alm * 1e3, "launches_per_step": launches,
            "pair_pass_frac": npairs * flop_per_pair(lmax) / t_pair / PEAK_FP32_VALU if t_pair > 0 else None}
    stages = {k: ms[i] / args.steps for i, k in
              enumerate(["grid_ms", "pair_bin_ms", "pair_alm_ms", "contract_ms", "finalize_ms"])}
    fp64 = None
    if not args.no_fp64 and prec_id != T.PREC_FP64:
        print("[bench] c5 fp64 comparison", file=sys.stderr, flush=True)
        dt64, ms64, nl64, np64, out64 = run(T.PREC_FP64, 1, 0)
        err = (out - out64).abs().max().item() / out64.abs().max().item()
        fp64 = {"value": np64 / dt64, "unit": "pairs/s", "ms_per_step": dt64 * 1e3,
                "catalogs_per_hour": ncat * 3600.0 / dt64, "speedup_mixed_vs_fp64": dt64 / dt,
                "mixed_rel_err_vs_fp64_path": err, "pairs_equal": int(np64) == int(npairs),
                "plan": plans.get(T.PREC_FP64)}
    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        n0 = int(sizes[0])
        cpu = cpu_baseline(pos[:n0].cpu().numpy(), box, edges, lmax, w=w[:n0].cpu().numpy(),
                           what="catalogue 0 (data + 5x randoms)")
    # weights make the split-BF16 request run the six-product split
    eff = {"bf16x3": "bf16x6"}.get(args.precision, args.precision)
    line = {
        "metric": METRIC, "value": npairs / dt, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec_id != T.PREC_FP64 else "f64", "data": "synthetic",
        "config": {"workload": f"large batched sweep with randoms: {ncat} of {ncat_sweep} catalogues timed "
                               f"(N_D log-uniform [1e5,4e5] Zel'dovich+RSD + 5 N_D randoms, weights 1 and "
                               f"-N_D/N_R), 1500 Mpc/h boxes, 12 bins [10,130] Mpc/h, lmax 10, L<=4 "
                               f"({len(mults)} multipoles)",
                   "precision": args.precision, "precision_effective": eff, "ncat": int(ncat),
                   "points": int(sizes.sum()), "pairs_per_step": int(npairs), "parallelism": "single GPU"},
        "catalogs_per_hour": ncat * 3600.0 / dt,
        "sweep_hours_extrapolated": ncat_sweep / (ncat * 3600.0 / dt),
        "plan": plans.get(prec_id),
        "stages_ms": stages,
        "roofline": roof,
        "fp64_path": fp64,
        "cpu_baseline": cpu,
        "build": build_info(),
    }
    print(json.dumps(line))


def bench_cov(args):
    """Covariance step of Sec. 4.3 at the paper's size: 3000 mock data vectors of
    336 entries (the joint 2PCF + 3PCF vector of its covariance figure), taken
    by offset from rows of 400 values; covariance, then Hartlap precision."""
    import torch
    from paper_2408_03036_amd import tpcf as T

    nm, stride, nd = 3000, 400, 336
    g = torch.Generator(device="cuda:0")
    g.manual_seed(2408030360)
    # correlated Gaussian mock vectors (stand-ins for the measured multipoles)
    Lmix = torch.randn((stride, stride), generator=g, device="cuda:0", dtype=torch.float64) * 0.05
    Lmix += torch.eye(stride, device="cuda:0", dtype=torch.float64)
    src = (torch.randn((nm, stride), generator=g, device="cuda:0", dtype=torch.float64) @ Lmix.T).contiguous()
    off = np.sort(np.random.default_rng(2408030360).choice(stride, nd, replace=False)).astype(np.int64)
    torch.cuda.synchronize()
    h = T.Handle(100.0, np.linspace(0.0, 10.0, 2), 0)
    stream = torch.cuda.current_stream()

    def step():
        mean, cov = h.covariance(src, offsets=off)
        return cov, h.precision(cov, nm)

    for _ in range(args.warmup):
        step()
    h.sync()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_cov = t_inv = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev[0].record(stream)
        mean, cov = h.covariance(src, offsets=off)
        ev[1].record(stream)
        prec = h.precision(cov, nm)
        ev[2].record(stream)
        torch.cuda.synchronize()
        t_cov += ev[0].elapsed_time(ev[1])
        t_inv += ev[1].elapsed_time(ev[2])
    dt = (time.perf_counter() - t0) / args.steps
    h.close()
    t_cov /= args.steps
    t_inv /= args.steps
    # FP64 work: the covariance product (upper triangle, 2 flop per product) and the
    # Gauss-Jordan sweep (2 n^3)
    f_cov = float(nm) * nd * (nd + 1)
    f_inv = 2.0 * nd ** 3
    roof = {"kernel": "k_cov_syrk + k_cov_invert (FP64)", "bound": "mfma",
            "achieved": (f_cov + f_inv) / ((t_cov + t_inv) / 1e3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
            "frac": (f_cov + f_inv) / ((t_cov + t_inv) / 1e3) / 78.6e12, "traffic": None,
            "covariance_ms": t_cov, "precision_ms": t_inv}
    cpu = None
    if not args.no_cpu:
        from oracle import cov_oracle as V
        sub = src[:200].cpu().numpy()[:, off]
        t0 = time.perf_counter()
        V.covariance(sub)
        t1 = time.perf_counter() - t0
        cpu = {"value": 200 / t1, "unit": "data vectors/s", "cores": 1, "kind": "oracle",
               "sample": f"covariance loops of the oracle over the first 200 mocks ({nd} entries) in {t1:.1f} s"}
    line = {
        "metric": "mock data vectors/s into covariance + Hartlap precision (Sec. 4.3), 1 GPU",
        "value": nm / dt, "unit": "data vectors/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"covariance of {nm} mock data vectors of {nd} entries (offsets into rows of "
                               f"{stride}), Hartlap-corrected precision matrix",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ncat", type=int, default=64)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "bf16x6", "fp32", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--refine", type=int, default=0, help="fixed grid refinement (no plan tuning)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch plan")
    ap.add_argument("--plan-cache", default=None, help="JSON plan cache to read and extend")
    ap.add_argument("--aniso", action="store_true",
                    help="with --workload ss: the anisotropic pass and the tripolar edge correction")
    ap.add_argument("--workload", default="3pcf", choices=["3pcf", "xi", "cov", "ss", "c5"],
                    help="3pcf: the batched 3PCF run (default); xi: the anisotropic 2PCF; "
                         "c5: data + 5x randoms catalogues of the large sweep (a timed subset); "
                         "cov: covariance and precision over mock data vectors; "
                         "ss: Szapudi-Szalay estimator with 50x explicit randoms, edge-corrected")
    ap.add_argument("--isotropic", action="store_true",
                    help="3pcf: the isotropic schedule, multipoles (l, l, 0) only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the catalogue batch would be split across GPUs by whole catalogues).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "xi":
        bench_xi(args)
        return
    if args.workload == "cov":
        bench_cov(args)
        return
    if args.workload == "ss":
        bench_ss(args)
        return
    if args.workload == "c5":
        bench_c5(args)
        return

    import torch
    from paper_2408_03036_amd import tpcf as T

    dev = "cuda:0"
    box, sigma, fgrowth, grid = 1000.0, 6.0, 0.8, 256
    edges = np.linspace(20.0, 120.0, 11)
    lmax, Lmax = 10, 2
    mults = all_multipoles(lmax, Lmax)
    flags = 0
    if args.isotropic:
        mults = [(l, l, 0) for l in range(lmax + 1)]
        flags = T.F_ISOTROPIC
    print(f"[bench] generating {args.ncat} catalogues on the GPU", file=sys.stderr, flush=True)
    sizes, pos = make_batch(torch, args.ncat, 50_000, 300_000, box, sigma, fgrowth, grid, dev)
    ntot = int(sizes.sum())
    prec_id = {"bf16x3": T.PREC_MIXED_BF16X3, "bf16x6": T.PREC_MIXED_BF16X6,
               "fp32": T.PREC_FP32, "fp64": T.PREC_FP64}[args.precision]

    print(f"[bench] {args.precision}: {args.warmup} warmup + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    # 200 GiB of the 288 GB: two chunks of about 4.5M primaries with their hit lists
    h = T.Handle(box, edges, lmax, precision=prec_id, flags=flags, grid_refine=args.refine,
                 workspace_limit=200 << 30)
    plan = tune(h, sizes, pos, None, sizes, args)
    h.set_timing(True)
    rebinned0 = h.rebinned_count()  # the tuner's passes are not counted
    dt, ms, nl, npairs, out = time_steps(torch, h, sizes, pos, mults, args.steps, args.warmup)
    rebinned = (h.rebinned_count() - rebinned0) / max(args.steps + args.warmup, 1)
    h.close()
    value = npairs / dt
    cats_per_hour = args.ncat * 3600.0 / dt

    # dominant kernel: the harmonic pass (stage 2)
    t_alm = ms[2] / max(nl[2], 1) / 1e3
    launches_per_step = nl[2] / args.steps
    flop_launch = npairs * flop_per_pair(lmax) / launches_per_step
    achieved = flop_launch / t_alm
    traffic = None
    if args.ncat == 64 and prec_id != T.PREC_FP64:
        traffic = measured_traffic(["paper_2408_03036_amd/csrc/tpcf_pairs.hip",
                                    "paper_2408_03036_amd/csrc/tpcf_internal.h",
                                    "paper_2408_03036_amd/csrc/tpcf.cpp"])
    roof = {"kernel": "k_pair_alm<float,10> (harmonic pass)", "bound": "alu",
            "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU, "traffic": traffic,
            "flop_per_pair": flop_per_pair(lmax), "avg_launch_ms": t_alm * 1e3,
            "launches_per_step": launches_per_step}
    # the whole pair pass (binning + harmonics), algorithmic F(lmax) per pair
    t_pair = (ms[1] + ms[2]) / args.steps / 1e3
    if t_pair > 0:
        roof["pair_pass_frac"] = npairs * flop_per_pair(lmax) / t_pair / PEAK_FP32_VALU
        roof["pair_pass_ms"] = t_pair * 1e3
    if args.ncat == 64 and prec_id != T.PREC_FP64 and not args.isotropic:
        ex = executed_flop(["paper_2408_03036_amd/csrc/tpcf_pairs.hip",
                            "paper_2408_03036_amd/csrc/tpcf_internal.h",
                            "paper_2408_03036_amd/csrc/tpcf.cpp"])
        if ex is not None:
            roof["executed_flop_per_pair"] = ex["per_pair"]
            roof["executed_frac"] = npairs / launches_per_step * ex["per_pair"] / t_alm / PEAK_FP32_VALU
            roof["executed_source"] = ex["summary"]
    stages = {"grid_ms": ms[0] / args.steps, "pair_bin_ms": ms[1] / args.steps,
              "pair_alm_ms": ms[2] / args.steps, "contract_ms": ms[3] / args.steps,
              "finalize_ms": ms[4] / args.steps}
    cflop = contraction_flop(sizes, len(edges) - 1, lmax)
    mfma_mult = {T.PREC_MIXED_BF16X3: 3, T.PREC_MIXED_BF16X6: 6}.get(prec_id, 1)
    contraction = {"dense_flop": cflop, "ms": stages["contract_ms"],
                   "tflops_fp32_equiv": cflop / (stages["contract_ms"] / 1e3) / 1e12
                   if stages["contract_ms"] > 0 else None,
                   "mfma_products_per_fp32_product": mfma_mult}
    nflop = needed_contraction_flop(sizes, len(edges) - 1, lmax, Lmax)
    contraction["needed_flop"] = nflop
    if prec_id in (T.PREC_MIXED_BF16X3, T.PREC_MIXED_BF16X6) and stages["contract_ms"] > 0:
        contraction["frac_bf16_peak"] = cflop * mfma_mult / (stages["contract_ms"] / 1e3) / PEAK_BF16_MFMA
        contraction["needed_frac_bf16_peak"] = nflop * mfma_mult / (stages["contract_ms"] / 1e3) / PEAK_BF16_MFMA
    if args.isotropic:
        # only the l1 = l2 blocks, on FP64 MFMA: sum over catalogues, (l, m) and parts of 2 P nb^2
        nb = len(edges) - 1
        iflop = sum(2.0 * nb * nb * float(P) * (1 if m == 0 else 2)
                    for P in sizes for m in range(lmax + 1) for _ in range(m, lmax + 1))
        contraction = {"schedule": "isotropic (l1 = l2 blocks, FP64 MFMA)", "flop": iflop,
                       "ms": stages["contract_ms"],
                       "frac_fp64_mfma_peak": iflop / (stages["contract_ms"] / 1e3) / 78.6e12
                       if stages["contract_ms"] > 0 else None}

    fp64 = None
    if not args.no_fp64 and prec_id != T.PREC_FP64:
        print("[bench] fp64 comparison", file=sys.stderr, flush=True)
        h = T.Handle(box, edges, lmax, precision=T.PREC_FP64, flags=flags, grid_refine=args.refine,
                     workspace_limit=96 << 30)
        plan64 = tune(h, sizes, pos, None, sizes, args)
        h.set_timing(True)
        dt64, ms64, nl64, np64, out64 = time_steps(torch, h, sizes, pos, mults, max(2, args.steps // 2), 1)
        h.close()
        ref = out64.abs().max().item()
        err = (out - out64).abs().max().item() / ref
        fp64 = {"value": np64 / dt64, "unit": "pairs/s", "ms_per_step": dt64 * 1e3,
                "catalogs_per_hour": args.ncat * 3600.0 / dt64,
                "pair_alm_ms": ms64[2] / max(2, args.steps // 2),
                "contract_ms": ms64[3] / max(2, args.steps // 2),
                "speedup_mixed_vs_fp64": dt64 / dt,
                "mixed_rel_err_vs_fp64_path": err, "pairs_equal": int(np64) == int(npairs), "plan": plan64}

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        n0 = int(sizes[0])
        cpu = cpu_baseline(pos[:n0].cpu().numpy(), box, edges, lmax)

    line = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec_id != T.PREC_FP64 else "f64",
        "data": "synthetic",
        "config": {"workload": f"batched covariance run: {args.ncat} Zel'dovich+RSD catalogues, "
                               f"sizes log-uniform [5e4,3e5] ({ntot} points), 1000 Mpc/h boxes, "
                               f"10 bins [20,120] Mpc/h, lmax 10, "
                               + (f"isotropic schedule ({len(mults)} multipoles (l,l,0))" if args.isotropic
                                  else f"L<=2 ({len(mults)} multipoles)"),
                   "precision": args.precision, "ncat": args.ncat, "points": ntot,
                   "pairs_per_step": int(npairs), "parallelism": "single GPU"},
        "catalogs_per_hour": cats_per_hour,
        "plan": plan,
        "stages_ms": stages,
        "rebinned_primaries_per_step": rebinned,
        "roofline": roof,
        "contraction": contraction,
        "fp64_path": fp64,
        "cpu_baseline": cpu,
        "build": build_info(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
