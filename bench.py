"""Benchmark of the FC grid-scan hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c5] [--form fp64]
                    [--legs fp32,split_bf16,split_fp16] [--serving-requests R]

Default workload (c5): D = 5 grid 16^5 (G = 1 048 576 points), N = 57 bins, 16
true points x 10 000 universes (160 000 universes, 1.68e11 universe x
grid-point chi^2 evaluations per step), scanned in FP64 (the paper's
arithmetic), with 0.6827 / 0.90 / 0.95 critical values and a 200-bin
histogram per true point.  The other workloads: c1 (D = 2 20 x 20, N = 38,
one true point x 1000 universes), c2 (D = 2 100 x 100, N = 57, 256 x 2000)
and c3 (D = 3 60^3, N = 57, 64 x 4000).  Inputs are seeded synthetic data from
the toy oscillation model, resident in HBM before the timed region.

One step = covariance factors for every grid point (FP64 Cholesky + inverse,
stored in the scan form) + the scan of all universes (minimum, argmin,
Delta chi^2) + critical values.  The dominant kernel is also timed alone
(HIP events around its launches, on its stream).  Legs on the same inputs: the
FP32 and split BF16 / FP16 forms (scan time, roofline, error against the FP64
result on every universe and against the oracle on a sample).  Further legs:
the one-matrix scan (Algorithm 1 as printed, and its iteration) and the
full-surface region on the c2 grid, and a serving leg that replays a seeded
Poisson stream of FC requests (K log-uniform in [500, 20000], three resident
grids) through a plain FIFO loop and through the continuous-batching server,
with p50/p99 latency beside throughput.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("universe×gridpoint χ² evals/s at max|Δχ²| err vs FP64; "
          "FC request p50/p99 latency")
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "split_bf16": 2500e12, "split_fp16": 2500e12}
DTYPE = {"fp32": "f32", "fp64": "f64", "split_bf16": "bf16x2+f32acc", "split_fp16": "f16x2+f32acc"}
TOL = {"fp32": 1e-6, "fp64": 1e-11, "split_bf16": 1e-4, "split_fp16": 1e-4}
ALPHA = (0.6827, 0.9, 0.95)
N_BINS, HIST_HI = 200, 50.0


def flop_per_eval(N: int) -> int:
    # the method's work per evaluation in factor form: N subtractions, the
    # triangular W r (N(N+1)/2 multiply-adds), N squares and N adds
    return N * N + 4 * N


def mfma_flop_per_eval(N: int) -> int:
    # the part of it on the matrix cores: the triangular W r
    return N * (N + 1)


def vector_flop_per_eval(N: int, form: str, scan: str) -> int:
    # the rest, on the vector ALUs: the residual's N subtractions (not in the
    # FP32 grouped form, whose residual is formed once per universe) and the
    # N squares and adds
    return (2 * N if (form == "fp32" and scan == "points") else 3 * N)


def split_flop_per_eval(N: int) -> int:
    # split forms: three 16-bit products (hi*hi, hi*lo, lo*hi) per multiply-add
    # of the triangular W r, on the 16-bit matrix cores
    return 3 * N * (N + 1)


KERNEL = {"fp64": "k_scan_f64m", "fp32": "k_scan_fp32_pts", "split_bf16": "k_scan_split",
          "split_fp16": "k_scan_split"}


WORKLOADS = {
    "c1": dict(desc="c1: D=2 grid 20x20 (G=400), N=38, 1 true point x 1000 universes",
               steps=10, warmup=2, cpu_per_point=1000, serving=0),
    "c2": dict(desc="c2: D=2 grid 100x100 (G=10000), N=57, 256 true points x 2000 universes",
               steps=5, warmup=1, cpu_per_point=100, serving=200),
    "c3": dict(desc="c3: D=3 grid 60^3 (G=216000), N=57, 64 true points x 4000 universes",
               steps=3, warmup=1, cpu_per_point=8, serving=0),
    "c5": dict(desc="c5: D=5 grid 16^5 (G=1048576), N=57, 16 true points x 10000 universes",
               steps=3, warmup=1, cpu_per_point=16, serving=200),
}

# HBM traffic of the scan kernel per launch, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by the same counters over a copy of known size
# (the profiles directory holds the summaries).  Valid only while the kernel's
# sources hash to the value the counters were taken with.
FP32_SOURCES = ("paper_2002_07858_amd/csrc/k_scan.hip", "paper_2002_07858_amd/csrc/fc_internal.h")
SPLIT_SOURCES = ("paper_2002_07858_amd/csrc/k_scan_split.hip",
                 "paper_2002_07858_amd/csrc/fc_internal.h")
FP64_SOURCES = ("paper_2002_07858_amd/csrc/k_scan64.hip",
                "paper_2002_07858_amd/csrc/fc_internal.h")
# FETCH_SIZE (KiB x 1024 x 2.0000) + WRITE_SIZE (KiB x 1024 x 1.0000) of one launch
# (a leg's: mean of the three launches of one run)
TRAFFIC = {
    ("c5", "fp64", "points"): {"bytes_per_launch": 985414308 * 2048 + 1281250 * 1024,
                               "source_hash": "7c799a98aa98fe16", "sources": FP64_SOURCES,
                               "profile": "profiles/k_scan_f64m_c5.md"},
    ("c5", "fp32", "points"): {"bytes_per_launch": 227249134 * 2048 + 641250 * 1024,
                               "source_hash": "37a4a054150dd848", "sources": FP32_SOURCES,
                               "profile": "profiles/k_scan_c5_fp32_split_counters.md"},
    ("c5", "split_fp16", "points"): {"bytes_per_launch": 2194617926 * 2048 + 2561250 * 1024,
                                     "source_hash": "98549ac6fbe21dfe", "sources": SPLIT_SOURCES,
                                     "profile": "profiles/k_scan_c5_fp32_split_counters.md"},
    ("c5", "split_bf16", "points"): {"bytes_per_launch": 568374400 * 2048 + 6721251 * 1024,
                                     "source_hash": "98549ac6fbe21dfe", "sources": SPLIT_SOURCES,
                                     "profile": "profiles/k_scan_c5_fp32_split_counters.md"},
}


def kernel_source_hash(sources) -> str:
    """Hash of a kernel's sources with // comments and blank lines removed (a
    comment edit does not invalidate the counters; any code edit does)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def copy_probe(mib: int):
    """A plain device-to-device copy of known size, for counter calibration."""
    import torch
    n = (mib << 20) // 4
    x = torch.arange(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    assert bool((y[-16:] == x[-16:]).all())
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "launches": 3}))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads():
    """Threads for the oracle: the CPUs this process may run on, capped by the
    host share the environment grants (OMP_NUM_THREADS when set)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    share = int(env) if env.isdigit() and int(env) > 0 else n
    return max(1, min(n, share)), n


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(pr, per_point: int, dev_out: dict, tol: float):
    """Time the FP64 oracle on a bounded sample and measure the device error on it."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import parity
    idx, seg = [], [0]
    for s in range(len(pr.seg_off) - 1):
        lo, hi = int(pr.seg_off[s]), int(pr.seg_off[s + 1])
        idx += list(range(lo, min(hi, lo + per_point)))
        seg.append(len(idx))
    idx = np.array(idx)
    nt, visible = host_threads()
    t0 = time.perf_counter()
    ref = oracle.scan(pr.S, pr.F, pr.d[idx], pr.p_idx[idx], nthreads=nt)
    dt = time.perf_counter() - t0
    evals = len(idx) * pr.G
    rep = parity.report({k: v[idx] for k, v in dev_out.items()}, ref, tol)
    # critical values of the sampled universes, device values vs oracle values
    c_dev, _ = oracle.critical_value(dev_out["dchi2"][idx], seg, ALPHA, with_hist=False)
    c_ref, _ = oracle.critical_value(ref["dchi2"], seg, ALPHA, with_hist=False)
    rep["crit_abs_err_sample"] = float(np.abs(c_dev - c_ref).max())
    rep["_sample"] = (idx, ref)   # reused by the form legs, removed before printing
    base = {"value": evals / dt, "unit": "evals/s", "cores": nt, "kind": "oracle",
            "cpu_model": cpu_model(), "cpus_visible": visible,
            "sample": f"first {min(per_point, int(pr.seg_off[1]))} universes of each of the "
                      f"{len(pr.seg_off) - 1} true points x all {pr.G} grid points "
                      f"({evals:.3g} evals, {dt:.1f} s on {nt} threads, FP64 Cholesky per grid "
                      f"point + forward substitution)"}
    return base, rep


# ---------------------------------------------------------------------------
# Serving: FC requests against the three resident grids (D=2 20x20 N=38,
# D=2 100x100 N=57, D=3 60^3 N=57), Poisson arrivals, K log-uniform in
# [500, 20000]; plain = one request at a time through fc_scan (FIFO),
# batched = the continuous-batching server, in FP32 and split FP16.
# ---------------------------------------------------------------------------
def serving_requests(grids, n_req, seed=3):
    import math
    import fcgen
    rng = fcgen.rng_for(4, 3, seed)
    reqs = []
    for j in range(n_req):
        gi = int(rng.integers(0, len(grids)))
        pr = grids[gi][0]
        p = int(rng.integers(0, pr.G))
        K = int(math.floor(math.exp(rng.uniform(math.log(500), math.log(20000)))))
        d = fcgen.universes(4, j, pr.S[p], pr.F, K)
        reqs.append((gi, p, d))
    return reqs


def run_plain(fc, grids, reqs, arrivals):
    """FIFO, one request at a time: upload, fc_scan, fc_critical_value, copy back."""
    import torch
    lat, evals = [], 0.0
    t0 = time.perf_counter()
    for (gi, p, d), ta in zip(reqs, arrivals):
        now = time.perf_counter() - t0
        if now < ta:
            time.sleep(ta - now)
        g = grids[gi][1]
        K = d.shape[0]
        d_t = torch.as_tensor(d).cuda()
        p_t = torch.full((K,), p, dtype=torch.int64, device="cuda")
        o = [torch.empty(K, dtype=torch.float64, device="cuda") for _ in range(3)]
        am = torch.empty(K, dtype=torch.int64, device="cuda")
        fc.fc_scan(g, fc.FC_FORM_FP32, d_t, p_t, o[0], o[1], am, o[2])
        seg = torch.tensor([0, K], dtype=torch.int64, device="cuda")
        crit = torch.empty((1, len(ALPHA)), dtype=torch.float64, device="cuda")
        hist = torch.empty((1, N_BINS + 1), dtype=torch.int64, device="cuda")
        fc.fc_critical_value(seg, o[0], ALPHA, crit, N_BINS, HIST_HI, hist)
        o[0].cpu(), crit.cpu(), hist.cpu()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - ta)
        evals += K * grids[gi][0].G
    wall = time.perf_counter() - t0
    return lat, wall, evals


def run_batched(fc, grids, reqs, arrivals, form, policy):
    import threading
    server = fc.Server([g for _, g in grids], form=form, hbm_budget=16 << 30,
                       host_budget=4 << 30, alpha=ALPHA, n_bins=N_BINS, hist_hi=HIST_HI,
                       policy=policy)
    ids = [None] * len(reqs)
    t0 = time.perf_counter()

    def submitter():
        for k, ((gi, p, d), ta) in enumerate(zip(reqs, arrivals)):
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            ids[k] = server.submit(gi, p, d)

    th = threading.Thread(target=submitter)
    th.start()
    lat = {}
    hbm_peak, t_stat = 0, 0.0
    while len(lat) < len(reqs):
        if time.perf_counter() - t_stat > 0.01:   # request data resident in HBM
            hbm_peak = max(hbm_peak, server.stats()["hbm_in_use"])
            t_stat = time.perf_counter()
        for k, i in enumerate(ids):
            if i is None or k in lat:
                continue
            st, r = server.poll(i)
            if st == fc.FC_REQ_FAILED:
                raise RuntimeError("served request failed")
            if r is not None:
                lat[k] = r["latency"]
        time.sleep(0.0005)
        if time.perf_counter() - t0 > 600:
            raise RuntimeError("serving run did not finish")
    th.join()
    wall = time.perf_counter() - t0
    st = server.stats()
    server.destroy()
    return [lat[k] for k in range(len(reqs))], wall, st["evals"], st["launches"], hbm_peak


GRID_NAMES = ("20x20 N=38", "100x100 N=57", "60^3 N=57")


def summarize(lat, wall, evals, n, grid_of=None):
    a = np.asarray(lat) * 1e3
    out = {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
           "mean_ms": float(a.mean()), "throughput_req_s": n / wall,
           "evals_per_s": evals / wall}
    if grid_of is not None:  # latency per grid class
        gi = np.asarray(grid_of)
        out["per_grid"] = {GRID_NAMES[k]: {"n": int((gi == k).sum()),
                                           "p50_ms": float(np.percentile(a[gi == k], 50)),
                                           "p99_ms": float(np.percentile(a[gi == k], 99))}
                           for k in range(len(GRID_NAMES)) if (gi == k).any()}
    return out


def serving_bench(n_req: int, loads=(0.8,)):
    import fcgen
    import paper_2002_07858_amd as fc
    grids = []
    for name in ("c1", "c2", "c3"):
        pr = fcgen.make_problem(name, K=1, true_subset=[0])
        g = fc.fc_build_grid(pr.axes, pr.S)
        fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32 | fc.FC_FORM_SPLIT_FP16)
        grids.append((pr, g))
    log(f"[bench] serving: generating {n_req} requests")
    reqs = serving_requests(grids, n_req)
    # plain capacity: the first 40 requests back to back
    n_cap = min(40, n_req)
    lat, wall, _ = run_plain(fc, grids, reqs[:n_cap], [0.0] * n_cap)
    capacity = n_cap / wall
    out = {"requests": n_req, "grids": list(GRID_NAMES),
           "grid_hbm_bytes": [int(fc.fc_grid_device_bytes(g)) for _, g in grids],
           "K": "log-uniform [500, 20000]", "plain_capacity_req_s": capacity, "loads": {}}
    rng = fcgen.rng_for(4, 3, 1)
    gaps = rng.exponential(1.0, size=n_req)
    for load in loads:
        if load == "sat":
            # every request queued at once: throughput is each mode's capacity
            lam = float("inf")
            arrivals = np.zeros(n_req)
        else:
            lam = float(load) * capacity
            arrivals = np.cumsum(gaps / lam) - gaps[0] / lam
        log(f"[bench] serving load {load}: lambda {lam:.1f}/s")
        res = {"lambda_req_s": lam if np.isfinite(lam) else "all at t=0"}
        grid_of = [r[0] for r in reqs]
        log("[bench]   plain_fp32")
        lat, wall, ev = run_plain(fc, grids, reqs, arrivals)
        res["plain_fp32"] = summarize(lat, wall, ev, n_req, grid_of)
        for name, form, policy in (
                ("batched_fp32_fifo", fc.FC_FORM_FP32, fc.FC_SCHED_FIFO),
                ("batched_fp32_fair", fc.FC_FORM_FP32, fc.FC_SCHED_FAIR),
                ("batched_split_fp16_fifo", fc.FC_FORM_SPLIT_FP16, fc.FC_SCHED_FIFO)):
            log(f"[bench]   {name}")
            lat, wall, ev, launches, hbm = run_batched(fc, grids, reqs, arrivals, form, policy)
            res[name] = summarize(lat, wall, ev, n_req, grid_of)
            res[name]["launches"] = launches
            res[name]["request_hbm_peak_bytes"] = hbm
        out["loads"][str(load)] = res
    for _, g in grids:
        g.destroy()
    return out


# ---------------------------------------------------------------------------
# One matrix per universe scan (Algorithm 1 as printed) and its iteration
# (Section 2, step 5): a GEMM on the FP64 matrix cores.
# ---------------------------------------------------------------------------
def fixed_bench(pr, d_t, p_t):
    import torch
    import paper_2002_07858_amd as fc
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, pr.stat_mode, pr.stat_diag, forms=fc.FC_FORM_FP64)
    K = int(d_t.shape[0])
    o = {k: torch.empty(K, dtype=torch.float64, device="cuda") for k in ("dchi2", "chi2_min",
                                                                       "chi2_p")}
    o["argmin"] = torch.empty(K, dtype=torch.int64, device="cuda")
    it = torch.empty(K, dtype=torch.int32, device="cuda")
    out = {}
    for name, max_iter in (("fixed", 0), ("iterated", 10)):
        fc.fc_scan_fixed_m(g, d_t, p_t, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"],
                           max_iter, iters=it)                        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fc.fc_scan_fixed_m(g, d_t, p_t, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"],
                           max_iter, iters=it)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        scans = float(K + int(it.sum().item()))
        evals = scans * pr.G
        flops = evals * 2 * pr.N                         # the y.t_q cross term
        r = {"seconds": dt, "universe_scans": scans, "evals": evals, "evals_per_s": evals / dt,
             "roofline": {"bound": "mfma", "achieved": flops / dt / 1e12, "peak": 78.6,
                          "unit": "TFLOP/s", "frac": flops / dt / 78.6e12}}
        if max_iter:
            r["iterations_hist"] = np.bincount(it.cpu().numpy()).tolist()
        out[name] = r
    g.destroy()
    # the iterated results, for the CPU-baseline leg's error report
    return out, {k: v.cpu().numpy() for k, v in o.items()}


def fixed_err(pr, dev, n_sample=60):
    """CPU-baseline leg: the iterated one-matrix results against the oracle on
    a sample of universes."""
    import oracle
    idx = np.random.default_rng(5).choice(pr.K, n_sample, replace=False)
    ref = oracle.scan_fixed_m(pr.S, pr.F, pr.d[idx], pr.p_idx[idx], 10)
    scale = np.maximum(1.0, ref["chi2_p"])
    return {"n": int(n_sample),
            "e_rel": float((np.abs(dev["dchi2"][idx] - ref["dchi2"]) / scale).max()),
            "argmin_agree": float((dev["argmin"][idx] == ref["argmin"]).mean())}


# ---------------------------------------------------------------------------
# Full-surface FC: every grid point a true point, universes drawn on the
# device, per-point universe counts refined near the contour (fc_region).
# ---------------------------------------------------------------------------
def region_bench(pr, form_name: str, K0=256, K_max=4096, z=2.0):
    import torch
    import fcgen
    import paper_2002_07858_amd as fc
    form = {"fp32": fc.FC_FORM_FP32, "fp64": fc.FC_FORM_FP64, "split_bf16": fc.FC_FORM_SPLIT_BF16,
            "split_fp16": fc.FC_FORM_SPLIT_FP16}[form_name]
    c = fcgen.universes(pr.config, 77777, pr.S[pr.G // 2 + 17], pr.F, 1)[0]
    g = fc.fc_build_grid(pr.axes, pr.S, central=c)
    fc.fc_build_covariance(g, pr.F, pr.stat_mode, pr.stat_diag, forms=form | fc.FC_FORM_FP64)
    dd = torch.empty(pr.G, dtype=torch.float64, device="cuda")
    fc.fc_data_scan(g, dd)
    crit = torch.empty((pr.G, len(ALPHA)), dtype=torch.float64, device="cuda")
    acc = torch.empty((pr.G, len(ALPHA)), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = fc.fc_region(g, form, dd, crit, acc, K0=K0, K_max=K_max, z=z, seed=2020,
                        alpha=ALPHA)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.destroy()
    Ku = info["K_used"]
    counts = {int(k): int((Ku == k).sum()) for k in np.unique(Ku)}
    uniform = float(pr.G) * K_max * pr.G
    return {"grid_points": pr.G, "form": form_name, "K0": K0, "K_max": K_max, "z": z,
            "seconds": dt, "rounds": info["rounds"], "evals": info["evals"],
            "evals_per_s": info["evals"] / dt, "points_per_K": counts,
            "mean_K": float(Ku.mean()),
            "evals_vs_uniform_K_max": info["evals"] / uniform,
            "region_points": [int(x) for x in acc.sum(dim=0).cpu().tolist()]}


# ---------------------------------------------------------------------------
# Universes drawn on the device (fc_generate_universes) in the workload's shape:
# the same true points and universe counts, timed with events on the launch
# stream; two launches with one seed must agree bit for bit.
# ---------------------------------------------------------------------------
def gen_bench(fc, grid, pr, pts_t, so_t, reps=3):
    import torch
    K, N = pr.K, pr.N
    d = torch.empty((K, N), dtype=torch.float64, device="cuda")
    d2 = torch.empty_like(d)
    uf = torch.zeros(pts_t.numel(), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    fc.fc_generate_universes(grid, pts_t, so_t, 2020, d2, u_first=uf)  # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(reps):
        ev[0].record(stream)
        fc.fc_generate_universes(grid, pts_t, so_t, 2020, d, u_first=uf)
        ev[1].record(stream)
        ev[1].synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    t = float(np.mean(ms)) * 1e-3
    nbytes = K * N * 8
    return {"universes": K, "bins": N, "ms": t * 1e3, "universes_per_s": K / t,
            "bytes_written": nbytes, "GBps": nbytes / t / 1e9,
            "bitwise_deterministic": bool(torch.equal(d, d2)),
            "kernel": "k_gen_universes",
            "work_per_universe": "N Poisson draws (PTRS) + N normals (Philox4x64-10) + "
                                 "N(N+1)/2 FMAs of the systematic factor"}


# ---------------------------------------------------------------------------
# Grid sharding on one device: the grid cut into equal slices, each scanned by
# its own call (one device's share of a grid-sharded job, at its real shape),
# merged through one shared (key, chi2_p) state, checked bit for bit against
# the one-call scan's outputs.
# ---------------------------------------------------------------------------
def shard_bench(fc, grid, form, form_name, scan_entry, pr, d_t, p_t, pts_t, so_t, ref, n_shards):
    import torch
    K, G = pr.K, pr.G
    edges = [G * i // n_shards for i in range(n_shards + 1)]
    nq_max = max(b - a for a, b in zip(edges[:-1], edges[1:]))
    ws = None
    if scan_entry == "points":
        ws = torch.empty(fc.fc_scan_points_slice_workspace(grid, form, int(so_t.numel()) - 1, K,
                                                           nq_max),
                         dtype=torch.uint8, device="cuda")
    keys = torch.empty(K, dtype=torch.int64, device="cuda")
    chi2_p = torch.empty(K, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_shards + 1)]
    for _ in range(2):  # an untimed pass over the slices, then the timed one
        fc.fc_scan_state_init(keys, chi2_p)
        evs[0].record(stream)
        for i, (a, b) in enumerate(zip(edges[:-1], edges[1:])):
            if scan_entry == "points":
                fc.fc_scan_points_slice(grid, form, pts_t, so_t, d_t, a, b - a, keys, chi2_p,
                                        workspace=ws)
            else:
                fc.fc_scan_slice(grid, form, d_t, p_t, a, b - a, keys, chi2_p)
            evs[i + 1].record(stream)
    o = {k: torch.empty(K, dtype=torch.float64, device="cuda") for k in ("dchi2", "chi2_min")}
    o["argmin"] = torch.empty(K, dtype=torch.int64, device="cuda")
    fc.fc_scan_state_finalize(grid, p_t, keys, chi2_p, o["dchi2"], o["chi2_min"], o["argmin"])
    torch.cuda.synchronize()
    ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(n_shards)]
    mid = float(np.median(ms))
    equal = all(bool(torch.equal(o[k], ref[k])) for k in o) and bool(torch.equal(chi2_p,
                                                                                  ref["chi2_p"]))
    slice_evals = [float(K) * (b - a) for a, b in zip(edges[:-1], edges[1:])]
    flops = slice_evals[0] * (split_flop_per_eval(pr.N) if form_name.startswith("split")
                              else mfma_flop_per_eval(pr.N))
    return {"shards": n_shards, "grid_points_per_shard": edges[1] - edges[0],
            "universes": K, "scan_entry": scan_entry, "slice_ms": ms,
            "slice_evals_per_s": slice_evals[0] / (mid * 1e-3),
            "slice_roofline_frac": flops / (mid * 1e-3) / PEAK[form_name],
            "sum_ms": float(sum(ms)),
            "merged_equals_one_call": equal}


# ---------------------------------------------------------------------------
# The other arithmetic forms on the same inputs: scan time (HIP events around
# the call and around the dominant kernel alone), roofline, and the error
# against the FP64 result on every universe and against the oracle on the
# CPU-baseline sample.
# ---------------------------------------------------------------------------
def roofline_of(form: str, scan: str, N: int, evals: float, kernel_s: float):
    """Roofline of the dominant kernel: the matrix-core work of the contraction
    (the triangular W r; split forms: three 16-bit products per multiply-add)
    against the peak of the form's datatype; the vector work beside it."""
    split = form.startswith("split")
    mf = split_flop_per_eval(N) if split else mfma_flop_per_eval(N)
    achieved = evals * mf / kernel_s
    r = {"kernel": KERNEL[form] if scan == "points" or form != "fp32" else "k_scan_fp32",
         "bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[form] / 1e12,
         "unit": "TFLOP/s", "frac": achieved / PEAK[form],
         "flop_per_eval_mfma": mf,
         "flop_per_eval_vector": vector_flop_per_eval(N, form, scan),
         "frac_method_flops": evals * flop_per_eval(N) / kernel_s /
         PEAK["fp32" if split else form],
         "kernel_ms": kernel_s * 1e3, "traffic": None}
    return r


def profiled_kernel_s(fc, form: str, scan: str):
    name = KERNEL[form] if scan == "points" or form != "fp32" else "k_scan_fp32"
    n, ms = fc.fc_profile_read(name)
    return (ms / n * 1e-3) if n else None


def forms_leg(fc, grid, pr, forms, pts_t, so_t, d_t, ref64, sample, steps=2):
    import torch
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import parity
    K, G, N = pr.K, pr.G, pr.N
    out = {}
    o = {k: torch.empty(K, dtype=torch.float64, device="cuda") for k in ("dchi2", "chi2_min",
                                                                       "chi2_p")}
    o["argmin"] = torch.empty(K, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    code = {"fp32": fc.FC_FORM_FP32, "fp64": fc.FC_FORM_FP64,
            "split_bf16": fc.FC_FORM_SPLIT_BF16, "split_fp16": fc.FC_FORM_SPLIT_FP16}
    scale = np.maximum(1.0, ref64["chi2_p"])
    for name in forms:
        form = code[name]
        log(f"[bench] leg {name}")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        fc.fc_build_covariance(grid, pr.F, pr.stat_mode, pr.stat_diag, forms=form)
        ev[1].record(stream)
        ev[1].synchronize()
        cov_ms = ev[0].elapsed_time(ev[1])
        ws = torch.empty(fc.fc_scan_points_workspace(grid, form, int(so_t.numel()) - 1, K),
                         dtype=torch.uint8, device="cuda")
        ms = []
        for i in range(steps + 1):          # the first pass is a warm-up
            if i == 1:
                fc.fc_profile_enable(True)
            ev[0].record(stream)
            fc.fc_scan_points(grid, form, pts_t, so_t, d_t, o["dchi2"], o["chi2_min"],
                              o["argmin"], o["chi2_p"], workspace=ws)
            ev[2].record(stream)
            ev[2].synchronize()
            if i:
                ms.append(ev[0].elapsed_time(ev[2]))
        ks = profiled_kernel_s(fc, name, "points")
        fc.fc_profile_enable(False)
        t = float(np.mean(ms)) * 1e-3
        dev = {k: v.cpu().numpy() for k, v in o.items()}
        e_all = np.abs(dev["dchi2"] - ref64["dchi2"]) / scale
        rl = roofline_of(name, "points", N, float(K) * G, ks if ks else t)
        tr = TRAFFIC.get((pr.name, name, "points"))
        if tr is not None and tr["source_hash"] == kernel_source_hash(tr["sources"]):
            rl["traffic"] = tr["bytes_per_launch"]
            rl["traffic_GBps"] = tr["bytes_per_launch"] / (rl["kernel_ms"] * 1e-3) / 1e9
            rl["traffic_source"] = tr["profile"]
        r = {"scan_ms": t * 1e3, "covariance_ms": cov_ms, "evals_per_s": K * G / t,
             "roofline": rl,
             "vs_fp64_all_universes": {"n": K, "e_rel": float(e_all.max()),
                                       "e_abs": float(np.abs(dev["dchi2"] - ref64["dchi2"]).max()),
                                       "argmin_equal_frac": float((dev["argmin"] ==
                                                                   ref64["argmin"]).mean())}}
        if sample is not None:
            idx, ref = sample
            e = parity.report({k: v[idx] for k, v in dev.items()}, ref, TOL[name])
            e.update(parity.argmin_validity(pr, {k: v[idx] for k, v in dev.items()},
                                            pr.d[idx], ref, TOL[name]))
            r["vs_oracle_sample"] = e
        out[name] = r
    return out


def device_record():
    """The device and software the line was measured on, and the peak
    denominators of the roofline fractions."""
    import ctypes
    import torch
    props = torch.cuda.get_device_properties(0)
    rec = {"name": props.name, "arch": getattr(props, "gcnArchName", None),
           "compute_units": props.multi_processor_count,
           "hbm_bytes": props.total_memory, "hip": torch.version.hip, "torch": torch.__version__,
           "peaks_per_s": {**{k: v for k, v in PEAK.items()}, "hbm_bytes": 8.0e12}}
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0:  # hipDeviceAttributeClockRate (kHz)
            rec["max_sclk_mhz"] = v.value / 1000.0
    except OSError:
        pass
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--form", default="fp64", choices=["fp32", "fp64", "split_bf16", "split_fp16"],
                    help="scan form of the headline (default fp64, the paper's arithmetic)")
    ap.add_argument("--legs", default=None,
                    help="comma-separated other forms run on the same inputs (default: all "
                         "other forms; 'none' to skip)")
    ap.add_argument("--scan", default="points", choices=["points", "universes"],
                    help="scan entry: fc_scan_points (universes grouped by true point, "
                    "default) or fc_scan (per-universe true points)")
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-per-point", type=int, default=None,
                    help="universes per true point in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=None,
                    help="requests in the serving leg (0 to skip it; default 200)")
    ap.add_argument("--fixed", type=int, default=1,
                    help="1: the one-matrix scan leg on the c2 grid (0 to skip)")
    ap.add_argument("--gen", type=int, default=1,
                    help="1: time fc_generate_universes in the workload's shape (0 to skip)")
    ap.add_argument("--region", type=int, default=1,
                    help="1: the full-surface region leg on the c2 grid (0 to skip)")
    ap.add_argument("--shards", type=int, default=8,
                    help="grid-sharding leg in the FP32 form: slices of the grid scanned by "
                         "separate calls (0: off)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this size (counter calibration)")
    ap.add_argument("--serving-loads", default="0.5,0.8,sat",
                    help="comma-separated arrival rates as fractions of the plain capacity "
                         "('sat': every request queued at t = 0, which measures capacity)")
    args = ap.parse_args()
    wl = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = wl["steps"]
    if args.warmup is None:
        args.warmup = wl["warmup"]
    if args.cpu_per_point is None:
        args.cpu_per_point = wl["cpu_per_point"]
    if args.serving_requests is None:
        args.serving_requests = wl["serving"]
    if args.legs is None:
        legs = [f for f in ("fp32", "split_bf16", "split_fp16", "fp64") if f != args.form]
    else:
        legs = [] if args.legs == "none" else [f for f in args.legs.split(",") if f]
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the scan is "
              "single-GPU by design; see the multi-GPU section of the design notes.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import fcgen
    import paper_2002_07858_amd as fc

    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
        return
    fc.lib()
    code = {"fp32": fc.FC_FORM_FP32, "fp64": fc.FC_FORM_FP64,
            "split_bf16": fc.FC_FORM_SPLIT_BF16, "split_fp16": fc.FC_FORM_SPLIT_FP16}
    form = code[args.form]

    log(f"[bench] generating {args.workload} inputs")
    pr = fcgen.make_problem(args.workload)
    G, N, K = pr.G, pr.N, pr.K
    dev = torch.device("cuda")
    d_t = torch.as_tensor(pr.d).to(dev)
    p_t = torch.as_tensor(pr.p_idx).to(dev)
    so_t = torch.as_tensor(pr.seg_off).to(dev)
    n_seg = len(pr.seg_off) - 1
    outs = {k: torch.empty(K, dtype=torch.float64, device=dev) for k in ("dchi2", "chi2_min",
                                                                        "chi2_p")}
    outs["argmin"] = torch.empty(K, dtype=torch.int64, device=dev)
    crit = torch.empty((n_seg, len(ALPHA)), dtype=torch.float64, device=dev)
    hist = torch.empty((n_seg, N_BINS + 1), dtype=torch.int64, device=dev)
    log("[bench] grid residency")
    grid = fc.fc_build_grid(pr.axes, pr.S)
    stream = torch.cuda.current_stream()

    ev = {k: torch.cuda.Event(enable_timing=True) for k in ("c0", "c1", "s0", "s1", "k1")}

    # universes grouped by true point (Algorithm 1's shape): fc_scan_points with
    # a workspace allocated once; --scan universes uses fc_scan with per-universe
    # true points instead
    pts_t = torch.as_tensor(pr.p_idx[pr.seg_off[:-1]]).to(dev)
    ws = None
    if args.scan == "points":
        ws = torch.empty(fc.fc_scan_points_workspace(grid, form, n_seg, K), dtype=torch.uint8,
                         device=dev)

    def step(times=None):
        ev["c0"].record(stream)
        fc.fc_build_covariance(grid, pr.F, pr.stat_mode, pr.stat_diag, forms=form)
        ev["c1"].record(stream)
        ev["s0"].record(stream)
        if args.scan == "points":
            fc.fc_scan_points(grid, form, pts_t, so_t, d_t, outs["dchi2"], outs["chi2_min"],
                              outs["argmin"], outs["chi2_p"], workspace=ws)
        else:
            fc.fc_scan(grid, form, d_t, p_t, outs["dchi2"], outs["chi2_min"], outs["argmin"],
                       outs["chi2_p"])
        ev["s1"].record(stream)
        fc.fc_critical_value(so_t, outs["dchi2"], ALPHA, crit, N_BINS, HIST_HI, hist)
        ev["k1"].record(stream)
        if times is not None:
            ev["k1"].synchronize()
            times["cov"].append(ev["c0"].elapsed_time(ev["c1"]))
            times["scan"].append(ev["s0"].elapsed_time(ev["s1"]))
            times["crit"].append(ev["s1"].elapsed_time(ev["k1"]))

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    first = None
    times = {"cov": [], "scan": [], "crit": []}
    log(f"[bench] timing {args.steps} steps")
    fc.fc_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(times)
        log(f"[bench] step {i}: scan {times['scan'][-1]:.2f} ms")
        if first is None:
            first = (outs["dchi2"].clone(), outs["argmin"].clone(), crit.clone())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = profiled_kernel_s(fc, args.form, args.scan)
    fc.fc_profile_enable(False)

    evals = K * G
    value = evals * args.steps / wall
    scan_ms = float(np.mean(times["scan"]))
    roofline = roofline_of(args.form, args.scan, N, float(evals),
                           kernel_s if kernel_s else scan_ms * 1e-3)
    roofline["kernel_timing"] = ("HIP events around each launch of the kernel on its stream, "
                                 f"mean over the {args.steps} timed steps")
    tr = TRAFFIC.get((args.workload, args.form, args.scan))
    if tr is not None and tr["source_hash"] == kernel_source_hash(tr["sources"]):
        roofline["traffic"] = tr["bytes_per_launch"]
        roofline["traffic_GBps"] = tr["bytes_per_launch"] / (roofline["kernel_ms"] * 1e-3) / 1e9
        roofline["traffic_source"] = tr["profile"]

    deterministic = bool(torch.equal(first[0], outs["dchi2"]) and
                         torch.equal(first[1], outs["argmin"]) and
                         torch.equal(first[2], crit)) if first is not None else None
    dev_out = {k: v.cpu().numpy() for k, v in outs.items()}
    res = {"metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.form], "data": "synthetic",
           "config": {"workload": wl["desc"] + ", per-point FP64 covariance factor, "
                                  f"{args.form} scan, crit at 0.6827/0.9/0.95 + 200-bin hist",
                      "G": G, "N": N, "K_total": K, "evals_per_step": evals,
                      "form": args.form, "scan_entry": "fc_scan_points" if args.scan == "points"
                      else "fc_scan", "parallelism": "single-gpu"},
           "phases_ms": {k: float(np.mean(v)) for k, v in times.items()},
           "scan_evals_per_s": evals / (scan_ms * 1e-3),
           "bitwise_deterministic": deterministic,
           "roofline": roofline,
           "device": device_record()}
    sample = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        base, rep = cpu_baseline(pr, args.cpu_per_point, dev_out, TOL[args.form])
        res["cpu_baseline"] = base
        sample = rep.pop("_sample")
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import parity
        idx, ref = sample
        rep.update(parity.argmin_validity(pr, {k: v[idx] for k, v in dev_out.items()},
                                          pr.d[idx], ref, TOL[args.form]))
        res["err_vs_fp64"] = rep
    if legs:
        res["forms_same_inputs"] = forms_leg(fc, grid, pr, legs, pts_t, so_t, d_t, dev_out,
                                             sample)
    if args.shards > 0:
        log(f"[bench] grid sharding leg ({args.shards} slices, FP32)")
        fc.fc_build_covariance(grid, pr.F, pr.stat_mode, pr.stat_diag, forms=fc.FC_FORM_FP32)
        ref32 = {k: torch.empty(K, dtype=torch.float64, device=dev) for k in ("dchi2", "chi2_min",
                                                                            "chi2_p")}
        ref32["argmin"] = torch.empty(K, dtype=torch.int64, device=dev)
        fc.fc_scan_points(grid, fc.FC_FORM_FP32, pts_t, so_t, d_t, ref32["dchi2"],
                          ref32["chi2_min"], ref32["argmin"], ref32["chi2_p"])
        res["grid_shard"] = shard_bench(fc, grid, fc.FC_FORM_FP32, "fp32", "points", pr, d_t, p_t,
                                        pts_t, so_t, ref32, args.shards)
        del ref32
    if args.gen:
        log("[bench] universes drawn on the device")
        res["universe_generation"] = gen_bench(fc, grid, pr, pts_t, so_t)
    grid.destroy()
    del d_t, p_t, outs
    torch.cuda.empty_cache()
    if args.fixed or args.region:
        pr2 = pr if args.workload == "c2" else fcgen.make_problem("c2")
    if args.fixed:
        log("[bench] one-matrix scan (c2 grid)")
        d2 = torch.as_tensor(pr2.d).to(dev)
        p2 = torch.as_tensor(pr2.p_idx).to(dev)
        res["fixed_matrix"], fixed_dev = fixed_bench(pr2, d2, p2)
        res["fixed_matrix"]["workload"] = WORKLOADS["c2"]["desc"]
        if not args.no_cpu_baseline:
            res["fixed_matrix"]["iterated"]["err_vs_oracle"] = fixed_err(pr2, fixed_dev)
        del d2, p2
    if args.region:
        log("[bench] full-surface region (c2 grid)")
        res["region"] = region_bench(pr2, "fp32")
    if args.serving_requests > 0:
        res["serving"] = serving_bench(args.serving_requests,
                                       tuple(x if x == "sat" else float(x)
                                             for x in args.serving_loads.split(",")))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
