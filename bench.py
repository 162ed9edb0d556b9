#!/usr/bin/env python3
"""Benchmark of the sketch / Gram / leverage / least-squares hot path on one
MI355X.

One step is one pass of the whole path over the sparse workload (CSR A,
1,000,000 x 500, density 1e-3, FP64; CountSketch r = 250,000 buckets then a
Gaussian with m = 2,000 rows):

    C     = G*S*A                  sketch_gcs   (hash, binning, S*A, Gaussian GEMM)
    Gram  = A^T A                  gram
    R, R^-1 of C                   sketch_qr
    theta = rownorm^2(A R^-1)      rownorms_sq  (sketched leverage scores)
    x     = argmin ||A x - b||     lsq_solve    (LSQR preconditioned by R^-1)

Inputs are synthetic and seeded (the paper's matrices are random with
unstated distributions) and are resident in HBM before timing starts.
The FP64 plain path and the paths with the BF16 and FP8 Gaussian GEMMs are
all timed (``--prec all``, the default); the BF16 path is the headline and
the other two are reported beside it.  Prints ONE JSON line.  ``value`` is GB/s of A
through the whole step (bytes of A = values + column indices + row
pointers, per step, divided by the step time).  The dominant kernel (the
Gaussian product; for this sparse workload k_gauss_sparse, bound by the
VALU work of drawing G) is timed with HIP events on its own stream inside
the library and reported as a roofline fraction; the CPU oracle is timed on
a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

WORKLOADS = {
    # name: (kind, n, d, density, r, m)
    "csr-1e6x500": ("csr", 1_000_000, 500, 1e-3, 250_000, 2000),
    "dense-20000x50": ("dense", 20_000, 50, None, 2500, 200),
}
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0
# VALU peak in lane-operations: the FP32 vector rate, 157.3 TFLOP/s at 256 CUs
# and 2.4 GHz, is 128 FP32 FMA lanes per CU per clock (a wave64 v_fma_f32 in
# two cycles per SIMD; psk_probe_valu_f32 reaches ~82% of it without packed
# instructions), one lane-operation per FMA: 157.3 / 2 = 78.65 T/s
PEAK_VALU_TOPS = 157.3 / 2
# VALU lane-operations per Gaussian sample of the sparse product's G (BF16):
# a Philox4x32-10 block and its Box-Muller pair of pairs give 4 samples for
# 20 64-bit multiplies, 20 three-input XORs and 71 further operations
# (uniforms, 2 log, 2 sqrt, sin/cos polynomials, products), log and sqrt at
# half rate (+4), and 8 for the rounding to bfloat16: 123 per 4 samples
VALU_OPS_PER_SAMPLE_BF16 = 123 / 4

# HBM bytes per launch of the dominant kernel from hardware counters
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, the factors measured on a copy
# kernel of known size), valid only for the kernel source they were taken
# on: the figure is dropped (null) as soon as the source hash differs.
PMC_TRAFFIC = {
    ("csr-1e6x500", "bf16"): {
        "source": "paper_2203_02798_amd/csrc/k_gauss_sparse.hip",
        "sha256_prefix": "813cd88f73adeb9b",
        "fetch_kib": 23572.2, "write_kib": 31250.0,
        "fetch_scale": 2.000, "write_scale": 1.000,
        "profile": "profiles/gauss_sparse_bf16_csr-1e6x500_pmc.md",
    },
}


def pmc_traffic(workload, prec):
    import hashlib
    t = PMC_TRAFFIC.get((workload, prec))
    if t is None:
        return None
    with open(os.path.join(HERE, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha256_prefix"]:
            return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def a_bytes(a, kind):
    if kind == "csr":
        return a.nnz * (a.data.itemsize + 4) + (a.shape[0] + 1) * 8
    return a.size * a.itemsize


def make_inputs(name):
    import synth
    kind, n, d, dens, r, m = WORKLOADS[name]
    if kind == "csr":
        a = synth.csr_uniform(n, d, dens, seed=0)
    else:
        a = synth.dense_gaussian(n, d, seed=0)
    rng = np.random.default_rng(1)
    xt = rng.standard_normal(d)
    b = a @ xt + 1e-3 * rng.standard_normal(n)
    return kind, a, b, r, m


def serving_trace_gpu(torch, num, seed, n_lo, n_hi, device):
    """Synthetic least-squares requests drawn on the device: n log-uniform in
    [n_lo, n_hi], d uniform over {32, 64, 128, 256}, condition number
    log-uniform in [1, 1e8]; A = X diag(s) V^T with X ~ N(0,1)/sqrt(n), V the
    Q factor of a Gaussian, s geometric from 1 to 1/cond; b = A x + 1e-3 e."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(num):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        d = int(rng.choice([32, 64, 128, 256]))
        cond = float(np.exp(rng.uniform(0.0, np.log(1e8))))
        g = torch.Generator(device=device)
        g.manual_seed(seed * 100003 + k)
        x = torch.randn(n, d, generator=g, device=device, dtype=torch.float64) / n ** 0.5
        v, _ = torch.linalg.qr(torch.randn(d, d, generator=g, device=device,
                                           dtype=torch.float64))
        sv = torch.logspace(0.0, -np.log10(cond), d, device=device, dtype=torch.float64)
        a = ((x * sv) @ v.T).contiguous()
        xt = torch.randn(d, generator=g, device=device, dtype=torch.float64)
        b = a @ xt + 1e-3 * torch.randn(n, generator=g, device=device, dtype=torch.float64)
        reqs.append(dict(a=a, b=b, n=n, d=d, cond=cond, m=4 * d, r=min(d * d, n), seed=k))
    torch.cuda.synchronize(device)
    return reqs


def serving_bench(api, torch, device, num=64, slots=8, pool_gb=16.0):
    """Closed-loop runs (all requests queued at t = 0) of the request server
    for the FP64 and BF16 sketch at two sketch sizes (m = 4d and 8d; r =
    min(d^2, n) >= m), and an open-loop run (Poisson arrivals at 0.8x the best
    FP64 rate) with the best BF16 configuration."""
    reqs = serving_trace_gpu(torch, num, 0, 1e4, 2e5, device)
    pool = int(pool_gb * (1 << 30))

    def run(prec, mf, esc=0.0, arrivals=None):
        with api.Server(pool, slots=slots, device=device) as srv:
            t0 = time.perf_counter()
            pend = []
            for k, q in enumerate(reqs):
                if arrivals is not None:
                    wait = arrivals[k] - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                m = mf * q["d"]
                r = max(min(q["d"] * q["d"], q["n"]), m)
                pend.append(srv.submit_lsq(q["a"], q["b"], m=m, r=r, seed=q["seed"],
                                           prec=prec, escalate_cond=esc))
            res = [srv.wait(t) for t, _ in pend]
            wall = time.perf_counter() - t0
            st = srv.stats()
        lat = np.array([1e3 * (r_["t_end"] - r_["t_submit"]) for r_ in res])
        out = {"prec": prec, "m": f"{mf}d", "solves_per_s": num / wall,
               "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "wall_s": wall,
               "failed": sum(1 for r_ in res if r_["status"] != "PSK_OK"),
               "inflight_peak": st["inflight_peak"], "pool_peak_bytes": st["pool_peak"],
               "lsqr_iters_mean": float(np.mean([r_["iters"] for r_ in res]))}
        if prec == "bf16":
            out["escalate_cond"] = esc if esc else 1e4
            out["escalated_to_f64"] = int(sum(1 for r_ in res if r_["prec_used"] == "f64"))
        return out, [x for _, x in pend]

    runs = {}
    sols = {}
    for prec, mf, esc in (("f64", 4, 0.0), ("f64", 8, 0.0), ("bf16", 4, 0.0),
                          ("bf16", 8, 0.0), ("bf16", 8, 1e3), ("bf16", 16, 0.0)):
        key = f"{prec}_m{mf}d" + ("_esc1e3" if esc else "")
        log(f"serving: {num} requests, closed loop, {key}")
        runs[key], sols[key] = run(prec, mf, esc)
    ok = lambda k: runs[k]["failed"] == 0
    best64 = max((k for k in runs if k.startswith("f64") and ok(k)),
                 key=lambda k: runs[k]["solves_per_s"])
    best16 = max((k for k in runs if k.startswith("bf16") and ok(k)),
                 key=lambda k: runs[k]["solves_per_s"])
    # residual of each solution, best BF16 vs best FP64 configuration
    rel = []
    for q, xa, xb in zip(reqs, sols[best64], sols[best16]):
        ra = torch.linalg.vector_norm(q["b"] - q["a"] @ xa).item()
        rb = torch.linalg.vector_norm(q["b"] - q["a"] @ xb).item()
        rel.append(abs(rb - ra) / ra)
    rate = 0.8 * runs[best64]["solves_per_s"]
    arr = np.cumsum(np.random.default_rng(1).exponential(1.0 / rate, size=num))
    prec, mf = runs[best16]["prec"], int(runs[best16]["m"][:-1])
    esc = 1e3 if best16.endswith("esc1e3") else 0.0
    log(f"serving: open loop, Poisson arrivals at {rate:.1f}/s, {best16}")
    ol, _ = run(prec, mf, esc, arrivals=arr)
    olf, _ = run("f64", int(runs[best64]["m"][:-1]), 0.0, arrivals=arr)
    return {
        "trace": (f"{num} synthetic LSQ requests, n log-uniform [1e4, 2e5], d in "
                  "{32,64,128,256}, cond log-uniform [1, 1e8], r = max(min(d^2, n), m), "
                  "A resident in HBM before submission"),
        "slots": slots, "pool_bytes": pool,
        "closed_loop": runs,
        "best_fp64": best64, "best_bf16": best16,
        "bf16_vs_fp64_solves": runs[best16]["solves_per_s"] / runs[best64]["solves_per_s"],
        "resid_rel_diff_max": float(max(rel)),
        "open_loop": {"arrival_rate": rate, best16: ol, best64: olf},
    }


def gaussian_only_bench(api, torch, A, m, n, d, nnz, seed, steps, warmup):
    """G*A (sketch_g, the Gaussian-only sketch of CSR A, BF16 G) on the same
    matrix: m n normals and one FMA per (row of G, nonzero of A), the same
    kernel as the combined sketch with one bucket per row."""
    for _ in range(warmup):
        api.sketch_g(A, m, seed, prec="bf16")
    torch.cuda.synchronize()
    with api.kernel_timing() as kt:
        t0 = time.perf_counter()
        for _ in range(steps):
            api.sketch_g(A, m, seed, prec="bf16")
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        stats = kt.stats()
    gg_ms, gg_n = stats.get("gauss_gemm", (0.0, 0))
    launch = gg_ms / max(gg_n, 1)
    ops = m * n * VALU_OPS_PER_SAMPLE_BF16 + m * nnz
    ach = ops / (launch * 1e-3) / 1e12 if launch > 0 else 0.0
    return {"call": "sketch_g", "prec": "bf16", "m": m, "ms_per_call": 1e3 * wall,
            "stage_ms": {k: round(v[0] / steps, 4) for k, v in sorted(stats.items())},
            "roofline": {"bound": "alu", "kernel": "k_gauss_sparse", "achieved": ach,
                         "peak": PEAK_VALU_TOPS, "unit": "T VALU lane-ops/s",
                         "frac": ach / PEAK_VALU_TOPS, "launch_ms": launch,
                         "samples_per_launch": m * n, "fma_per_launch": m * nnz}}


def leverage_jl_bench(api, torch, steps, warmup, n=4_000_000, d=256, r=65536, m=1024,
                      t=64, seed=0):
    """leverage_sketch on the dense tall-skinny FP32 configuration (4,000,000 x
    256, singular values geometric from 1 to 1e-6, 5% of rows scaled by 100),
    with and without the JL step.  A = Z diag(s) V^T with Z Gaussian and V
    orthogonal, generated on the device.  The sketch is FP64 (at cond 1e6 a
    BF16 S A loses the small singular directions).  Reported: time per call,
    the row-norm product's time (n d^2 against n d t multiply-adds), and the
    spread of theta(t) / theta(0), which the JL bound keeps near
    1 +- sqrt(2/t) per row."""
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    v, _ = torch.linalg.qr(torch.randn(d, d, generator=g, device="cuda:0",
                                       dtype=torch.float64))
    s = torch.logspace(0, -6, d, dtype=torch.float64, device="cuda:0")
    w = (s[:, None] * v.T).to(torch.float32)
    A = torch.randn(n, d, generator=g, device="cuda:0", dtype=torch.float32) @ w
    hot = torch.randperm(n, generator=g, device="cuda:0")[: n // 20]
    A[hot] *= 100.0
    torch.cuda.synchronize()
    out = {"workload": f"dense FP32 {n} x {d}, r = {r}, m = {m}, sketch f64", "t": t}
    th = {}
    for tt in (0, t):
        for _ in range(warmup):
            api.leverage_sketch(A, m, r, seed, t=tt)
        torch.cuda.synchronize()
        with api.kernel_timing() as kt:
            t0 = time.perf_counter()
            for _ in range(steps):
                res = api.leverage_sketch(A, m, r, seed, t=tt)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / steps
            stats = kt.stats()
        rn_ms = stats.get("rownorm", (0.0, 0))[0] / steps
        k = tt if tt > 0 else d
        out[f"t{tt}"] = {"ms_per_call": 1e3 * wall, "rownorm_ms": rn_ms,
                         "rownorm_tflops": 2.0 * n * d * k / (rn_ms * 1e-3) / 1e12
                         if rn_ms > 0 else None,
                         "stage_ms": {kk: round(vv[0] / steps, 4)
                                      for kk, vv in sorted(stats.items())}}
        th[tt] = res
    # the sketch alone in the configuration's own precision (BF16 G)
    for _ in range(warmup):
        api.sketch_gcs(A, m, r, seed, prec="bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.sketch_gcs(A, m, r, seed, prec="bf16")
    torch.cuda.synchronize()
    sk = (time.perf_counter() - t0) / steps
    out["sketch_gcs_bf16"] = {"ms_per_call": 1e3 * sk, "gbs": n * d * 4 / sk / 1e9}
    ratio = (th[t] / th[0]).cpu().numpy()
    out["jl_ratio"] = {"min": float(ratio.min()), "max": float(ratio.max()),
                       "std": float(ratio.std()), "jl_std": float(np.sqrt(2.0 / t))}
    out["sum_theta_t0"] = float(th[0].sum())
    del A
    torch.cuda.empty_cache()
    return out


def css_bench(api, torch, A, d, r, seed, steps, warmup):
    """Column subset selection on the bench matrix with the algorithm's own
    sketch sizes (m = 2d Gaussian rows; r = d^2 buckets is the bench's r):
    the first k pivots for k = d/5 and k = d, and Algorithm ls_hrn_exact's
    leverage scores of the d/5 selected columns, BF16 Gaussian product."""
    m = 2 * d
    kk = max(d // 5, 1)
    calls = {
        f"css_select_k{kk}": lambda: api.css_select(A, m, r, kk, seed, prec="bf16"),
        f"css_select_k{d}": lambda: api.css_select(A, m, r, d, seed, prec="bf16"),
        f"leverage_css_k{kk}": lambda: api.leverage_css(A, m, r, kk, seed, prec="bf16"),
    }
    out = {"m": m, "r": r, "prec": "bf16"}
    for name, f in calls.items():
        for _ in range(warmup):
            f()
        torch.cuda.synchronize()
        with api.kernel_timing() as kt:
            t0 = time.perf_counter()
            for _ in range(steps):
                f()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / steps
            stats = kt.stats()
        out[name] = {"ms_per_call": 1e3 * wall,
                     "stage_ms": {k: round(v[0] / steps, 4) for k, v in sorted(stats.items())}}
    return out


def zipf_fp8_bench(api, torch, steps, warmup, n=10_000_000, d=1000, dens=1e-4, r=1_000_000,
                   m=4000, seed=0):
    """G*S*A with the FP8 Gaussian product on the Zipf-row CSR configuration
    (10,000,000 x 1,000 FP32, density 1e-4, Zipf(1.5) row lengths, r = 1e6,
    m = 4,000), A resident in HBM."""
    import synth
    a = synth.csr_zipf(n, d, dens, seed=seed, dtype=np.float32)
    A = api.CsrMatrix.from_scipy(a, device="cuda:0")
    for _ in range(warmup):
        api.sketch_gcs(A, m, r, seed, prec="fp8")
    torch.cuda.synchronize()
    with api.kernel_timing() as kt:
        t0 = time.perf_counter()
        for _ in range(steps):
            api.sketch_gcs(A, m, r, seed, prec="fp8")
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        stats = kt.stats()
    nbytes = a_bytes(a, "csr")
    return {"workload": f"CSR {n} x {d} FP32, Zipf rows, nnz {a.nnz}, r = {r}, m = {m}",
            "ms_per_call": 1e3 * wall, "gbs": nbytes / wall / 1e9, "a_bytes": nbytes,
            "stage_ms": {k: round(v[0] / steps, 4) for k, v in sorted(stats.items())}}


def direct_bench(api, torch, A, a, b, bd, m, r, seed, steps, warmup, lsqr_resid):
    """The direct solvers on the same matrix: exact leverage scores and least
    squares from the Gram matrix, and sketch-and-solve with the bench's
    sketch (BF16 G), each timed alone, with the quality of its result."""
    calls = {
        "leverage_gram": lambda: api.leverage_gram(A),
        "lsq_gram": lambda: api.lsq_gram(A, bd),
        "lsq_sketch_solve_bf16": lambda: api.lsq_sketch_solve(A, bd, m, r, seed, prec="bf16"),
    }
    out = {}
    for name, f in calls.items():
        for _ in range(warmup):
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = f()
        torch.cuda.synchronize()
        out[name] = {"ms_per_call": 1e3 * (time.perf_counter() - t0) / steps}
        v = res.cpu().numpy()
        if name == "leverage_gram":
            out[name]["sum_minus_d"] = float(v.sum() - a.shape[1])
        else:
            rn = float(np.linalg.norm(b - a @ v))
            out[name]["resid"] = rn
            out[name]["resid_vs_lsqr"] = rn / lsqr_resid
    return out


def cpu_baseline(kind, a, b, r, m, seed, budget_s=12.0):
    """The oracle on the host: every stage in full except the Gaussian GEMM,
    whose bucket batches (Algorithm countgauss_multiply) are timed on a
    prefix until ~budget_s and scaled by the batch count."""
    from oracle import gram as og
    from oracle import leverage as olev
    from oracle import sketch as osk
    import scipy.linalg as sla
    from scipy.sparse.linalg import LinearOperator, lsqr
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    t = {}
    t0 = time.perf_counter()
    sa = osk.sketch_cs(a, r, seed)
    t["sketch_cs"] = time.perf_counter() - t0
    batch = 4096
    nb = (r + batch - 1) // batch
    c = np.zeros((m, sa.shape[1]))
    t0 = time.perf_counter()
    done = 0
    for b0 in range(0, r, batch):
        b1 = min(r, b0 + batch)
        c += osk.gaussian_block(m, b0, b1, seed) @ sa[b0:b1]
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t["gauss_gemm"] = (time.perf_counter() - t0) * nb / done
    t0 = time.perf_counter()
    og.gram(1.0, a)
    t["gram"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    rr = olev.qr_r(c)  # C from the sampled batches: same shape, same QR cost
    ri = olev.tri_inv(rr)
    t["qr"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    n = a.shape[0]
    for i0 in range(0, n, 200_000):
        og.rownorms_sq(1.0, a[i0:i0 + 200_000], ri)
    t["rownorms"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    op = LinearOperator(a.shape, matvec=lambda y: a @ (ri @ y),
                        rmatvec=lambda u: ri.T @ (a.T @ u), dtype=np.float64)
    y = lsqr(op, b, atol=1e-14, btol=1e-14, iter_lim=100)[0]
    _ = ri @ y
    t["lsq"] = time.perf_counter() - t0
    total = sum(t.values())
    sample = (f"all stages in full except the Gaussian GEMM: {done} of {nb} bucket "
              f"batches of {batch} timed and scaled")
    return total, cores, sample, t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="csr-1e6x500", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="all", choices=["f64", "bf16", "fp8", "all"],
                    help="Gaussian GEMM precision; 'all' times the FP64 plain path, "
                         "the BF16 path and the FP8 path and reports BF16 as the "
                         "headline")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the request-server measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the Gaussian-only sketch, direct-solver, column-selection, Zipf FP8, JL "
                         "leverage measurements "
                         "(hardware-counter runs: one workload per kernel)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run 4 elementwise copies of MIB "
                         "MiB (FP64) whose HBM bytes are known, to scale hardware "
                         "FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by rows of A; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_02798_amd import api

    if args.copy_calibration:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nb, "bytes_written": nb,
                                               "launches": 4}}), flush=True)
        return

    log(f"generating workload {args.workload}")
    kind, a, b, r, m = make_inputs(args.workload)
    n, d = a.shape
    nbytes = a_bytes(a, kind)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if kind == "csr":
        A = api.CsrMatrix.from_scipy(a, device=dev)
    else:
        A = torch.from_numpy(a).to(dev)
    bd = torch.from_numpy(b).to(dev)
    torch.cuda.synchronize()

    seed = args.seed

    def run_path(prec):
        def step():
            C = api.sketch_gcs(A, m, r, seed, prec=prec)
            Gm = api.gram(A)
            R, Ri = api.sketch_qr(C)
            th = api.rownorms_sq(A, Ri)
            x, info = api.lsq_solve(A, bd, Rinv=Ri, max_iter=200, refine=1, check_every=8)
            return C, Gm, th, x, info

        log(f"[{prec}] warmup {args.warmup}")
        for _ in range(args.warmup):
            out = step()
        torch.cuda.synchronize()
        log(f"[{prec}] timing {args.steps} steps")
        lat = []
        stream = torch.cuda.current_stream(dev)
        # inside the timed steps only the Gaussian product is bracketed (the
        # roofline's launch time); every bracket costs host time, so the
        # per-stage breakdown comes from two further steps afterwards
        with api.kernel_timing(only=("gauss_gemm",)) as kt:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            for _ in range(args.steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                out = step()
                e1.record(stream)
                e1.synchronize()
                lat.append(e0.elapsed_time(e1))
            torch.cuda.synchronize()
            t_total = time.perf_counter() - t_start
            gg_ms, gg_n = kt.stats().get("gauss_gemm", (0.0, 0))
        n_stage = 2
        with api.kernel_timing() as kt:
            for _ in range(n_stage):
                step()
            torch.cuda.synchronize()
            stats = kt.stats()
        info = out[4]
        lat = np.array(lat)
        per = {k: v[0] / n_stage for k, v in stats.items()}
        sketch_ms = sum(per.get(k, 0.0) for k in ("cs_bin", "cs_scatter", "sa_limbs",
                                                   "sa_quant", "gauss_gemm", "gemm_reduce"))
        # residual of the returned solution, for the FP64-vs-BF16 comparison
        x = out[3].cpu().numpy()
        res = float(np.linalg.norm(b - a @ x))
        return {
            "value": nbytes * args.steps / t_total / 1e9,
            "ms_per_step": 1e3 * t_total / args.steps,
            "solves_per_s": args.steps / t_total,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "sketch_gcs_gbs": nbytes / (sketch_ms * 1e-3) / 1e9 if sketch_ms > 0 else None,
            "stage_ms": {k: round(v, 4) for k, v in sorted(per.items())},
            "lsq": {"iters": info["iters"], "status": info["status"], "resid": res},
            "gg_avg_ms": gg_ms / max(gg_n, 1),
            "sparse_product": "sa_entries" in stats,
        }

    paths = [args.prec] if args.prec != "all" else ["f64", "bf16", "fp8"]
    res = {p: run_path(p) for p in paths}
    head = "bf16" if "bf16" in res else paths[0]
    hr = res[head]
    flops = (2.0 * r - 1.0) * m * d
    gg_avg = hr["gg_avg_ms"]
    if hr["sparse_product"] and head == "bf16":
        # k_gauss_sparse: bound by the VALU work of drawing G (m r samples)
        # plus one FMA per (row of G, nonzero of S*A)
        if kind == "csr":
            h, _ = api.cs_hash(n, r, seed, device=dev)
            rows = np.repeat(np.arange(n), np.diff(a.indptr))
            keys = h.cpu().numpy().astype(np.int64)[rows] * d + a.indices
            nnz_sa = int(np.unique(keys).size)
        else:
            nnz_sa = r * d
        ops = m * r * VALU_OPS_PER_SAMPLE_BF16 + m * nnz_sa
        achieved = ops / (gg_avg * 1e-3) / 1e12 if gg_avg > 0 else 0.0
        roof = {"bound": "alu", "kernel": "k_gauss_sparse", "achieved": achieved,
                "peak": PEAK_VALU_TOPS, "unit": "T VALU lane-ops/s",
                "frac": achieved / PEAK_VALU_TOPS,
                "traffic": pmc_traffic(args.workload, head),
                "traffic_unit": "bytes per launch", "launch_ms": gg_avg,
                "ops_per_launch": ops, "samples_per_launch": m * r,
                "valu_ops_per_sample": VALU_OPS_PER_SAMPLE_BF16,
                "nnz_sa": nnz_sa, "fma_per_launch": m * nnz_sa}
    else:
        peak = {"f64": PEAK_FP64_TFLOPS, "bf16": PEAK_BF16_TFLOPS,
                "fp8": PEAK_FP8_TFLOPS}[head]
        achieved = flops / (gg_avg * 1e-3) / 1e12 if gg_avg > 0 else 0.0
        roof = {"bound": "mfma", "kernel": "gauss_gemm", "achieved": achieved,
                "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "traffic_unit": "bytes per launch",
                "launch_ms": gg_avg, "flops_per_launch": flops}
    # the rates this device sustains (ceiling probes), beside the datasheet's
    ceil = None
    if not args.no_extras:
        log("ceiling probes: copy, FP64 MFMA, VALU")
        ceil = api.measure_ceilings(dev)
        if roof["bound"] == "alu":
            roof["measured_peak"] = ceil["valu_Tops"]
        elif head == "f64":
            roof["measured_peak"] = ceil["fp64_mfma_TFs"]
        if "measured_peak" in roof:
            roof["frac_measured"] = roof["achieved"] / roof["measured_peak"]
    rec = {
        "metric": "GB/s of A sketched (G·S·A) + LSQ solves/s, p50/p99 latency vs FP64 plain path",
        "value": hr["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "dtype_detail": {"bf16": "Gaussian product with bf16 G and S*A as two bf16 limbs, "
                                 "fp32 accumulation; hash, S*A, Gram, QR, row norms and "
                                 "LSQR in f64",
                         "fp8": "Gaussian GEMM fp8 e4m3 operands (per-128 E8M0 scales) "
                                "with fp32 accumulation; the rest in f64",
                         "f64": "f64 throughout"}[head],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d,
                   "nnz": int(a.nnz) if kind == "csr" else n * d,
                   "density": WORKLOADS[args.workload][3], "r": r, "m": m,
                   "a_bytes": nbytes, "parallelism": "single-gpu"},
        "solves_per_s": hr["solves_per_s"],
        "p50_ms": hr["p50_ms"],
        "p99_ms": hr["p99_ms"],
        "sketch_gcs_gbs": hr["sketch_gcs_gbs"],
        "stage_ms": hr["stage_ms"],
        "lsq": hr["lsq"],
        "roofline": roof,
    }
    if ceil is not None:
        rec["ceilings"] = {**ceil, "datasheet": {"hbm_GBs": 8000.0,
                                                 "fp64_mfma_TFs": PEAK_FP64_TFLOPS,
                                                 "bf16_mfma_TFs": PEAK_BF16_TFLOPS,
                                                 "fp8_mfma_TFs": PEAK_FP8_TFLOPS,
                                                 "valu_Tops": PEAK_VALU_TOPS},
                           "probes": "psk_probe_copy (1 GiB read + 1 GiB written), "
                                     "psk_probe_mfma_f64, psk_probe_mfma_lowp (bf16, fp8), "
                                     "psk_probe_valu_f32; best of 3"}
    keys = ("value", "ms_per_step", "solves_per_s", "p50_ms", "p99_ms", "sketch_gcs_gbs",
            "stage_ms", "lsq")
    if head != "f64" and "f64" in res:
        f = res["f64"]
        rec["fp64_path"] = {k: f[k] for k in keys}
        rec["speedup_vs_fp64_path"] = f["ms_per_step"] / hr["ms_per_step"]
    if head != "fp8" and "fp8" in res:
        f = res["fp8"]
        rec["fp8_path"] = {k: f[k] for k in keys}
        gg = f["gg_avg_ms"]
        rec["fp8_path"]["gauss_gemm_roofline"] = {
            "achieved": flops / (gg * 1e-3) / 1e12 if gg > 0 else 0.0,
            "peak": PEAK_FP8_TFLOPS, "unit": "TFLOP/s",
            "frac": (flops / (gg * 1e-3) / 1e12) / PEAK_FP8_TFLOPS if gg > 0 else 0.0}
        if ceil is not None and gg > 0:
            g8 = rec["fp8_path"]["gauss_gemm_roofline"]
            g8["measured_peak"] = ceil["fp8_mfma_TFs"]
            g8["frac_measured"] = g8["achieved"] / ceil["fp8_mfma_TFs"]
    if head == "bf16" and kind == "csr" and not args.no_extras:
        rec["gaussian_only"] = gaussian_only_bench(api, torch, A, m, n, d, int(a.nnz), seed,
                                                   args.steps, args.warmup)
        rec["direct"] = direct_bench(api, torch, A, a, b, bd, m, r, seed, args.steps,
                                     args.warmup, hr["lsq"]["resid"])
        rec["css"] = css_bench(api, torch, A, d, r, seed, args.steps, args.warmup)
        log("FP8 sketch of the Zipf CSR 10,000,000 x 1,000")
        rec["zipf_fp8"] = zipf_fp8_bench(api, torch, args.steps, args.warmup)
        log("leverage scores with the JL step, dense FP32 4,000,000 x 256")
        rec["leverage_jl"] = leverage_jl_bench(api, torch, args.steps, args.warmup)
        if ceil is not None:
            for tt in ("t0", f"t{rec['leverage_jl']['t']}"):
                tf = rec["leverage_jl"][tt]["rownorm_tflops"]
                if tf:
                    rec["leverage_jl"][tt]["rownorm_frac"] = tf / PEAK_FP64_TFLOPS
                    rec["leverage_jl"][tt]["rownorm_frac_measured"] = tf / ceil["fp64_mfma_TFs"]
    if not args.no_serving:
        rec["serving"] = serving_bench(api, torch, dev)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        tot, cores, sample, parts = cpu_baseline(kind, a, b, r, m, seed)
        rec["cpu_baseline"] = {"value": nbytes / tot / 1e9, "unit": "GB/s", "cores": cores,
                               "kind": "oracle", "sample": sample,
                               "stage_s": {k: round(v, 3) for k, v in parts.items()}}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
