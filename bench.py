#!/usr/bin/env python3
"""Benchmark of the sketch / Gram / leverage / least-squares hot path on one
MI355X.

Headline: one step is one pass of the path over the dense tall-skinny
workload (A 4,000,000 x 256 FP32, singular values geometric from 1 to 1e-6,
5% of rows scaled by 100; CountSketch r = 65,536 buckets, Gaussian m = 1,024
rows) in the paper's arithmetic, FP64:

    C     = G*S*A                  sketch_gcs   (hash, binning, S*A, Gaussian GEMM)
    Gram  = A^T A                  gram         (second stream, beside the two above)
    R, R^-1 of C                   sketch_qr
    theta = rownorm^2(A R^-1)      rownorms_sq  (sketched leverage scores)

The Gram depends on A alone, so it runs on a second HIP stream while the
sketch and its QR run on the first; the row norms start when both are done,
alone on the GPU.  The same step run on one stream is reported beside it.

Inputs are synthetic and seeded (the paper's matrices are random with
unstated distributions) and are resident in HBM before timing starts.
``value`` is GB/s of A through the whole step (bytes of A per step divided
by the step time).  The dominant kernel of the step is timed with HIP events
on its own stream inside the library and reported as a roofline fraction
against the FP64 matrix peak, on the method's own flops.  Beside it: the
BF16 and FP8 sketches of the same matrix with their perturbation delta, the
small dense workload's latency, the sparse workload (CSR 1e6 x 500) with
least squares, the Zipf CSR 1e7 x 1000 FP8 sketch and leverage scores, the
request server on the 512-request least-squares trace, and the CPU oracle
timed on a bounded sample of the headline workload.  Prints ONE JSON line.
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

METRIC = "GB/s of A sketched (G·S·A) + LSQ solves/s, p50/p99 latency vs FP64 plain path"
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0
PEAK_HBM_GBS = 8000.0
# VALU peak in lane-operations: the FP32 vector rate, 157.3 TFLOP/s at 256 CUs
# and 2.4 GHz, is 128 FP32 FMA lanes per CU per clock, one lane-operation per
# FMA: 157.3 / 2 = 78.65 T/s
PEAK_VALU_TOPS = 157.3 / 2

# Headline workload: dense coherent FP32 n x d, r buckets, m Gaussian rows
HEAD = dict(n=4_000_000, d=256, r=65536, m=1024, smin=1e-6)

# HBM bytes per launch of the headline's dominant kernels from hardware
# counters (FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale, the factors
# measured on a copy kernel of known size), valid only for the kernel source
# they were taken on: a figure is dropped (null) as soon as the source hash
# differs.
PMC_TRAFFIC = {
    "k_gram_syrk": {
        "source": "paper_2203_02798_amd/csrc/k_dense.hip",
        "sha256_prefix": "be36c3e0e668d061",
        "fetch_kib": 4068896.1, "write_kib": 69821.0,
        "fetch_scale": 2.000, "write_scale": 1.000,
        "profile": "profiles/step_dense-4e6x256_pmc.md",
    },
    "k_rownorm_bres": {
        "source": "paper_2203_02798_amd/csrc/k_dense.hip",
        "sha256_prefix": "be36c3e0e668d061",
        "fetch_kib": 6241491.0, "write_kib": 329335.0,
        "fetch_scale": 2.000, "write_scale": 1.000,
        "profile": "profiles/step_dense-4e6x256_pmc.md",
    },
}


def pmc_traffic(kernel):
    import hashlib
    t = PMC_TRAFFIC.get(kernel)
    if t is None or t["sha256_prefix"] is None:
        return None
    with open(os.path.join(HERE, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha256_prefix"]:
            return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def csr_bytes(a):
    """Everything the method reads of a CSR matrix: values, int32 column
    indices, int64 row pointers."""
    return a.nnz * (a.data.itemsize + 4) + (a.shape[0] + 1) * 8


def timed(torch, f, steps, warmup, stream=None):
    """(mean wall seconds per call, per-call event milliseconds) of f."""
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        f()
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    if steps == 0:  # warm-up only
        return 0.0, lat
    return (time.perf_counter() - t0) / steps, lat


# ---------------------------------------------------------------------------
# headline: the FP64 step on the dense coherent 4e6 x 256 matrix
# ---------------------------------------------------------------------------
def headline(api, torch, A, steps, warmup, seed):
    n, d, r, m = HEAD["n"], HEAD["d"], HEAD["r"], HEAD["m"]
    nbytes = n * d * 4

    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()  # default priority, as every stream here

    def step():
        # the Gram on the side stream, after whatever the main stream holds;
        # the sketch, its QR and the row norms on the main stream, which then
        # waits for the Gram
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            Gm = api.gram(A)
        C = api.sketch_gcs(A, m, r, seed, prec="f64")
        R, Ri = api.sketch_qr(C)
        th = api.rownorms_sq(A, Ri)
        stream.wait_stream(side)
        Gm.record_stream(stream)
        return C, Gm, Ri, th

    def step_serial():
        C = api.sketch_gcs(A, m, r, seed, prec="f64")
        Gm = api.gram(A)
        R, Ri = api.sketch_qr(C)
        th = api.rownorms_sq(A, Ri)
        return C, Gm, Ri, th

    log(f"[f64] warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"[f64] timing {steps} steps")
    # inside the timed steps only the two dominant kernels are bracketed (each
    # bracket costs host time); the per-stage breakdown comes from two
    # one-stream steps afterwards, each kernel alone on the GPU
    with api.kernel_timing(only=("gram", "rownorm")) as kt:
        wall, lat = timed(torch, step, steps, 0, stream)
        kst = kt.stats()
    log(f"[f64] timing {steps} one-stream steps")
    wall_serial, _ = timed(torch, step_serial, steps, 1, stream)
    with api.kernel_timing() as kt:
        for _ in range(2):
            out = step_serial()
        torch.cuda.synchronize()
        per = {k: v[0] / 2 for k, v in kt.stats().items()}
    chk = step()
    torch.cuda.synchronize()
    same = all(bool(torch.equal(x, y)) for x, y in zip(chk, out))
    th = out[3]
    sketch_ms = sum(per.get(k, 0.0) for k in ("cs_bin", "cs_scatter", "gauss_gemm",
                                                "gemm_reduce"))
    lat = np.array(lat)
    # method's own flops: the Gram matrix's d(d+1)/2 distinct dot products of
    # length n (2 n d (d+1) / 2), the row norms' product with the triangular
    # R^{-1} (sum_j 2 (j+1) per row) and the squares: n d (d+2); executed
    # flops: the 16 x 16 blocks of the upper block triangle (Gram), the K
    # chunks of the paired 32-column tiles up to each tile's extent, less the
    # zero quarter of each diagonal chunk inside d (row norms)
    flops = {"gram": n * d * (d + 1), "rownorm": n * d * (d + 2)}
    tiles = (d + 31) // 32
    exe = {"gram": n * ((d + 15) // 16) * ((d + 15) // 16 + 1) // 2 * 512,
           "rownorm": int(n * 2 * 32 * 32 * sum(t + 1 - (0.25 if 32 * t + 32 <= d else 0.0)
                                                 for t in range(tiles)))}
    kern = {}
    for name, kname in (("gram", "k_gram_syrk"), ("rownorm", "k_rownorm_bres")):
        ms, cnt = kst.get(name, (0.0, 0))
        launch = ms / max(cnt, 1)
        ach = flops[name] / (launch * 1e-3) / 1e12 if launch > 0 else 0.0
        kern[name] = {"kernel": kname, "launch_ms": launch, "launches": cnt,
                      "flops_per_launch": flops[name], "achieved_TFs": ach,
                      "frac": ach / PEAK_FP64_TFLOPS,
                      "executed_flops_per_launch": exe[name],
                      "executed_TFs": exe[name] / (launch * 1e-3) / 1e12 if launch > 0 else 0.0}
    dom = max(kern, key=lambda k: kern[k]["launch_ms"])
    k = kern[dom]
    roof = {"bound": "mfma", "kernel": k["kernel"], "achieved": k["achieved_TFs"],
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": k["frac"],
            "traffic": pmc_traffic(k["kernel"]), "traffic_unit": "bytes per launch",
            "launch_ms": k["launch_ms"], "flops_per_launch": k["flops_per_launch"],
            "flops_basis": "method's own flops (Gram: n d (d+1), symmetric; row norms: "
                           "n d (d+2), triangular R^-1)",
            "executed_TFs": k["executed_TFs"],
            "executed_frac": k["executed_TFs"] / PEAK_FP64_TFLOPS}
    # the S*A stage against HBM: A read once, S*A (FP64) written, bins
    sa_bytes = nbytes + r * d * 8 + n * 4 * 2
    scat = per.get("cs_scatter", 0.0)
    res = {
        "value": nbytes * steps / (wall * steps) / 1e9,
        "ms_per_step": 1e3 * wall,
        "one_stream_ms_per_step": 1e3 * wall_serial,
        "two_stream_results_identical": same,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "sketch_gcs_ms": sketch_ms,
        "sketch_gcs_gbs": nbytes / (sketch_ms * 1e-3) / 1e9 if sketch_ms > 0 else None,
        "scatter_hbm": {"bytes": sa_bytes, "ms": scat,
                        "GBs": sa_bytes / (scat * 1e-3) / 1e9 if scat > 0 else None,
                        "frac": sa_bytes / (scat * 1e-3) / 1e9 / PEAK_HBM_GBS if scat > 0 else None,
                        "stage_frac_with_binning":
                            sa_bytes / ((scat + per.get("cs_bin", 0.0)) * 1e-3) / 1e9 /
                            PEAK_HBM_GBS if scat > 0 else None},
        "stage_ms": {kk: round(v, 4) for kk, v in sorted(per.items())},
        "kernels": kern,
        "roofline": roof,
        "sum_theta": float(th.sum().item()),
    }
    return res


def reduced_sketches(api, torch, A, steps, warmup, seed):
    """The BF16 and FP8 sketches of the headline matrix: time per call, GB/s of
    A, and delta = ||(C^ - C) R^{-1}||_2 against the FP64 sketch, with the
    leverage bracket it allows; plus the JL step's effect on the row norms."""
    n, d, r, m = HEAD["n"], HEAD["d"], HEAD["r"], HEAD["m"]
    nbytes = n * d * 4
    c64 = api.sketch_gcs(A, m, r, seed, prec="f64")
    out = {}
    for prec in ("bf16", "fp8"):
        f = lambda: api.sketch_gcs(A, m, r, seed, prec=prec)
        timed(torch, f, 0, warmup)
        with api.kernel_timing() as kt:
            wall, _ = timed(torch, f, steps, 0)
            st = kt.stats()
        ch = f()
        delta = api.sketch_delta(ch, c64).item()
        out[prec] = {"ms_per_call": 1e3 * wall, "gbs": nbytes / wall / 1e9,
                     "delta": delta,
                     "leverage_ratio_bound": (1 - delta) ** -2 - 1 if delta < 1 else None,
                     "valid_delta_lt_half": delta < 0.5,
                     "stage_ms": {k: round(v[0] / steps, 4) for k, v in sorted(st.items())}}
    return out


def leverage_jl(api, torch, A, steps, warmup, seed, t=64):
    """leverage_sketch (FP64 sketch) with and without the JL step on the
    headline matrix: time per call and the row-norm product's time."""
    n, d, r, m = HEAD["n"], HEAD["d"], HEAD["r"], HEAD["m"]
    out = {"t": t}
    th = {}
    for tt in (0, t):
        f = lambda: api.leverage_sketch(A, m, r, seed, t=tt)
        timed(torch, f, 0, warmup)
        with api.kernel_timing() as kt:
            wall, _ = timed(torch, f, steps, 0)
            st = kt.stats()
        rn = st.get("rownorm", (0.0, 1))
        rn_ms = rn[0] / max(rn[1], 1)
        out[f"t{tt}"] = {"ms_per_call": 1e3 * wall, "rownorm_ms": rn_ms}
        th[tt] = f()
    ratio = (th[t] / th[0]).cpu().numpy()
    out["jl_ratio"] = {"std": float(ratio.std()), "jl_std": float(np.sqrt(2.0 / t))}
    return out


# ---------------------------------------------------------------------------
# the small dense workload: end-to-end latency
# ---------------------------------------------------------------------------
def small_latency(api, torch, steps=50, warmup=5):
    import synth
    n, d, r, m = 20000, 50, 2500, 200
    a = synth.dense_gaussian(n, d, seed=0)
    rng = np.random.default_rng(1)
    b = a @ rng.standard_normal(d) + 1e-3 * rng.standard_normal(n)
    A = torch.from_numpy(a).cuda()
    bd = torch.from_numpy(b).cuda()

    def step():
        C = api.sketch_gcs(A, m, r, 0)
        api.gram(A)
        _, Ri = api.sketch_qr(C)
        api.rownorms_sq(A, Ri)
        return api.lsq_solve(A, bd, Rinv=Ri, max_iter=200, refine=1, check_every=8)

    wall, lat = timed(torch, step, steps, warmup)
    x, info = step()
    return {"workload": f"dense FP64 {n} x {d}, r = {r}, m = {m}", "steps": steps,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": 1e3 * wall, "lsq_iters": info["iters"],
            "note": "one step: sketch, Gram, QR, row norms and LSQR; latency-bound "
                    "(every stage is microseconds of work)"}


def check_once(api, torch, A):
    """psk_check on a resident CSR matrix, once, marking it checked so that
    the timed calls skip their own structure pass; its milliseconds."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    api.check(A, mark=True)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0)


# ---------------------------------------------------------------------------
# the sparse workload CSR 1e6 x 500: the step with least squares per precision
# ---------------------------------------------------------------------------
def csr_workload(api, torch, steps, warmup, seed):
    import synth
    n, d, dens, r, m = 1_000_000, 500, 1e-3, 250_000, 2000
    a = synth.csr_uniform(n, d, dens, seed=0)
    rng = np.random.default_rng(1)
    b = a @ rng.standard_normal(d) + 1e-3 * rng.standard_normal(n)
    A = api.CsrMatrix.from_scipy(a, device="cuda:0")
    bd = torch.from_numpy(b).cuda()
    nbytes = csr_bytes(a)
    out = {"workload": f"CSR {n} x {d} FP64, density {dens}, r = {r}, m = {m}",
           "a_bytes": nbytes}
    # the step with the per-call structure check (every CSR call checks A on
    # the device and synchronises), then A checked once and marked
    def step_unchecked():
        C = api.sketch_gcs(A, m, r, seed)
        api.gram(A)
        _, Ri = api.sketch_qr(C)
        api.rownorms_sq(A, Ri)
        return api.lsq_solve(A, bd, Rinv=Ri, max_iter=200, refine=1, check_every=8)
    wall_u, _ = timed(torch, step_unchecked, steps, warmup)
    out["f64_ms_per_step_checking_each_call"] = 1e3 * wall_u
    out["check_once_ms"] = check_once(api, torch, A)
    c64 = api.sketch_gcs(A, m, r, seed)
    for prec in ("f64", "bf16", "fp8"):
        def step():
            C = api.sketch_gcs(A, m, r, seed, prec=prec)
            api.gram(A)
            _, Ri = api.sketch_qr(C)
            api.rownorms_sq(A, Ri)
            return C, api.lsq_solve(A, bd, Rinv=Ri, max_iter=200, refine=1, check_every=8)
        wall, lat = timed(torch, step, steps, warmup)
        with api.kernel_timing() as kt:
            C, (x, info) = step()
            torch.cuda.synchronize()
            st = kt.stats()
        res = float(np.linalg.norm(b - a @ x.cpu().numpy()))
        delta, delta_ms = 0.0, None
        if prec != "f64":
            # the perturbation against the FP64 sketch (outside the step),
            # and what one such call costs (its QR of C included)
            delta = api.sketch_delta(C, c64).item()
            dwall, _ = timed(torch, lambda: api.sketch_delta(C, c64), 3, 1)
            delta_ms = 1e3 * dwall
        out[prec] = {"gbs": nbytes / wall / 1e9, "ms_per_step": 1e3 * wall,
                     "solves_per_s": 1.0 / wall,
                     "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)),
                     "delta": delta, "delta_ms": delta_ms,
                     "lsq": {"iters": info["iters"], "status": info["status"], "resid": res},
                     "stage_ms": {k: round(v[0], 4) for k, v in sorted(st.items())}}
    out["bf16_vs_fp64_step"] = out["f64"]["ms_per_step"] / out["bf16"]["ms_per_step"]
    # the Gaussian product over S*A's nonzeros (BF16): bound by drawing G
    return out, A, a, b, bd


def gaussian_only(api, torch, A, m, seed, steps, warmup):
    f = lambda: api.sketch_g(A, m, seed, prec="bf16")
    wall, _ = timed(torch, f, steps, warmup)
    return {"call": "sketch_g", "prec": "bf16", "m": m, "ms_per_call": 1e3 * wall}


def direct_bench(api, torch, A, a, b, bd, m, r, seed, steps, warmup):
    calls = {
        "leverage_gram": lambda: api.leverage_gram(A),
        "lsq_gram": lambda: api.lsq_gram(A, bd),
        "lsq_sketch_solve_bf16": lambda: api.lsq_sketch_solve(A, bd, m, r, seed, prec="bf16"),
    }
    out = {}
    for name, f in calls.items():
        wall, _ = timed(torch, f, steps, warmup)
        out[name] = {"ms_per_call": 1e3 * wall}
    return out


def css_bench(api, torch, A, d, r, seed, steps, warmup):
    m = 2 * d
    kk = max(d // 5, 1)
    calls = {
        f"css_select_k{kk}": lambda: api.css_select(A, m, r, kk, seed, prec="bf16"),
        f"css_select_k{d}": lambda: api.css_select(A, m, r, d, seed, prec="bf16"),
        f"leverage_css_k{kk}": lambda: api.leverage_css(A, m, r, kk, seed, prec="bf16"),
    }
    out = {"m": m, "r": r, "prec": "bf16"}
    for name, f in calls.items():
        wall, _ = timed(torch, f, steps, warmup)
        out[name] = {"ms_per_call": 1e3 * wall}
    return out


# ---------------------------------------------------------------------------
# the Zipf CSR 1e7 x 1000 FP32: FP8 sketch and leverage scores
# ---------------------------------------------------------------------------
def zipf_workload(api, torch, steps, warmup, seed):
    import synth
    n, d, dens, r, m = 10_000_000, 1000, 1e-4, 1_000_000, 4000
    a = synth.csr_zipf(n, d, dens, seed=seed, dtype=np.float32)
    A = api.CsrMatrix.from_scipy(a, device="cuda:0")
    nbytes = csr_bytes(a)
    out = {"workload": f"CSR {n} x {d} FP32, Zipf(1.5) rows, nnz {a.nnz}, "
                       f"non-empty rows {int((np.diff(a.indptr) > 0).sum())}, r = {r}, m = {m}",
           "a_bytes": nbytes}
    out["check_once_ms"] = check_once(api, torch, A)
    c64 = api.sketch_gcs(A, m, r, seed)
    for prec in ("fp8", "f64"):
        f = lambda: api.sketch_gcs(A, m, r, seed, prec=prec)
        timed(torch, f, 0, warmup)
        with api.kernel_timing() as kt:
            wall, _ = timed(torch, f, steps, 0)
            st = kt.stats()
        out[prec] = {"ms_per_call": 1e3 * wall, "gbs": nbytes / wall / 1e9,
                     "stage_ms": {k: round(v[0] / steps, 4) for k, v in sorted(st.items())}}
    out["fp8"]["delta"] = api.sketch_delta(api.sketch_gcs(A, m, r, seed, prec="fp8"), c64).item()
    f = lambda: api.leverage_sketch(A, m, r, seed, t=0, prec="fp8")
    wall, _ = timed(torch, f, steps, warmup)
    th = f()
    out["leverage_fp8"] = {"ms_per_call": 1e3 * wall, "sum_theta": float(th.sum().item())}
    # OSNAP with s = 8 non-zeros per column at one eighth of the CountSketch
    # rows: S*A costs s passes over the entries, the Gaussian product shrinks
    # with r
    s_os, r_os = 8, r // 8
    osn = {"s": s_os, "r": r_os}
    c64o = api.sketch_osnap(A, s_os, m, r_os, seed)
    for prec in ("fp8", "f64"):
        f = lambda: api.sketch_osnap(A, s_os, m, r_os, seed, prec=prec)
        timed(torch, f, 0, warmup)
        with api.kernel_timing() as kt:
            wall, _ = timed(torch, f, steps, 0)
            st = kt.stats()
        osn[prec] = {"ms_per_call": 1e3 * wall, "gbs": nbytes / wall / 1e9,
                     "stage_ms": {k: round(v[0] / steps, 4) for k, v in sorted(st.items())}}
    osn["fp8"]["delta"] = api.sketch_delta(api.sketch_osnap(A, s_os, m, r_os, seed, prec="fp8"),
                                           c64o).item()
    del c64o

    def lev_osnap():
        _, ri = api.sketch_qr(api.sketch_osnap(A, s_os, m, r_os, seed, prec="fp8"))
        return api.rownorms_sq(A, ri)
    wall, _ = timed(torch, lev_osnap, steps, warmup)
    osn["leverage_fp8"] = {"ms_per_call": 1e3 * wall,
                           "sum_theta": float(lev_osnap().sum().item())}
    out["osnap"] = osn
    return out


# ---------------------------------------------------------------------------
# the paper's own matrix shapes (its Table of test matrices, tall case):
# 2,097,152 x 512 FP64, dense and 5% sparse, r = 100 d = 51,200, m = 2 d
# ---------------------------------------------------------------------------
def paper_shape(api, torch, steps, warmup, seed):
    n, d = 2_097_152, 512
    r, m = 100 * d, 2 * d
    out = {"shape": f"{n} x {d} FP64, r = {r}, m = {m}",
           "note": "the paper's tall test shape; its matrices' distributions are unstated, so "
                   "N(0,1) entries (dense) and uniform 5% positions with N(0,1) values (CSR) "
                   "stand in"}
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    A = torch.randn(n, d, dtype=torch.float64, device="cuda:0", generator=g)
    nbytes = n * d * 8
    for prec in ("f64", "bf16"):
        f = lambda: api.sketch_gcs(A, m, r, seed, prec=prec)
        wall, _ = timed(torch, f, steps, warmup)
        out[f"dense_{prec}"] = {"ms_per_call": 1e3 * wall, "gbs": nbytes / wall / 1e9}
    del A
    # CSR: each of the n d positions kept with probability 0.05 (drawn on the
    # device), column indices increasing within a row
    keep = torch.rand(n, d, device="cuda:0", generator=g) < 0.05
    pos = keep.nonzero()
    del keep
    counts = torch.bincount(pos[:, 0], minlength=n)
    indptr = torch.zeros(n + 1, dtype=torch.int64, device="cuda:0")
    indptr[1:] = torch.cumsum(counts, 0)
    indices = pos[:, 1].to(torch.int32)
    del pos, counts
    values = torch.randn(indices.numel(), dtype=torch.float64, device="cuda:0", generator=g)
    C = api.CsrMatrix(indptr, indices, values, (n, d))
    nnz = int(indices.numel())
    cbytes = nnz * (8 + 4) + (n + 1) * 8
    out["csr_nnz"] = nnz
    out["csr_check_once_ms"] = check_once(api, torch, C)
    for prec in ("f64", "bf16"):
        f = lambda: api.sketch_gcs(C, m, r, seed, prec=prec)
        wall, _ = timed(torch, f, steps, warmup)
        out[f"csr_{prec}"] = {"ms_per_call": 1e3 * wall, "gbs": cbytes / wall / 1e9}
    del C, indptr, indices, values
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# serving: 512 least-squares requests, Poisson arrivals, HBM-pool admission
# ---------------------------------------------------------------------------
def serving_bench(api, torch, num=512, slots=8, pools_gb=(32.0, 128.0), n_hi=1e6,
                  mfs=(8, 32)):
    import synth
    log(f"serving: drawing {num} requests on the device")
    reqs = synth.lsq_trace_torch(num, 0, 1e4, n_hi, device="cuda:0")
    torch.cuda.synchronize()
    abytes = sum(q["a"].numel() * 8 for q in reqs)
    kappa_edges = [1.0, 1e2, 1e4, 1e6, 1e8 + 1]

    def run(prec, mf, pool_gb, arrivals=None, want_delta=False):
        pool = int(pool_gb * (1 << 30))
        with api.Server(pool, slots=slots, device="cuda:0") as srv:
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
                                           prec=prec, want_delta=want_delta))
            res = [srv.wait(t) for t, _ in pend]
            wall = time.perf_counter() - t0
            st = srv.stats()
        lat = np.array([1e3 * (r_["t_end"] - r_["t_submit"]) for r_ in res])
        out = {"prec": prec, "m": f"{mf}d", "pool_gb": pool_gb, "solves_per_s": num / wall,
               "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "wall_s": wall,
               "failed": sum(1 for r_ in res if r_["status"] != "PSK_OK"),
               "inflight_peak": st["inflight_peak"], "pool_peak_bytes": st["pool_peak"],
               "lsqr_iters_mean": float(np.mean([r_["iters"] for r_ in res])),
               "escalated_to_f64": int(sum(1 for r_ in res if prec != "f64" and
                                           r_["prec_used"] == "f64"))}
        return out, res, [x for _, x in pend]

    runs = {}
    sols = {}
    # every precision at m = 8d in each pool, and at m = 32d in the larger
    # pool: a cheaper Gaussian product affords more sketch rows, which cut
    # LSQR's iterations (cond(A R^-1) <= (1 + eps) / (1 - eps), eps ~ sqrt(d/m))
    big = int(max(pools_gb))
    grid = [(prec, 8, pool_gb) for pool_gb in pools_gb for prec in ("f64", "bf16", "fp8")]
    grid += [(prec, mf, float(big)) for mf in mfs if mf != 8 for prec in ("f64", "bf16", "fp8")]
    for prec, mf, pool_gb in grid:
        key = f"{prec}_m{mf}d_pool{int(pool_gb)}g"
        log(f"serving: closed loop {key}")
        runs[key], _, sols[key] = run(prec, mf, pool_gb)
    ok = lambda k: runs[k]["failed"] == 0
    at_big = [k for k in runs if k.endswith(f"pool{big}g") and ok(k)]
    best64 = max([k for k in at_big if k.startswith("f64")],
                 key=lambda k: runs[k]["solves_per_s"])
    red = [k for k in at_big if not k.startswith("f64")]
    bestred = max(red, key=lambda k: runs[k]["solves_per_s"]) if red else None
    mf_of = lambda k: int(k.split("_m")[1].split("d_")[0])
    # residuals of each reduced-precision solution against the FP64 one
    rel = {}
    for key in red:
        worst = 0.0
        for q, xa, xb in zip(reqs, sols[best64], sols[key]):
            ra = torch.linalg.vector_norm(q["b"] - q["a"] @ xa).item()
            rb = torch.linalg.vector_norm(q["b"] - q["a"] @ xb).item()
            worst = max(worst, abs(rb - ra) / ra)
        rel[key] = worst
    # per condition-number bucket: delta, iterations, escalations (a separate
    # pass with want_delta, not timed against the others)
    buckets = {}
    for prec in ("bf16", "fp8"):
        log(f"serving: delta pass {prec}")
        _, res, _ = run(prec, 8, float(big), want_delta=True)
        for lo, hi in zip(kappa_edges[:-1], kappa_edges[1:]):
            idx = [i for i, q in enumerate(reqs) if lo <= q["cond"] < hi]
            if not idx:
                continue
            ds = [res[i]["delta_est"] for i in idx if res[i]["prec_used"] == prec]
            key = f"{prec}_cond_{lo:.0e}_{hi:.0e}"
            buckets[key] = {
                "requests": len(idx),
                "escalated_to_f64": int(sum(1 for i in idx if res[i]["prec_used"] == "f64")),
                "lsqr_iters_mean": float(np.mean([res[i]["iters"] for i in idx])),
                "delta_max_kept": float(max(ds)) if ds else None,
                "delta_median_kept": float(np.median(ds)) if ds else None}
    # Poisson arrivals at 0.5, 0.8 and 1.2 times the FP64 path's closed-loop
    # rate mu (request k keeps its seed): latency below, near and above
    # saturation
    mu = runs[best64]["solves_per_s"]
    open_loop = {}
    for frac in (0.5, 0.8, 1.2):
        rate = frac * mu
        arr = np.cumsum(np.random.default_rng(1).exponential(1.0 / rate, size=num))
        log(f"serving: open loop at {rate:.1f}/s ({frac} mu)")
        key = f"{frac}mu"
        open_loop[key] = {"arrival_rate": rate}
        open_loop[key]["f64"], _, _ = run("f64", mf_of(best64), float(big), arrivals=arr)
        if bestred:
            pr = runs[bestred]["prec"]
            open_loop[key][pr], _, _ = run(pr, mf_of(bestred), float(big), arrivals=arr)
    out = {
        "trace": (f"{num} synthetic LSQ requests, n log-uniform [1e4, {n_hi:.0e}], d in "
                  "{32,64,128,256}, cond log-uniform [1, 1e8], b = A x + 1e-3 e, "
                  f"m in {{{', '.join(f'{mf}d' for mf in mfs)}}}, "
                  "r = max(min(d^2, n), m); A resident in HBM before submission"),
        "a_bytes_total": abytes, "slots": slots, "pools_gb": list(pools_gb),
        "closed_loop": runs,
        "best_fp64": best64, "best_reduced": bestred,
        "reduced_vs_fp64_solves": (runs[bestred]["solves_per_s"] /
                                   runs[best64]["solves_per_s"]) if bestred else None,
        "resid_rel_diff_max": rel,
        "by_cond": buckets,
        "open_loop": {"mu_f64_closed_loop": mu, **open_loop},
    }
    del reqs
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# the CPU oracle on a bounded sample of the headline workload
# ---------------------------------------------------------------------------
def cpu_baseline(A, seed, rows=500_000, budget_s=8.0):
    """The oracle's FP64 step on the host: S*A, the Gram matrix and the row
    norms on the first `rows` rows of the headline matrix (scaled by n/rows),
    the Gaussian product's bucket batches on a prefix until ~budget_s
    (scaled by the batch count), and the QR of the m x d sketch in full."""
    from oracle import gram as og
    from oracle import leverage as olev
    from oracle import sketch as osk
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    n, d, r, m = HEAD["n"], HEAD["d"], HEAD["r"], HEAD["m"]
    a = A[:rows].cpu().numpy().astype(np.float64)
    scale = n / rows
    t = {}
    t0 = time.perf_counter()
    sa = osk.sketch_cs(a, r, seed)
    t["sketch_cs"] = (time.perf_counter() - t0) * scale
    batch = 4096
    nb = (r + batch - 1) // batch
    c = np.zeros((m, d))
    t0 = time.perf_counter()
    done = 0
    for b0 in range(0, r, batch):
        c += osk.gaussian_block(m, b0, min(r, b0 + batch), seed) @ sa[b0:b0 + batch]
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t["gauss_gemm"] = (time.perf_counter() - t0) * nb / done
    t0 = time.perf_counter()
    og.gram(1.0, a)
    t["gram"] = (time.perf_counter() - t0) * scale
    t0 = time.perf_counter()
    rr = olev.qr_r(c)
    ri = olev.tri_inv(rr)
    t["qr"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    og.rownorms_sq(1.0, a, ri)
    t["rownorms"] = (time.perf_counter() - t0) * scale
    total = sum(t.values())
    sample = (f"first {rows} of {n} rows for S*A, Gram and row norms (times scaled by "
              f"{scale:.0f}); {done} of {nb} Gaussian bucket batches of {batch} timed and "
              f"scaled; QR of the {m} x {d} sketch in full")
    return total, cores, sample, t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true",
                    help="run the serving trace alone and print its record")
    ap.add_argument("--csr-only", action="store_true",
                    help="run the CSR 1e6 x 500 workload alone and print its record "
                         "(hardware-counter runs of the sparse products)")
    ap.add_argument("--no-extras", action="store_true",
                    help="the headline step only (hardware-counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run 4 elementwise copies of MIB MiB "
                         "(FP64) whose HBM bytes are known, to scale hardware FETCH_SIZE / "
                         "WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by rows of A; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
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

    torch.cuda.set_device(0)
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(api, torch)}), flush=True)
        return
    if args.csr_only:
        csr, *_ = csr_workload(api, torch, args.steps, args.warmup, args.seed)
        print(json.dumps({"csr_1e6x500": csr}), flush=True)
        return
    seed = args.seed
    n, d, r, m = HEAD["n"], HEAD["d"], HEAD["r"], HEAD["m"]
    log(f"generating the dense coherent FP32 {n} x {d} matrix on the device")
    A = synth.dense_coherent_torch(n, d, seed=seed, smin=HEAD["smin"], device="cuda:0")
    torch.cuda.synchronize()
    hr = headline(api, torch, A, args.steps, args.warmup, seed)
    rec = {
        "metric": METRIC,
        "value": hr["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "dtype_detail": "FP64 throughout: S*A summed in FP64 from the FP32 entries, G and "
                        "the Gaussian product, Gram, QR and row norms in FP64",
        "data": "synthetic",
        "config": {"workload": "dense-4e6x256", "n": n, "d": d, "a_dtype": "f32",
                   "structure": "singular values geometric 1 .. 1e-6, 5% of rows x100",
                   "r": r, "m": m, "a_bytes": n * d * 4, "parallelism": "single-gpu",
                   "step": "sketch_gcs (f64), sketch_qr, rownorms_sq on one stream, gram "
                           "on a second beside them"},
        "one_stream_ms_per_step": hr["one_stream_ms_per_step"],
        "two_stream_results_identical": hr["two_stream_results_identical"],
        "p50_ms": hr["p50_ms"],
        "p99_ms": hr["p99_ms"],
        "sketch_gcs_gbs": hr["sketch_gcs_gbs"],
        "stage_ms": hr["stage_ms"],
        "scatter_hbm": hr["scatter_hbm"],
        "kernels": hr["kernels"],
        "roofline": hr["roofline"],
    }
    if not args.no_extras:
        log("BF16 / FP8 sketches of the headline matrix and their delta")
        rec["reduced_sketches"] = reduced_sketches(api, torch, A, args.steps, args.warmup, seed)
        log("leverage scores with the JL step")
        rec["leverage_jl"] = leverage_jl(api, torch, A, args.steps, args.warmup, seed)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        tot, cores, sample, parts = cpu_baseline(A, seed)
        rec["cpu_baseline"] = {"value": n * d * 4 / tot / 1e9, "unit": "GB/s", "cores": cores,
                               "kind": "oracle", "sample": sample,
                               "stage_s": {k: round(v, 3) for k, v in parts.items()}}
    del A
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("ceiling probes")
        ceil = api.measure_ceilings("cuda:0")
        rec["ceilings"] = {**ceil, "datasheet": {"hbm_GBs": PEAK_HBM_GBS,
                                                 "fp64_mfma_TFs": PEAK_FP64_TFLOPS,
                                                 "bf16_mfma_TFs": PEAK_BF16_TFLOPS,
                                                 "fp8_mfma_TFs": PEAK_FP8_TFLOPS,
                                                 "valu_Tops": PEAK_VALU_TOPS}}
        log("small dense workload latency")
        rec["small_dense"] = small_latency(api, torch)
        log("sparse workload CSR 1e6 x 500")
        csr, Ac, ac, bc, bdc = csr_workload(api, torch, args.steps, args.warmup, seed)
        csr["gaussian_only"] = gaussian_only(api, torch, Ac, 2000, seed, args.steps, args.warmup)
        csr["direct"] = direct_bench(api, torch, Ac, ac, bc, bdc, 2000, 250_000, seed,
                                     args.steps, args.warmup)
        csr["css"] = css_bench(api, torch, Ac, 500, 250_000, seed, args.steps, args.warmup)
        rec["csr_1e6x500"] = csr
        del Ac, bdc
        torch.cuda.empty_cache()
        log("Zipf CSR 1e7 x 1000 FP32")
        rec["zipf_1e7x1000"] = zipf_workload(api, torch, args.steps, args.warmup, seed)
        torch.cuda.empty_cache()
        log("the paper's tall shape, dense and 5% sparse")
        rec["paper_shape"] = paper_shape(api, torch, args.steps, args.warmup, seed)
    if not args.no_serving:
        rec["serving"] = serving_bench(api, torch)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
