#!/usr/bin/env python3
"""Throughput of the BPMF Gibbs sweep (Algorithm 1) on one MI355X.

A step is one full sweep: hyper draw of V, update of every movie, hyper draw
of U, update of every user, prediction of the test set.  The default
workload has the shape of a 20M-rating recommender (M = 138,493 users,
N = 26,744 movies, 20,000,263 ratings, 10% held out, K = 32, FP32), made by
the seeded generators in ``synth``; inputs are resident in HBM before the
timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 (matrix cores), TFLOP/s
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 (matrix cores), TFLOP/s
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s
L2_BYTES = 4 << 20  # one XCD's L2

WORKLOADS = {
    # name: (generator, K, precision)
    "movielens": (synth.movielens_like, 32, "fp32"),
    "netflix": (synth.netflix_like, 100, "fp32"),
    "netflix_mini": (synth.netflix_mini, 100, "fp32"),
    "chembl": (synth.chembl_like, 64, "fp32"),
    "planted": (synth.planted, 10, "fp64"),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic(K, deg, n_low, other_rows, gather_row_bytes, src_bytes):
    """Per-launch algorithmic work of one side's row update (every row).

    Rows that are factorised (all but the n_low of smallest degree): K(K+1) +
    2K FLOP per rating (lower-triangle Gram + rhs) and K^3/3 + 2K^2 per row
    (Cholesky + two triangular solves).  Rows on the rank-one path (degree
    d): 2K d^2 + 12 K d + K^2 FLOP (the d rank-one factors, each applied to the
    later gathered rows, the rhs and the two solves through the d factors,
    and the product with chol(Lambda)^-T), plus K^2 per row of the other side
    for its transform by chol(Lambda)^-1 when the side has such rows.
    Bytes: 8 per rating (neighbour id + rating), the gathered row (K x element
    size) per rating when the gathered factor exceeds one L2, and the written
    row.  Returns (Gram FLOP, factorisation FLOP, bytes)."""
    deg = np.sort(np.asarray(deg, np.int64))  # ascending: the rank-one rows are the first n_low
    low = deg[:n_low].astype(np.float64)
    full = deg[n_low:]
    gram = float(full.sum()) * (K * (K + 1) + 2 * K)
    fact = len(full) * (K ** 3 / 3.0 + 2 * K * K)
    if n_low:
        fact += float((2 * K * low * low + 12 * K * low + K * K).sum()) + float(other_rows) * K * K
    nnz = int(deg.sum())
    gather = gather_row_bytes * nnz if src_bytes > L2_BYTES else 0
    byts = 8 * nnz + gather + 4 * K * len(deg)
    return gram, fact, byts


def side_degrees(r):
    """Degrees of the rows of each side: users (CSR rows) and movies (columns)."""
    return {"U": np.diff(r.csr_ptr), "V": np.bincount(r.csr_col, minlength=r.N)}


PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (matrix cores), TFLOP/s
# The FP32 Gram of the matrix-core kernels (K <= 128) runs on the BF16
# matrix cores as six products of three-part BF16 splits per FP32 product.
P3_PRODUCTS = 6
P3_KMAX = 128


def split_work(K, prec):
    """Whether the Gram and the factorisation are priced apart: the BF16-Gram
    form, and FP32 at K <= 128 (Gram on the BF16 matrix cores); the divisor
    of the BF16 rate for the Gram (products per algorithmic product)."""
    if prec == "bf16":
        return True, 1
    if prec == "fp32" and K <= P3_KMAX:
        return True, P3_PRODUCTS
    return False, 1


def gram_arith(K, prec):
    """How the row kernels form the Gram for this precision and K."""
    if prec == "fp64":
        return "fp64"
    if prec == "bf16":
        return "bf16 products, fp32 accumulation"
    if K <= P3_KMAX:
        return "fp32 as three bf16 parts, six products, fp32 accumulation"
    return "fp32"


GATHER_SOURCES_MB = (3.4, 18.0, 96.0, 192.0)  # one L2, Infinity Cache, HBM-sized sources


def measure_peaks(row_bytes, src_bytes):
    """Peaks measured on this GPU by the library's micro-benchmarks: a stream
    triad (HBM), the FP32 vector and the FP32 / BF16 / FP64 matrix-core
    rates, and random whole-row gathers of `row_bytes` (the gathered factor's
    row, rounded up to 16 B) from sources of the standard sizes and of this
    workload's two factors (`src_bytes`)."""
    import paper_1705_04159_amd as bp

    rb = (row_bytes + 15) // 16 * 16
    out = {
        "hbm_triad_gbs": round(bp.peak_triad(1 << 30, 10), 1),
        "fp32_valu_tflops": round(bp.peak_compute(bp.PEAK_FP32_VALU), 2),
        "fp32_mfma_tflops": round(bp.peak_compute(bp.PEAK_FP32_MFMA), 2),
        "bf16_mfma_tflops": round(bp.peak_compute(bp.PEAK_BF16_MFMA), 1),
        "fp64_mfma_tflops": round(bp.peak_compute(bp.PEAK_FP64_MFMA), 2),
        "gather_row_bytes": rb,
        "gather_gbs": {},
    }
    sizes = sorted(set([int(mb * 1e6) for mb in GATHER_SOURCES_MB] + [int(b) for b in src_bytes]))
    for b in sizes:
        out["gather_gbs"][str(b)] = round(bp.peak_gather(max(b, rb), rb, 1 << 23, 5), 1)
    return out


def sweep_roofline(K, prec, r, ms_per_step, peaks, n_low=None):
    """T_roof of one sweep: the sum over the two sides of
    max(matrix-core time, vector time, memory time) of that side's row
    updates, with the algorithmic work of `algorithmic` for every row and
    rating.  Against the spec sheet (FP32 work at 157.3 TFLOP/s; in the
    BF16-Gram form the Gram at 2.5 PFLOP/s and the factorisation at
    157.3, and the same split for FP32 at K <= 128 with the Gram at 2.5 / 6
    PFLOP/s; bytes at 8 TB/s, the gather counted only when its source exceeds
    one L2) and against the measured peaks (the same split of the work;
    compulsory bytes at the triad rate plus every gathered row at the
    measured gather rate for a source of that factor's size).  The fraction
    is T_roof over the measured sweep time."""
    esize = 8 if prec == "fp64" else (2 if prec == "bf16" else 4)
    ld = K if prec == "fp64" else (K + 3) // 4 * 4
    sides = {"V": (r.N, r.M * ld * esize, r.M), "U": (r.M, r.N * ld * esize, r.N)}
    degs = side_degrees(r)
    n_low = n_low or {}
    res = {"sides": {}}
    tot_spec = tot_meas = 0.0
    for name, (rows, src, other) in sides.items():
        gram, fact, byts = algorithmic(K, degs[name], n_low.get(name, 0), other, ld * esize, src)
        gathered = ld * esize * r.nnz
        compulsory = byts - (gathered if src > L2_BYTES else 0)
        split, nprod = split_work(K, prec)
        if prec == "fp64":
            spec = {"mfma": (gram + fact) / (PEAK_FP64_TFLOPS * 1e12), "valu": 0.0}
        elif split:
            spec = {"mfma": gram * nprod / (PEAK_BF16_TFLOPS * 1e12), "valu": fact / (PEAK_FP32_TFLOPS * 1e12)}
        else:
            spec = {"mfma": (gram + fact) / (PEAK_FP32_TFLOPS * 1e12), "valu": 0.0}
        spec["hbm"] = byts / (PEAK_HBM_GBS * 1e9)
        b_spec = max(spec, key=spec.get)
        side = {"bound_spec": b_spec, "t_spec_ms": round(1e3 * spec[b_spec], 4)}
        tot_spec += spec[b_spec]
        if peaks:
            p32 = max(peaks["fp32_mfma_tflops"], peaks["fp32_valu_tflops"]) * 1e12
            if prec == "fp64":
                meas = {"mfma": (gram + fact) / (peaks["fp64_mfma_tflops"] * 1e12), "valu": 0.0}
            elif split:
                meas = {"mfma": gram * nprod / (peaks["bf16_mfma_tflops"] * 1e12), "valu": fact / p32}
            else:
                meas = {"mfma": (gram + fact) / (peaks["fp32_mfma_tflops"] * 1e12), "valu": 0.0}
            g = peaks["gather_gbs"][str(int(src))]
            meas["memory"] = compulsory / (peaks["hbm_triad_gbs"] * 1e9) + gathered / (g * 1e9)
            b_meas = max(meas, key=meas.get)
            side.update({"bound_measured": b_meas, "t_measured_ms": round(1e3 * meas[b_meas], 4),
                         "gather_gbs": g})
            tot_meas += meas[b_meas]
        res["sides"][name] = side
    res["t_roof_ms_spec"] = round(1e3 * tot_spec, 4)
    res["frac_spec"] = round(1e3 * tot_spec / ms_per_step, 4)
    if peaks:
        res["t_roof_ms_measured"] = round(1e3 * tot_meas, 4)
        res["frac_measured"] = round(1e3 * tot_meas / ms_per_step, 4)
    return res


FIG2_DEGREES = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192)
# kernel family: (split threshold, fast_kmax, rank-one cut-off, applies to degree d)
FIG2_VARIANTS = {
    "rank-one (VALU)": (1 << 24, 32, 16, lambda d: d <= 16),
    "MFMA, column-per-lane factorisation": (1 << 24, 32, 0, lambda d: True),
    "MFMA, blocked factorisation": (1 << 24, 0, 0, lambda d: True),
    "split into segments of 128": (128, 32, 0, lambda d: d > 128),
}


def uniform_degree(d, N, n_rows, seed):
    """n_rows users with exactly d distinct ratings each over N movies
    (start + 7919 j mod N: distinct for d <= N, as 7919 is prime to N)."""
    import types

    rng = np.random.default_rng(seed)
    start = rng.integers(0, N, n_rows)
    cols = (start[:, None] + 7919 * np.arange(d, dtype=np.int64)[None, :]) % N
    cols.sort(axis=1)
    n_test = 1000
    return types.SimpleNamespace(
        name="uniform-degree-%d" % d, M=n_rows, N=N, nnz=n_rows * d,
        csr_ptr=np.arange(n_rows + 1, dtype=np.int64) * d, csr_col=cols.ravel().astype(np.int32),
        csr_val=(3.5 + rng.standard_normal(n_rows * d)).astype(np.float32),
        test_row=rng.integers(0, n_rows, n_test).astype(np.int32),
        test_col=rng.integers(0, N, n_test).astype(np.int32),
        test_val=np.full(n_test, 3.5, np.float32))


def fit_fixed_plus_per_rating(d, t):
    """Least-squares fit of t = a + b d in relative error (each point weighted
    by 1 / t), the paper's per-item cost model (a fixed cost plus a cost per
    rating).  Returns (a, b)."""
    d, t = np.asarray(d, np.float64), np.asarray(t, np.float64)
    A = np.stack([1.0 / t, d / t], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, np.ones_like(t), rcond=None)
    return float(a), float(b)


def fig2_per_degree(K, N, seed, max_ratings=16_000_000):
    """Per-row cost of each kernel family against the row's degree (users of
    one degree each, the gathered factor V of the 20M shape's size), from the
    eager U-side phases (row kernel + split finishing) of three sweeps; then
    the fixed + per-rating fit of each family."""
    import paper_1705_04159_amd as bp

    res = {"K": K, "N": N, "degrees": list(FIG2_DEGREES), "rows": [], "ns_per_row": {}, "fit": {}}
    for v in FIG2_VARIANTS:
        res["ns_per_row"][v] = []
    for d in FIG2_DEGREES:
        n_rows = max(8192, min(262144, max_ratings // d))
        r = uniform_degree(d, N, n_rows, seed + d)
        s = bp.Sampler(r, K, prec="fp32", seed=seed)
        t = 1
        res["rows"].append(n_rows)
        for v, (split, kmax, low, applies) in FIG2_VARIANTS.items():
            if not applies(d):
                res["ns_per_row"][v].append(None)
                continue
            s.set_plan(split, kmax, low)
            s.run_sweeps(t, 2)
            ph = s.profile_sweeps(t + 2, 3)
            t += 5
            ms = float(ph[4] + ph[5])  # rows_U + split_U
            res["ns_per_row"][v].append(round(1e6 * ms / n_rows, 2))
        s.close()
        log("fig2 d=%d rows=%d: %s" % (d, n_rows, {v: res["ns_per_row"][v][-1] for v in FIG2_VARIANTS}))
    for v in FIG2_VARIANTS:
        pts = [(d, x) for d, x in zip(FIG2_DEGREES, res["ns_per_row"][v]) if x is not None]
        a, b = fit_fixed_plus_per_rating([p[0] for p in pts], [p[1] for p in pts])
        res["fit"][v] = {"fixed_ns": round(a, 2), "per_rating_ns": round(b, 4)}
    return res


def profiled_traffic(workload, K, prec, side):
    """HBM bytes per launch of the row kernel from the committed rocprofv3
    counter summaries (FETCH_SIZE and WRITE_SIZE, each scaled by the same
    counter on a copy of known size), or None when no summary covers this
    workload or a source file of the kernel changed since it was taken."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md"))):
        for line in open(path):
            if not line.startswith("traffic-json: "):
                continue
            rec = json.loads(line[len("traffic-json: "):])
            if (rec["workload"], rec["K"], rec["prec"], rec["side"]) != (workload, K, prec, side):
                continue
            h = hashlib.sha256()
            for f in rec["sources"]:
                h.update(open(os.path.join(ROOT, f), "rb").read())
            if h.hexdigest() != rec["sources_sha256"]:
                return None
            return int(rec["fetch_bytes"] + rec["write_bytes"])
    return None


def kernel_roofline(K, prec, r, k_ms, peaks, n_low, steps):
    """Roofline of the dominant kernel: the row update of the side that takes
    longer per launch (every kernel of that side's update, timed inside the
    timed sweeps), with its algorithmic FLOP and bytes per launch against
    the peak of its own arithmetic (FP32 matrix cores; in the BF16-Gram form
    the Gram at the BF16 peak and the factorisation at the FP32 one,
    time-weighted; for FP32 at K <= 128 the same with the Gram at a sixth of
    the BF16 peak) or HBM, whichever bound is higher; also against the peaks
    measured on this GPU, and the HBM traffic of the committed counter
    summary for this workload and side (None if there is none or the
    kernel's sources changed since)."""
    esize = 8 if prec == "fp64" else (2 if prec == "bf16" else 4)
    ld = K if prec == "fp64" else (K + 3) // 4 * 4
    degs = side_degrees(r)
    cand = {
        "rows_V": algorithmic(K, degs["V"], n_low.get("V", 0), r.M, ld * esize, r.M * ld * esize),
        "rows_U": algorithmic(K, degs["U"], n_low.get("U", 0), r.N, ld * esize, r.N * ld * esize),
    }
    dom = max(cand, key=lambda n: k_ms[n])
    gram, fact, byts = cand[dom]
    flops = gram + fact
    sec = k_ms[dom] / 1000.0
    peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
    split, nprod = split_work(K, prec)
    if split:
        peak = flops / (gram * nprod / PEAK_BF16_TFLOPS + fact / PEAK_FP32_TFLOPS)
    t_mfma = flops / (peak * 1e12)
    t_hbm = byts / (PEAK_HBM_GBS * 1e9)
    if t_hbm > t_mfma:
        roof = {"bound": "hbm", "achieved": round(byts / sec / 1e9, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": round(flops / sec / 1e12, 3), "peak": round(peak, 1),
                "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    if peaks:
        if roof["bound"] == "hbm":
            src = (r.M if dom == "rows_V" else r.N) * ld * esize
            gathered = ld * esize * r.nnz
            t_meas = ((byts - gathered) / (peaks["hbm_triad_gbs"] * 1e9)
                      + gathered / (peaks["gather_gbs"][str(int(src))] * 1e9))
            roof["peak_measured"] = round(byts / t_meas / 1e9, 1)
        else:
            p32 = peaks["fp32_mfma_tflops"]
            pm = p32
            if split:
                pm = flops / (gram * nprod / peaks["bf16_mfma_tflops"]
                              + fact / max(p32, peaks["fp32_valu_tflops"]))
            elif prec == "fp64":
                pm = peaks["fp64_mfma_tflops"]
            roof["peak_measured"] = round(pm, 2)
        roof["frac_measured"] = round(roof["achieved"] / roof["peak_measured"], 4)
    roof["flop_per_launch"] = round(flops)
    roof["bytes_per_launch"] = int(byts)
    roof["traffic"] = profiled_traffic(r.name, K, prec, dom[-1])
    roof["kernel"] = ("row update, side %s (every kernel of the side's update; mean of %d "
                      "sweeps in the timed region, %.4f ms)" % (dom[-1], steps, k_ms[dom]))
    return roof


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(r, K, seconds, seed):
    """The FP64 oracle timed on this host on a bounded sample of the same
    workload: random rows of both sides (in proportion M : N), updated with
    the oracle's row routine, first on one thread for a quarter of `seconds`,
    then on all host cores for the rest."""
    import oracle

    oracle.build()
    rng = np.random.default_rng(seed)
    ch = oracle.Chain(r.M, r.N, K, r.csr_ptr, r.csr_col, r.csr_val, r.test_row[:1],
                      r.test_col[:1], r.test_val[:1], seed=seed)
    mu, lam = np.zeros(K), np.eye(K) * K
    order = rng.permutation(r.M + r.N)
    cores = oracle.max_threads()

    def run(budget, start, batch):
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            q = (start + done) % len(order)
            sweep = 1 + (start + done) // len(order)
            sel = order[q:q + batch]
            u = sel[sel < r.M]
            v = sel[sel >= r.M] - r.M
            if len(v):
                oracle.update_rows(ch.csc_ptr, ch.csc_row, ch.csc_rc, ch.U, ch.V, mu, lam, 2.0, seed,
                                   oracle.ROW_V, sweep, rows=v)
            if len(u):
                oracle.update_rows(ch.csr_ptr, ch.csr_col, ch.csr_rc, ch.V, ch.U, mu, lam, 2.0, seed,
                                   oracle.ROW_U, sweep, rows=u)
            done += len(sel)
        return done, time.perf_counter() - t0

    oracle.set_threads(1)
    d1, e1 = run(0.25 * seconds, 0, 32)
    oracle.set_threads(cores)
    done, el = run(0.75 * seconds, d1, 512)
    return {"value": done / el, "unit": "row-updates/s", "cores": cores,
            "kind": "oracle",
            "one_thread_value": round(d1 / e1, 1),
            "cpu_model": cpu_model(),
            "sample": "%d row draws (FP64) over random rows of both sides of the same workload "
                      "(%d rows per sweep) on %d threads in %.1f s, after %d on one thread in %.1f s" % (
                          done, r.M + r.N, cores, el, d1, e1)}


def foldin_requests(r, n_req, seed, max_n=5000):
    """Synthetic new users: sizes log-uniform on [1, max_n], movies drawn by
    training popularity without repetition, ratings N(mean, 1) clipped to the
    training range (the values only matter for the arithmetic, not the load)."""
    rng = np.random.default_rng(seed)
    pop = np.bincount(r.csr_col, minlength=r.N).astype(np.float64) + 1.0
    cdf = np.cumsum(pop / pop.sum())
    lo, hi = float(r.csr_val.min()), float(r.csr_val.max())
    mu = float(r.csr_val.mean())
    sizes = np.minimum(np.round(np.exp(rng.uniform(0.0, np.log(max_n), n_req))).astype(np.int64),
                       r.N - 1)
    reqs = []
    for n in sizes:
        got = np.zeros(0, np.int64)
        while len(got) < n:
            draw = np.minimum(np.searchsorted(cdf, rng.random(int(1.3 * (n - len(got))) + 8)), r.N - 1)
            _, first = np.unique(np.concatenate([got, draw]), return_index=True)
            got = np.concatenate([got, draw])[np.sort(first)]
        movie = got[:n].astype(np.int32)
        rating = np.clip(rng.normal(mu, 1.0, n), lo, hi).astype(np.float32)
        reqs.append((movie, rating))
    return reqs, sizes


def foldin_bench(s, r, rate, seconds, seed, top_n=100, warm_seconds=0.0):
    """Open-loop Poisson arrivals at `rate` req/s for `warm_seconds` +
    `seconds`; latency is completion (seen by the scheduler) minus the
    scheduled arrival time, reported over the requests that arrive after the
    first `warm_seconds`."""
    rng = np.random.default_rng(seed + 1)
    n_req = int(rate * (seconds + warm_seconds))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    # at most 50,000 distinct requests, submitted cyclically on longer runs
    uniq, usizes = foldin_requests(r, min(n_req, 50000), seed)
    sizes = usizes[np.arange(n_req) % len(uniq)]
    # requests converted once, so that the submit loop itself keeps up
    # with the offered rate
    prep = [s.foldin_prepare(movie, rating) for movie, rating in uniq]
    # warm the path (first batch allocations, kernel loads)
    for i in range(min(8, len(prep))):
        s.foldin_submit_prepared(prep[i], top_n)
    s.foldin_drain()
    lag = np.zeros(n_req)
    ids = np.zeros(n_req, np.uint64)
    submit, clock, nu = s.foldin_submit_prepared, time.perf_counter, len(prep)
    t0 = clock()
    for i in range(n_req):
        a = arrivals[i]
        now = clock() - t0
        while now < a:
            if a - now > 2e-4:
                time.sleep(min(a - now - 1e-4, 1e-3))
            now = clock() - t0
        lag[i] = now - a
        ids[i] = submit(prep[i % nu], top_n)
    s.foldin_drain()
    t_end = time.perf_counter() - t0
    lat = np.zeros(n_req)
    for i in range(n_req):
        res = s.foldin_poll(int(ids[i]), top_n)
        lat[i] = res[3] + lag[i]
    keep = arrivals >= warm_seconds
    lat, sizes = lat[keep], sizes[keep]
    return {
        "offered_req_per_s": rate,
        "completed_req_per_s": round(n_req / t_end, 1),
        "n_requests": int(keep.sum()),
        "warmup_s": warm_seconds,
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "p999_ms": round(1e3 * float(np.percentile(lat, 99.9)), 3),
        "mean_ratings_per_request": round(float(sizes.mean()), 1),
        "samples": s.foldin_samples(),
        "top_n": top_n,
    }


def timed_config(r, K, prec, steps, seed, autotune=True, with_peaks=True, warm=2, reorder=False):
    """One workload in one precision: measured peaks (optional), autotuned
    plan (outside the timed region), `warm` warm-up sweeps, then `steps`
    timed sweeps of the sweep graph (wall clock around them, device idle on
    both sides); reports throughput, held-out RMSE, the row-update time per
    side measured inside the timed sweeps, the dominant kernel's roofline and
    the sweep roofline."""
    import paper_1705_04159_amd as bp

    peaks = None
    esize = 8 if prec == "fp64" else (2 if prec == "bf16" else 4)
    ld = K if prec == "fp64" else (K + 3) // 4 * 4
    if with_peaks:
        peaks = measure_peaks(ld * esize, (r.M * ld * esize, r.N * ld * esize))
    s = bp.Sampler(r, K, prec=prec, seed=seed, reorder=reorder)
    plan = None
    if autotune:
        split, kmax, low, tried = s.autotune(3)
        plan = {"split_threshold": split, "fast_kmax": kmax, "lowrank_dmax": low,
                "tried": [[a, b, c_, round(m, 4)] for a, b, c_, m in tried]}
    s.run_sweeps(1, warm)  # warm-up with the timed plan
    s.synchronize()
    t0 = time.perf_counter()
    avg, last = s.run_sweeps(warm + 1, steps)
    s.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    kv, ku = s.row_kernel_ms()
    k_ms = {"rows_V": kv, "rows_U": ku}
    n_low = {"U": s.lowrank_rows(bp.SIDE_U), "V": s.lowrank_rows(bp.SIDE_V)}
    s.close()
    return {"ms_per_step": round(ms, 3), "row_updates_per_s": round((r.M + r.N) / ms * 1e3, 1),
            "ratings_per_s": round(2 * r.nnz / ms * 1e3, 1),
            "rmse_avg": round(float(avg[-1]), 5), "rmse_last": round(float(last[-1]), 5),
            "row_kernel_ms": {"rows_V": round(kv, 3), "rows_U": round(ku, 3)},
            "lowrank_rows": n_low, "autotune": plan, "reorder": bool(reorder),
            "roofline": kernel_roofline(K, prec, r, k_ms, peaks, n_low, steps),
            "sweep_roofline": sweep_roofline(K, prec, r, ms, peaks, n_low),
            "peaks_measured": peaks}


def k100_compare(steps, seed, autotune=True, with_peaks=True, reorder=False, reorder_ab=False):
    """The 100M-rating shape at K = 100: the same chain (same seed, same
    Philox draws) in FP32 and in the BF16-Gram form, `steps` timed sweeps
    each after two warm-up sweeps; reports throughput and the held-out RMSE
    of both, and their ratio.  reorder: both contexts hold users and movies
    in degree order; reorder_ab: also time each precision in the other order
    (the reordering's effect on the gather-bound sides, same GPU)."""
    t = time.perf_counter()
    r = synth.netflix_like()
    log("generated %s: M=%d N=%d nnz=%d in %.1fs" % (r.name, r.M, r.N, r.nnz, time.perf_counter() - t))
    out = {"workload": r.name, "M": r.M, "N": r.N, "nnz_train": r.nnz, "K": 100, "steps": steps}
    for prec in ("fp32", "bf16"):
        out[prec] = timed_config(r, 100, prec, steps, seed, autotune, with_peaks, reorder=reorder)
        log("K=100 %s: %s" % (prec, {k: v for k, v in out[prec].items() if k != "peaks_measured"}))
        if reorder_ab:
            o = timed_config(r, 100, prec, steps, seed, autotune, False, reorder=not reorder)
            a, b = (o, out[prec]) if reorder else (out[prec], o)
            out[prec + "_order_ab"] = {
                "reordered": o["reorder"], "ms_per_step": o["ms_per_step"],
                "row_kernel_ms": o["row_kernel_ms"], "rmse_avg": o["rmse_avg"],
                "reordered_over_caller_order": {
                    "sweep": round(b["ms_per_step"] / a["ms_per_step"], 4),
                    "rows_V": round(b["row_kernel_ms"]["rows_V"] / a["row_kernel_ms"]["rows_V"], 4),
                    "rows_U": round(b["row_kernel_ms"]["rows_U"] / a["row_kernel_ms"]["rows_U"], 4)}}
            log("K=100 %s order A/B: %s" % (prec, out[prec + "_order_ab"]))
    out["bf16_speedup"] = round(out["fp32"]["ms_per_step"] / out["bf16"]["ms_per_step"], 3)
    out["rmse_avg_rel_diff"] = round(out["bf16"]["rmse_avg"] / out["fp32"]["rmse_avg"] - 1.0, 6)
    return out


def chembl_compare(steps, seed, autotune=True, with_peaks=True, reorder=False):
    """The compound x protein shape (483,500 x 5,775, 2,000,000 observations,
    20 columns holding 30%), K = 64, FP32: `steps` timed sweeps after the
    autotuner and two warm-up sweeps."""
    t = time.perf_counter()
    r = synth.chembl_like()
    log("generated %s: M=%d N=%d nnz=%d in %.1fs" % (r.name, r.M, r.N, r.nnz, time.perf_counter() - t))
    out = {"workload": r.name, "M": r.M, "N": r.N, "nnz_train": r.nnz, "K": 64, "precision": "fp32",
           "steps": steps}
    out.update(timed_config(r, 64, "fp32", steps, seed, autotune, with_peaks, reorder=reorder))
    log("compound x protein: %s" % {k: v for k, v in out.items() if k != "peaks_measured"})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="movielens", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--seed", type=int, default=102)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--foldin-rate", type=float, default=5000.0)
    ap.add_argument("--foldin-seconds", type=float, default=10.0)
    ap.add_argument("--foldin-warmup-seconds", type=float, default=2.0)
    ap.add_argument("--foldin-sweep", default="1000,2500,10000,20000,40000,80000,160000,240000",
                    help="offered loads (req/s) of the 1-s load sweep, comma separated; empty: none")
    ap.add_argument("--no-foldin", action="store_true")
    ap.add_argument("--k100-steps", type=int, default=50,
                    help="sweeps of the K = 100 comparison (100M-rating shape, FP32 vs BF16-Gram)")
    ap.add_argument("--no-k100", action="store_true")
    ap.add_argument("--chembl-steps", type=int, default=50,
                    help="sweeps of the compound x protein comparison (K = 64, FP32)")
    ap.add_argument("--no-chembl", action="store_true")
    ap.add_argument("--fig2", action="store_true",
                    help="only time each kernel family per row against the row's degree (K = 32, "
                         "N = 26,744) and fit the fixed + per-rating cost model; one JSON line")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the micro-benchmarks of the measured peaks")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default split threshold and kernel family")
    ap.add_argument("--plan", default=None, metavar="SPLIT,KMAX,LOWD",
                    help="fix the plan (split threshold, fast-kernel K cut-off, rank-one degree "
                         "cut-off) instead of autotuning, e.g. to profile the plan a timed run chose")
    ap.add_argument("--reorder", action=argparse.BooleanOptionalAction, default=True,
                    help="hold users and movies in descending degree order inside every context "
                         "(the library's reorder parameter; --no-reorder keeps the generator's order)")
    ap.add_argument("--k100-reorder-ab", action="store_true",
                    help="also time the K = 100 configurations in the other row order")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (torch), the "
                         "reference kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        n = args.copy_calibration << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.fig2:
        print(json.dumps({"fig2": fig2_per_degree(32, 26744, args.seed)}), flush=True)
        return

    import paper_1705_04159_amd as bp

    gen, K, prec = WORKLOADS[args.workload]
    prec = args.prec or prec
    t = time.perf_counter()
    r = gen()
    log("generated %s: M=%d N=%d nnz=%d test=%d in %.1fs" % (r.name, r.M, r.N, r.nnz,
                                                             len(r.test_row), time.perf_counter() - t))
    esize = 8 if prec == "fp64" else (2 if prec == "bf16" else 4)
    ld = K if prec == "fp64" else (K + 3) // 4 * 4
    peaks = None
    if not args.no_peaks:
        t = time.perf_counter()
        peaks = measure_peaks(ld * esize, (r.M * ld * esize, r.N * ld * esize))
        log("measured peaks (%.1fs): %s" % (time.perf_counter() - t, peaks))
    t = time.perf_counter()
    s = bp.Sampler(r, K, prec=prec, seed=args.seed, reorder=args.reorder)
    log("created context in %.1fs" % (time.perf_counter() - t))
    steps, warm = args.steps, args.warmup
    tuned = None
    if args.plan:
        split, kmax, low = (int(x) for x in args.plan.split(","))
        s.set_plan(split, kmax, low)
        tuned = {"split_threshold": split, "fast_kmax": kmax, "lowrank_dmax": low, "tried": "fixed"}
        log("plan fixed: split %d, kmax %d, low %d" % (split, kmax, low))
    elif not args.no_autotune:
        t = time.perf_counter()
        split, kmax, low, tried = s.autotune(5)
        tuned = {"split_threshold": split, "fast_kmax": kmax, "lowrank_dmax": low,
                 "tried": [[a, b, c_, round(m, 4)] for a, b, c_, m in tried]}
        log("autotune (%.1fs): split %d, kmax %d, low %d; tried %s" % (
            time.perf_counter() - t, split, kmax, low, tuned["tried"]))
    # the warm-up sweeps run right before the timed ones (the GPU's clocks
    # settle under load), with the plan that is timed
    if warm > 0:
        s.run_sweeps(1, warm)
        log("warmup %d sweeps done" % warm)
    s.synchronize()
    t0 = time.perf_counter()
    avg, last = s.run_sweeps(warm + 1, steps)  # returns after the stream is drained
    s.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = s.last_time_ms()
    ms_per_step = 1000.0 * wall / steps
    rows = r.M + r.N
    value = rows / (ms_per_step / 1000.0)
    log("timed %d sweeps: %.3f ms/sweep wall (%.3f device), rmse avg %.4f last %.4f" % (
        steps, ms_per_step, dev_ms / steps, avg[-1], last[-1]))

    # per-phase device times (eager launches bracketed by HIP events)
    pn = max(1, min(args.profile_steps, 64))
    ph = s.profile_sweeps(warm + steps + 1, pn)
    names = ["hyper_V", "rows_V", "split_V", "hyper_U", "rows_U", "split_U", "predict"]
    phase = {n: round(float(v), 4) for n, v in zip(names, ph)}
    log("phases (ms): %s" % phase)
    # row-kernel launch time measured inside the timed sweeps (HIP events on
    # the kernel's stream, one pair per replay)
    k_ms = dict(zip(["rows_V", "rows_U"], s.row_kernel_ms()))
    log("row kernel per launch (ms, timed sweeps): %s" % {k: round(v, 4) for k, v in k_ms.items()})
    # the timed stage of a side is its whole row update (every row finished)
    n_low = {"U": s.lowrank_rows(bp.SIDE_U), "V": s.lowrank_rows(bp.SIDE_V)}
    roof = kernel_roofline(K, prec, r, k_ms, peaks, n_low, steps)
    out = {
        "metric": "Gibbs row-updates/s",
        "value": round(value, 1),
        "unit": "row-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16-gram/f32"}[prec],
        "data": "synthetic",
        "config": {"workload": r.name, "M": r.M, "N": r.N, "nnz_train": r.nnz,
                   "n_test": int(len(r.test_row)), "K": K, "precision": prec,
                   "gram": gram_arith(K, prec), "reorder": bool(args.reorder),
                   "parallelism": "single-gpu"},
        "ratings_per_s": round(2 * r.nnz / (ms_per_step / 1000.0), 1),
        "rmse_avg": round(float(avg[-1]), 5),
        "rmse_last": round(float(last[-1]), 5),
        "phase_ms": phase,
        "row_kernel_ms": {k: round(v, 4) for k, v in k_ms.items()},
        "autotune": tuned,
        "roofline": roof,
        "sweep_roofline": sweep_roofline(K, prec, r, ms_per_step, peaks, n_low),
        "lowrank_rows": n_low,
        "peaks_measured": peaks,
    }
    if not args.no_foldin and prec == "fp32" and K <= 64:
        # 16 posterior samples from the running chain, then open-loop serving
        t = warm + steps + pn + 1
        for _ in range(16):
            s.run_sweeps(t, 1)
            t += 1
            s.store_sample()
        out["foldin"] = foldin_bench(s, r, args.foldin_rate, args.foldin_seconds, args.seed,
                                     warm_seconds=args.foldin_warmup_seconds)
        log("fold-in: %s" % out["foldin"])
        # offered-load sweep (1 s each) to locate the knee
        knee = []
        for rate in [float(x) for x in args.foldin_sweep.split(",") if x.strip()]:
            f = foldin_bench(s, r, rate, 1.0, args.seed + int(rate))
            knee.append({k: f[k] for k in ("offered_req_per_s", "completed_req_per_s", "p50_ms",
                                           "p99_ms")})
        out["foldin"]["load_sweep"] = knee
        log("fold-in load sweep: %s" % knee)
    s.close()
    if not args.no_k100 and args.workload == "movielens":
        out["k100"] = k100_compare(args.k100_steps, args.seed, not args.no_autotune, not args.no_peaks,
                                   args.reorder, args.k100_reorder_ab)
    if not args.no_chembl and args.workload == "movielens":
        out["chembl"] = chembl_compare(args.chembl_steps, args.seed, not args.no_autotune,
                                       not args.no_peaks, args.reorder)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(r, K, args.cpu_seconds, args.seed)
        log("cpu baseline: %s" % out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
