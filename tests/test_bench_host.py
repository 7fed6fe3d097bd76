"""Host-side pieces of bench.py (no GPU): the algorithmic work per launch,
the sweep roofline against the spec sheet, the per-degree inputs and the
fixed + per-rating cost fit."""
import os
import sys
import types

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_algorithmic_work_per_launch():
    # K = 2: per rating K(K+1) + 2K = 10 FLOP, per row K^3/3 + 2K^2 FLOP;
    # 9 rows with 100 ratings in all
    deg = np.array([30, 20, 20, 10, 10, 5, 5, 0, 0])
    gram, fact, byts = bench.algorithmic(2, deg, 0, 1000, 8, 1 << 30)
    assert gram == 1000
    assert abs(fact - 9 * (8 / 3 + 8)) < 1e-12
    assert byts == 8 * 100 + 8 * 100 + 4 * 2 * 9  # ids+ratings, gathered rows (source > L2), written rows
    _, _, b_small = bench.algorithmic(2, deg, 0, 1000, 8, 1 << 10)  # source fits L2: no gather bytes
    assert b_small == 8 * 100 + 4 * 2 * 9
    # the 4 rows of smallest degree (0, 0, 5, 5) on the rank-one path: no Gram or
    # factorisation for them, 2K d^2 + 12 K d + K^2 each, plus K^2 per row of the
    # other side (1000 rows) for the transform
    gram, fact, byts = bench.algorithmic(2, deg, 4, 1000, 8, 1 << 30)
    assert gram == 90 * 10
    low = 2 * 4 + 2 * (2 * 2 * 25 + 12 * 2 * 5 + 4)
    assert abs(fact - (5 * (8 / 3 + 8) + low + 1000 * 4)) < 1e-9
    assert byts == 8 * 100 + 8 * 100 + 4 * 2 * 9


def test_sweep_roofline_spec_terms():
    """The 20M shape at K = 32: the V side (gathering a 17.7 MB U) is bound by
    HBM, the U side by the matrix cores (its FP32 Gram as six BF16 products
    per FP32 product: 20.2 GFLOP x 6 at 2.5 PFLOP/s, 48 us); the sum is
    about 0.355 ms."""
    r = types.SimpleNamespace(M=138493, N=26744, nnz=18000237,
                              csr_ptr=np.linspace(0, 18000237, 138494).astype(np.int64),
                              csr_col=np.arange(18000237, dtype=np.int64) % 26744)
    res = bench.sweep_roofline(32, "fp32", r, 1.0, None)
    assert res["sides"]["V"]["bound_spec"] == "hbm" and res["sides"]["U"]["bound_spec"] == "mfma"
    assert 0.047 < res["sides"]["U"]["t_spec_ms"] < 0.05
    assert 0.34 < res["t_roof_ms_spec"] < 0.37
    assert res["frac_spec"] == res["t_roof_ms_spec"]
    # BF16-Gram at K = 100: V side HBM-bound, U side bound by the FP32 factorisation
    r = types.SimpleNamespace(M=480189, N=17770, nnz=90432457,
                              csr_ptr=np.linspace(0, 90432457, 480190).astype(np.int64),
                              csr_col=np.arange(90432457, dtype=np.int32) % 17770)
    res = bench.sweep_roofline(100, "bf16", r, 10.0, None)
    assert res["sides"]["V"]["bound_spec"] == "hbm" and res["sides"]["U"]["bound_spec"] == "valu"


def test_uniform_degree_rows():
    r = bench.uniform_degree(300, 26744, 50, 3)
    cols = r.csr_col.reshape(50, 300)
    assert (np.diff(cols, axis=1) > 0).all()  # sorted, distinct
    assert cols.min() >= 0 and cols.max() < 26744
    assert r.nnz == 15000 and r.csr_ptr[-1] == 15000


def test_fixed_plus_per_rating_fit():
    d = np.array([1, 2, 4, 8, 64, 512, 4096], np.float64)
    a, b = bench.fit_fixed_plus_per_rating(d, 120.0 + 0.35 * d)
    assert abs(a - 120.0) < 1e-9 and abs(b - 0.35) < 1e-12
    # noisy data: the relative-error fit keeps the small-degree points
    rng = np.random.default_rng(0)
    t = (120.0 + 0.35 * d) * (1 + 0.01 * rng.standard_normal(len(d)))
    a, b = bench.fit_fixed_plus_per_rating(d, t)
    assert abs(a / 120.0 - 1) < 0.05 and abs(b / 0.35 - 1) < 0.05
