"""Python binding of libbpmf.so: the MI355X (gfx950) BPMF Gibbs sampler.

Argument marshalling only: every step of the sampler (hyperparameter draw,
row updates, prediction) runs in the library's HIP kernels.  The binding
refuses to work without the built library -- there is no CPU fallback.

Names follow the paper (Vander Aa, Chakroun, Haber 2017): R is M x N
(users x movies), U is M x K, V is N x K; Algorithm 1 alternates a hyper
draw and an update of every movie, then of every user, then predicts the
test points.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbpmf.so")

SIDE_U, SIDE_V = 0, 1
FP64, FP32, BF16_GRAM = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16_GRAM, "bf16_gram": BF16_GRAM}

OK, PENDING = 0, 1
E_INVAL, E_RANGE, E_FORMAT, E_NOMEM, E_DEVICE = -1, -2, -3, -4, -5
E_BUSY, E_TOOBIG, E_NOSAMPLES, E_NOTFOUND, E_NOTSPD = -6, -7, -8, -9, -10

# Every symbol the C ABI exports (include/bpmf.h).
EXPORTS = [
    "bpmf_default_params", "bpmf_create", "bpmf_sample_hyper", "bpmf_update_side",
    "bpmf_run_sweeps", "bpmf_profile_sweeps", "bpmf_predict", "bpmf_predict_noalloc",
    "bpmf_get_factor", "bpmf_set_factor",
    "bpmf_get_factor_f64", "bpmf_set_factor_f64", "bpmf_get_hyper", "bpmf_set_hyper",
    "bpmf_get_csc", "bpmf_get_chain_state", "bpmf_set_chain_state", "bpmf_get_plan",
    "bpmf_mean_rating", "bpmf_synchronize",
    "bpmf_last_time_ms", "bpmf_row_kernel_ms", "bpmf_autotune", "bpmf_set_plan", "bpmf_last_error", "bpmf_destroy", "bpmf_store_sample",
    "bpmf_foldin_submit", "bpmf_foldin_poll", "bpmf_foldin_drain", "bpmf_foldin_samples",
    "bpmf_foldin_capacity", "bpmf_foldin_stats",
    # include/bpmf_peaks.h
    "bpmf_peak_triad", "bpmf_peak_compute", "bpmf_peak_gather",
]

PEAK_FP32_VALU, PEAK_FP32_MFMA, PEAK_BF16_MFMA, PEAK_FP64_MFMA = 0, 1, 2, 3


class BPMFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("bpmf status %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("beta0", ctypes.c_double),
        ("nu0", ctypes.c_double),
        ("mu0", ctypes.c_void_p),
        ("W0", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("center", ctypes.c_int32),
        ("burn_in", ctypes.c_int32),
        ("foldin_S", ctypes.c_int32),
        ("split_threshold", ctypes.c_int32),
        ("foldin_pool_bytes", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("reorder", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libbpmf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbpmf.so is not built (run `python -m paper_1705_04159_amd.build`); "
                              "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_double)
        L.bpmf_default_params.argtypes = [P, i32]
        L.bpmf_default_params.restype = None
        L.bpmf_create.argtypes = [i64, i64, P, P, P, P, P, P, i64, P, P, P, i64, P, P]
        L.bpmf_sample_hyper.argtypes = [P, i32, u32]
        L.bpmf_update_side.argtypes = [P, i32, u32]
        L.bpmf_run_sweeps.argtypes = [P, u32, u32, P, P]
        L.bpmf_predict.argtypes = [P, u32, i64, P, P, P, P, P]
        L.bpmf_predict_noalloc.argtypes = [P, i64, P, P, P]
        L.bpmf_profile_sweeps.argtypes = [P, u32, u32, P]
        for name in ("bpmf_get_factor", "bpmf_set_factor", "bpmf_get_factor_f64",
                     "bpmf_set_factor_f64"):
            getattr(L, name).argtypes = [P, i32, P]
        L.bpmf_get_hyper.argtypes = [P, i32, P, P]
        L.bpmf_set_hyper.argtypes = [P, i32, P, P]
        L.bpmf_get_csc.argtypes = [P, P, P, P]
        L.bpmf_get_chain_state.argtypes = [P, P, P]
        L.bpmf_set_chain_state.argtypes = [P, P, u32]
        L.bpmf_get_plan.argtypes = [P, i32, P, P, P]
        L.bpmf_mean_rating.argtypes = [P]
        L.bpmf_mean_rating.restype = dbl
        L.bpmf_synchronize.argtypes = [P]
        L.bpmf_last_time_ms.argtypes = [P, P]
        L.bpmf_row_kernel_ms.argtypes = [P, P]
        L.bpmf_autotune.argtypes = [P, ctypes.c_uint32, P, P, P, P, P, P, P, P]
        L.bpmf_set_plan.argtypes = [P, i32, i32, i32]
        L.bpmf_last_error.argtypes = [P]
        L.bpmf_last_error.restype = ctypes.c_char_p
        L.bpmf_destroy.argtypes = [P]
        L.bpmf_destroy.restype = None
        L.bpmf_store_sample.argtypes = [P]
        L.bpmf_foldin_submit.argtypes = [P, i32, P, P, i32, P]
        L.bpmf_foldin_poll.argtypes = [P, ctypes.c_uint64, P, P, P, P]
        L.bpmf_foldin_drain.argtypes = [P]
        L.bpmf_foldin_samples.argtypes = [P]
        L.bpmf_foldin_capacity.argtypes = [P]
        L.bpmf_foldin_capacity.restype = i64
        L.bpmf_foldin_stats.argtypes = [P, P, P, P, P]
        L.bpmf_peak_triad.argtypes = [i64, i32, P]
        L.bpmf_peak_compute.argtypes = [i32, i32, P]
        L.bpmf_peak_gather.argtypes = [i64, i32, i64, i32, P]
        _lib = L
    return _lib


def _peak_check(rc, what):
    if rc != OK:
        raise RuntimeError("%s failed with status %d" % (what, rc))


def peak_triad(bytes_per_array=1 << 30, reps=10):
    """HBM rate of a stream triad over three arrays on the current GPU, GB/s."""
    v = ctypes.c_double()
    _peak_check(lib().bpmf_peak_triad(int(bytes_per_array), int(reps), ctypes.byref(v)), "bpmf_peak_triad")
    return v.value


def peak_compute(kind, reps=5):
    """Dense rate of one instruction kind (PEAK_*) on the current GPU, TFLOP/s."""
    v = ctypes.c_double()
    _peak_check(lib().bpmf_peak_compute(int(kind), int(reps), ctypes.byref(v)), "bpmf_peak_compute")
    return v.value


def peak_gather(src_bytes, row_bytes, n_rows=1 << 23, reps=5):
    """Rate of random whole-row gathers of `row_bytes` from a `src_bytes`
    source on the current GPU, GB/s."""
    v = ctypes.c_double()
    _peak_check(lib().bpmf_peak_gather(int(src_bytes), int(row_bytes), int(n_rows), int(reps),
                                       ctypes.byref(v)), "bpmf_peak_gather")
    return v.value


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class Sampler:
    """One BPMF Gibbs chain resident on the current GPU.

    ratings: an object with M, N, csr_ptr, csr_col, csr_val, test_row,
    test_col, test_val (e.g. ``synth.Ratings``)."""

    def __init__(self, ratings, K, prec="fp32", alpha=2.0, beta0=2.0, nu0=None, mu0=None,
                 W0=None, seed=0, center=True, burn_in=0, split_threshold=0, csc=None,
                 foldin_S=16, foldin_pool_bytes=0, stream=None, reorder=False):
        L = lib()
        self.M, self.N, self.K = int(ratings.M), int(ratings.N), int(K)
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        p = Params()
        L.bpmf_default_params(ctypes.byref(p), self.K)
        p.prec = self.prec
        p.alpha, p.beta0 = float(alpha), float(beta0)
        p.nu0 = float(K if nu0 is None else nu0)
        self._mu0 = _c(mu0, np.float64)
        self._W0 = _c(W0, np.float64)
        p.mu0 = None if self._mu0 is None else self._mu0.ctypes.data
        p.W0 = None if self._W0 is None else self._W0.ctypes.data
        p.seed = int(seed)
        p.center = 1 if center else 0
        p.burn_in = int(burn_in)
        p.split_threshold = int(split_threshold)
        p.foldin_S = int(foldin_S)
        p.foldin_pool_bytes = int(foldin_pool_bytes)
        p.stream = None if stream is None else int(stream)  # a hipStream_t handle
        p.reorder = 1 if reorder else 0
        ptr = _c(ratings.csr_ptr, np.int64)
        col = _c(ratings.csr_col, np.int32)
        val = _c(ratings.csr_val, np.float32)
        tr = _c(ratings.test_row, np.int32)
        tc = _c(ratings.test_col, np.int32)
        tv = _c(ratings.test_val, np.float32)
        cp = cr = cv = None
        if csc is not None:
            cp, cr, cv = _c(csc[0], np.int64), _c(csc[1], np.int32), _c(csc[2], np.float32)
        self.nnz = int(ptr[-1])
        self.n_test = len(tr)
        ctx = ctypes.c_void_p()
        rc = L.bpmf_create(self.M, self.N, _ptr(ptr), _ptr(col), _ptr(val), _ptr(cp), _ptr(cr),
                           _ptr(cv), self.nnz, _ptr(tr), _ptr(tc), _ptr(tv), self.n_test,
                           ctypes.byref(p), ctypes.byref(ctx))
        if rc != OK:
            raise BPMFError(rc, L.bpmf_last_error(None).decode())
        self._ctx = ctx

    # -- plumbing --------------------------------------------------------
    def _check(self, rc):
        if rc not in (OK, PENDING):
            raise BPMFError(rc, lib().bpmf_last_error(self._ctx).decode())
        return rc

    def close(self):
        if getattr(self, "_ctx", None):
            lib().bpmf_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def rows(self, side):
        return self.M if side == SIDE_U else self.N

    @property
    def dtype(self):
        return np.float64 if self.prec == FP64 else np.float32

    # -- Algorithm 1 -------------------------------------------------------
    def sample_hyper(self, side, t):
        self._check(lib().bpmf_sample_hyper(self._ctx, side, t))

    def update_side(self, side, t):
        self._check(lib().bpmf_update_side(self._ctx, side, t))

    def run_sweeps(self, t0, n):
        avg = np.zeros(n)
        last = np.zeros(n)
        self._check(lib().bpmf_run_sweeps(self._ctx, t0, n, _ptr(avg), _ptr(last)))
        return avg, last

    def profile_sweeps(self, t0, n):
        """Eager sweeps with per-phase HIP events; returns the mean ms per sweep
        of (hyper V, rows V, split-finish V, hyper U, rows U, split-finish U,
        predict)."""
        out = np.zeros(7)
        self._check(lib().bpmf_profile_sweeps(self._ctx, t0, n, _ptr(out)))
        return out

    def predict_test(self, t):
        a = ctypes.c_double()
        b = ctypes.c_double()
        self._check(lib().bpmf_predict(self._ctx, t, 0, None, None, None, ctypes.byref(a),
                                       ctypes.byref(b)))
        return a.value, b.value

    def predict(self, row, col):
        row = _c(row, np.int32)
        col = _c(col, np.int32)
        out = np.zeros(len(row), np.float32)
        if len(row):
            self._check(lib().bpmf_predict(self._ctx, 0, len(row), _ptr(row), _ptr(col), _ptr(out),
                                           None, None))
        return out

    def predict_noalloc(self, row, col):
        """predict() through the entry point that allocates no device memory
        (at most 524,288 pairs per call)."""
        row = _c(row, np.int32)
        col = _c(col, np.int32)
        out = np.zeros(len(row), np.float32)
        self._check(lib().bpmf_predict_noalloc(self._ctx, len(row), _ptr(row), _ptr(col), _ptr(out)))
        return out

    # -- state -------------------------------------------------------------
    def get_factor(self, side):
        X = np.zeros((self.rows(side), self.K), self.dtype)
        self._check(lib().bpmf_get_factor(self._ctx, side, _ptr(X)))
        return X

    def set_factor(self, side, X):
        X = _c(X, self.dtype)
        assert X.shape == (self.rows(side), self.K)
        self._check(lib().bpmf_set_factor(self._ctx, side, _ptr(X)))

    def get_hyper(self, side):
        mu = np.zeros(self.K)
        Lam = np.zeros((self.K, self.K))
        self._check(lib().bpmf_get_hyper(self._ctx, side, _ptr(mu), _ptr(Lam)))
        return mu, Lam

    def set_hyper(self, side, mu, Lam):
        mu = _c(mu, np.float64)
        Lam = _c(Lam, np.float64)
        self._check(lib().bpmf_set_hyper(self._ctx, side, _ptr(mu), _ptr(Lam)))

    def get_chain_state(self):
        """(running sum of test predictions in the caller's pair order, number
        of sweeps in it)."""
        ps = np.zeros(self.n_test)
        n = ctypes.c_uint32()
        self._check(lib().bpmf_get_chain_state(self._ctx, _ptr(ps), ctypes.byref(n)))
        return ps, n.value

    def set_chain_state(self, pred_sum, n_avg):
        ps = _c(pred_sum, np.float64)
        assert ps.shape == (self.n_test,)
        self._check(lib().bpmf_set_chain_state(self._ctx, _ptr(ps), int(n_avg)))

    def get_csc(self):
        ptr = np.zeros(self.N + 1, np.int64)
        row = np.zeros(self.nnz, np.int32)
        rc = np.zeros(self.nnz, self.dtype)
        self._check(lib().bpmf_get_csc(self._ctx, _ptr(ptr), _ptr(row), _ptr(rc)))
        return ptr, row, rc

    def get_plan(self, side):
        perm = np.zeros(self.rows(side), np.int32)
        ns = ctypes.c_int64()
        self._check(lib().bpmf_get_plan(self._ctx, side, _ptr(perm), ctypes.byref(ns), None))
        return perm, ns.value

    def set_plan(self, split_threshold, fast_kmax, lowrank_dmax):
        """Fix the split threshold, kernel family cut-off and rank-one cut-off
        by hand (what autotune() would choose)."""
        self._check(lib().bpmf_set_plan(self._ctx, int(split_threshold), int(fast_kmax),
                                        int(lowrank_dmax)))

    def lowrank_rows(self, side):
        """Number of rows of `side` on the rank-one-update path."""
        nl = ctypes.c_int64()
        self._check(lib().bpmf_get_plan(self._ctx, side, None, None, ctypes.byref(nl)))
        return nl.value

    @property
    def mean_rating(self):
        return float(lib().bpmf_mean_rating(self._ctx))

    def synchronize(self):
        self._check(lib().bpmf_synchronize(self._ctx))

    # -- fold-in serving ------------------------------------------------------
    def store_sample(self):
        self._check(lib().bpmf_store_sample(self._ctx))

    def foldin_samples(self):
        return int(lib().bpmf_foldin_samples(self._ctx))

    def foldin_submit(self, movie, rating, top_n=100):
        movie = _c(movie, np.int32)
        rating = _c(rating, np.float32)
        rid = ctypes.c_uint64()
        self._check(lib().bpmf_foldin_submit(self._ctx, len(movie), _ptr(movie), _ptr(rating),
                                             int(top_n), ctypes.byref(rid)))
        return rid.value

    def foldin_prepare(self, movie, rating):
        """A request's arrays converted once for foldin_submit_prepared (for
        load generators that submit faster than per-call conversion allows)."""
        movie = _c(movie, np.int32)
        rating = _c(rating, np.float32)
        return (movie, rating, len(movie), _ptr(movie), _ptr(rating))

    def foldin_submit_prepared(self, prepared, top_n=100):
        """foldin_submit on foldin_prepare's result."""
        rid = ctypes.c_uint64()
        rc = lib().bpmf_foldin_submit(self._ctx, prepared[2], prepared[3], prepared[4], top_n,
                                      ctypes.byref(rid))
        if rc:
            self._check(rc)
        return rid.value

    def foldin_poll(self, req_id, top_n=100):
        """None while pending, else (movie ids, mean, var, latency seconds)."""
        ids = np.zeros(top_n, np.int32)
        mean = np.zeros(top_n, np.float32)
        var = np.zeros(top_n, np.float32)
        lat = ctypes.c_double()
        rc = lib().bpmf_foldin_poll(self._ctx, req_id, _ptr(ids), _ptr(mean), _ptr(var),
                                    ctypes.byref(lat))
        if rc == PENDING:
            return None
        self._check(rc)
        return ids, mean, var, lat.value

    def foldin_stats(self):
        """(batches launched, requests launched, most requests in one batch,
        most batches on the device at once)."""
        nb, nr = ctypes.c_int64(), ctypes.c_int64()
        mb, mi = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().bpmf_foldin_stats(self._ctx, ctypes.byref(nb), ctypes.byref(nr),
                                            ctypes.byref(mb), ctypes.byref(mi)))
        return nb.value, nr.value, mb.value, mi.value

    def foldin_capacity(self):
        return int(lib().bpmf_foldin_capacity(self._ctx))

    def foldin_drain(self):
        self._check(lib().bpmf_foldin_drain(self._ctx))

    def last_time_ms(self):
        ms = ctypes.c_double()
        self._check(lib().bpmf_last_time_ms(self._ctx, ctypes.byref(ms)))
        return ms.value

    def autotune(self, n_sweeps=3):
        """Time candidate plans (split threshold, kernel family, rank-one
        cut-off) on this context's data and keep the fastest; the chain state
        is unchanged.  Returns (split, kmax, low, [(split, kmax, low, ms), ...])."""
        sp, km, lo, nt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ts = (ctypes.c_int32 * 64)()
        tk = (ctypes.c_int32 * 64)()
        tl = (ctypes.c_int32 * 64)()
        tm = (ctypes.c_double * 64)()
        self._check(lib().bpmf_autotune(self._ctx, n_sweeps, ctypes.byref(sp), ctypes.byref(km),
                                        ctypes.byref(lo), ctypes.byref(nt), ts, tk, tl, tm))
        return sp.value, km.value, lo.value, [(ts[i], tk[i], tl[i], tm[i]) for i in range(nt.value)]

    def row_kernel_ms(self):
        """Mean per-launch device time (ms) of the row kernel of each side over
        the replays of the last run_sweeps call: (V side, U side)."""
        ms = (ctypes.c_double * 2)()
        self._check(lib().bpmf_row_kernel_ms(self._ctx, ms))
        return float(ms[0]), float(ms[1])
