"""FP64 CPU oracle for the BPMF Gibbs sweep -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
Python binding) never imports it, and the two share no code: the oracle's
Philox, Box-Muller, Marsaglia-Tsang, Cholesky, Wishart and Gibbs routines live
in ``bpmf_oracle.c`` and are written out from the mathematics.

What each function follows (Vander Aa, Chakroun, Haber 2017):
  * Sec. I -- R is M x N, U is M x K (users), V is N x K (movies).
  * Sec. II, Algorithm 1 -- sweep order: hyper(V), every movie, hyper(U),
    every user, predict all test points and compute RMSE.
  * Sec. II -- per-item work: K x K matrix/vector operations and one K x K
    factorisation (Cholesky here, no explicit inverse on the row path).
  * BPMF's conjugate conditionals (the model the paper cites in Sec. II) are
    derived in the C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bpmf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Philox stream ids of the noise specification (counter word 2 = stream<<24 | sub).
ROW_U, ROW_V, HYP_U, HYP_V, INIT_U, INIT_V, FOLDIN = 1, 2, 3, 4, 5, 6, 7


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_normals.argtypes = [u64, u32, u32, u32, u32, ctypes.c_int, P]
        L.orc_chi2.argtypes = [u64, u32, u32, u32, dbl, P]
        L.orc_chi2.restype = dbl
        L.orc_cholesky.argtypes = [ctypes.c_int, P]
        L.orc_row_draw_z.argtypes = [ctypes.c_int, dbl, i64, P, P, P, P, P, P, P, P]
        L.orc_update_rows.argtypes = [i64, ctypes.c_int, dbl, P, P, P, P, P, P, u64, u32, u32,
                                      P, i64, P]
        L.orc_hyper_draw.argtypes = [i64, ctypes.c_int, P, P, dbl, dbl, P, u64, u32, u32, P, P]
        L.orc_init_factor.argtypes = [u64, u32, i64, ctypes.c_int, dbl, P]
        L.orc_predict.argtypes = [i64, ctypes.c_int, P, P, P, P, dbl, P]
        L.orc_mean.argtypes = [i64, P]
        L.orc_mean.restype = dbl
        L.orc_foldin.argtypes = [ctypes.c_int, i64, ctypes.c_int, dbl, i64, P, P, P, P, P, u64,
                                 u32, u64, dbl, P, P, P]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


# --------------------------------------------------------------------------
# Noise
# --------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block for a 4-word counter and a 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def normals(seed: int, c0: int, c1: int, stream: int, c3: int, n: int) -> np.ndarray:
    """n Box-Muller normals from blocks (c0, c1, stream<<24 | b, c3)."""
    z = np.zeros(max(n, 1), np.float64)
    lib().orc_normals(seed, c0, c1, stream, c3, n, _p(z))
    return z[:n]


def row_noise(seed: int, stream: int, t: int, row: int, K: int) -> np.ndarray:
    return normals(seed, row, t, stream, 0, K)


def chi2(seed: int, stream: int, t: int, index: int, dof: float):
    """Marsaglia-Tsang chi-square draw; returns (value, attempts)."""
    att = np.zeros(1, np.int32)
    v = lib().orc_chi2(seed, stream, t, index, float(dof), _p(att))
    return v, int(att[0])


# --------------------------------------------------------------------------
# Linear algebra and the row conditional
# --------------------------------------------------------------------------
def cholesky(A) -> np.ndarray:
    L = _f64(A).copy()
    if lib().orc_cholesky(L.shape[0], _p(L)):
        raise np.linalg.LinAlgError("matrix is not SPD")
    return L


def row_draw_z(alpha: float, nbr, rc, Y, mu, Lam, z) -> np.ndarray:
    """Conditional draw of one row with caller-supplied normals z."""
    Y = _f64(Y)
    K = Y.shape[1]
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    rc = _f64(rc)
    mu, Lam, z = _f64(mu), _f64(Lam), _f64(z)
    x = np.zeros(K)
    work = np.zeros(K * K + K)
    if lib().orc_row_draw_z(K, float(alpha), len(nbr), _p(nbr), _p(rc), _p(Y), _p(mu), _p(Lam),
                            _p(z), _p(x), _p(work)):
        raise np.linalg.LinAlgError("row precision not SPD")
    return x


def update_rows(ptr, idx, rc, Y, X, mu, Lam, alpha, seed, stream, t, rows=None) -> None:
    """Draw rows of X (in place) from their neighbour lists against Y."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    rc = _f64(rc)
    Y = _f64(Y)
    assert X.dtype == np.float64 and X.flags.c_contiguous
    mu, Lam = _f64(mu), _f64(Lam)
    K = X.shape[1]
    lst = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    rc_ = lib().orc_update_rows(X.shape[0], K, float(alpha), _p(ptr), _p(idx), _p(rc), _p(Y),
                                _p(mu), _p(Lam), seed, stream, t,
                                None if lst is None else _p(lst),
                                0 if lst is None else len(lst), _p(X))
    if rc_:
        raise np.linalg.LinAlgError("row %d precision not SPD" % (-rc_ - 1))


def hyper_draw(X, mu0, beta0, nu0, W0, seed, stream, t):
    """Normal-Wishart posterior draw (mu, Lambda) from factor X (n x K)."""
    X = _f64(X)
    n, K = X.shape
    mu = np.zeros(K)
    Lam = np.zeros((K, K))
    if lib().orc_hyper_draw(n, K, _p(X), _p(_f64(mu0)), float(beta0), float(nu0), _p(_f64(W0)),
                            seed, stream, t, _p(mu), _p(Lam)):
        raise np.linalg.LinAlgError("hyper draw: matrix not SPD")
    return mu, Lam


def init_factor(seed: int, stream: int, rows: int, K: int) -> np.ndarray:
    X = np.zeros((rows, K))
    lib().orc_init_factor(seed, stream, rows, K, float(K) ** -0.25, _p(X))
    return X


def predict(row, col, U, V, offset: float) -> np.ndarray:
    row = np.ascontiguousarray(row, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    U, V = _f64(U), _f64(V)
    p = np.zeros(len(row))
    lib().orc_predict(len(row), U.shape[1], _p(row), _p(col), _p(U), _p(V), float(offset), _p(p))
    return p


def mean_rating(vals) -> float:
    v = np.ascontiguousarray(vals, dtype=np.float32)
    return float(lib().orc_mean(len(v), _p(v)))


def foldin(alpha, movie, rc, Vs, mus, Lams, seed, req, offset, stream=FOLDIN):
    """Reference fold-in of one new user against S stored samples.

    Returns (U_draws S x K, mean N, var N)."""
    Vs, mus, Lams = _f64(Vs), _f64(mus), _f64(Lams)
    S, N, K = Vs.shape
    movie = np.ascontiguousarray(movie, dtype=np.int32)
    rc = _f64(rc)
    U = np.zeros((S, K))
    mean = np.zeros(N)
    var = np.zeros(N)
    if lib().orc_foldin(S, N, K, float(alpha), len(movie), _p(movie), _p(rc), _p(Vs), _p(mus),
                        _p(Lams), seed, stream, req, float(offset), _p(U), _p(mean), _p(var)):
        raise np.linalg.LinAlgError("fold-in precision not SPD")
    return U, mean, var


def transpose_csr(M: int, N: int, ptr, idx, val):
    """CSR (rows M) -> CSC (rows N) with rows ascending inside each column."""
    ptr = np.asarray(ptr, np.int64)
    rows = np.repeat(np.arange(M, dtype=np.int32), np.diff(ptr))
    order = np.argsort(np.asarray(idx), kind="stable")
    cptr = np.zeros(N + 1, np.int64)
    np.cumsum(np.bincount(idx, minlength=N), out=cptr[1:])
    return cptr, rows[order].astype(np.int32), np.asarray(val)[order]


# --------------------------------------------------------------------------
# Algorithm 1 as a chain of the routines above
# --------------------------------------------------------------------------
class Chain:
    """The Gibbs sampler of Algorithm 1 in FP64.

    Sweep t (t = 1, 2, ...): hyper(V) -> all movies -> hyper(U) -> all users
    -> predict every test pair, keep the running mean of predictions for
    t > burn_in, and report (RMSE of the running mean, RMSE of this sample).
    """

    def __init__(self, M, N, K, csr_ptr, csr_col, csr_val, test_row, test_col, test_val,
                 seed, alpha=2.0, beta0=2.0, nu0=None, mu0=None, W0=None, center=True,
                 burn_in=0, U0=None, V0=None):
        self.M, self.N, self.K = M, N, K
        self.alpha, self.beta0 = float(alpha), float(beta0)
        self.nu0 = float(K if nu0 is None else nu0)
        self.mu0 = np.zeros(K) if mu0 is None else _f64(mu0)
        self.W0 = np.eye(K) if W0 is None else _f64(W0)
        self.seed = int(seed)
        self.burn_in = int(burn_in)
        self.rbar = mean_rating(csr_val) if center else 0.0
        self.csr_ptr = np.asarray(csr_ptr, np.int64)
        self.csr_col = np.asarray(csr_col, np.int32)
        self.csr_rc = np.asarray(csr_val, np.float32).astype(np.float64) - self.rbar
        self.csc_ptr, self.csc_row, csc_val = transpose_csr(M, N, csr_ptr, csr_col, csr_val)
        self.csc_rc = np.asarray(csc_val, np.float32).astype(np.float64) - self.rbar
        self.test_row = np.asarray(test_row, np.int32)
        self.test_col = np.asarray(test_col, np.int32)
        self.test_val = np.asarray(test_val, np.float32).astype(np.float64)
        self.U = init_factor(self.seed, INIT_U, M, K) if U0 is None else _f64(U0).copy()
        self.V = init_factor(self.seed, INIT_V, N, K) if V0 is None else _f64(V0).copy()
        self.pred_sum = np.zeros(len(self.test_row))
        self.n_avg = 0
        self.hyper = {}

    def sweep(self, t: int):
        muV, LamV = hyper_draw(self.V, self.mu0, self.beta0, self.nu0, self.W0, self.seed, HYP_V, t)
        update_rows(self.csc_ptr, self.csc_row, self.csc_rc, self.U, self.V, muV, LamV,
                    self.alpha, self.seed, ROW_V, t)
        muU, LamU = hyper_draw(self.U, self.mu0, self.beta0, self.nu0, self.W0, self.seed, HYP_U, t)
        update_rows(self.csr_ptr, self.csr_col, self.csr_rc, self.V, self.U, muU, LamU,
                    self.alpha, self.seed, ROW_U, t)
        self.hyper = {"V": (muV, LamV), "U": (muU, LamU)}
        return self.evaluate(t)

    def evaluate(self, t: int):
        p = predict(self.test_row, self.test_col, self.U, self.V, self.rbar)
        if t > self.burn_in:
            self.pred_sum += p
            self.n_avg += 1
        rmse_last = float(np.sqrt(np.mean((p - self.test_val) ** 2))) if len(p) else 0.0
        avg = self.pred_sum / self.n_avg if self.n_avg else p
        rmse_avg = float(np.sqrt(np.mean((avg - self.test_val) ** 2))) if len(p) else 0.0
        return rmse_avg, rmse_last

    def run(self, t0: int, n: int):
        return [self.sweep(t) for t in range(t0, t0 + n)]
