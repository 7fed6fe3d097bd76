"""Degree-order relabelling of a ratings problem in numpy, for the tests:
users and movies renumbered by descending rating count, ties by id (the
reordering of R before partitioning, Sec. IV-B), written independently of
the library's own relabelling."""
import numpy as np

import synth


def relabel(r):
    """Returns the relabelled Ratings and, per side, ext (ext[new] = old id)
    and inv (inv[old] = new id): (r2, ext_u, ext_v, inv_u, inv_v)."""
    M, N = r.M, r.N
    du = np.diff(r.csr_ptr)
    dv = np.bincount(r.csr_col, minlength=N)
    ou = np.lexsort((np.arange(M), -du)).astype(np.int32)
    ov = np.lexsort((np.arange(N), -dv)).astype(np.int32)
    iu = np.empty(M, np.int32)
    iu[ou] = np.arange(M, dtype=np.int32)
    iv = np.empty(N, np.int32)
    iv[ov] = np.arange(N, dtype=np.int32)
    rows = iu[r.coo_rows()]
    cols = iv[r.csr_col]
    o = np.argsort(rows.astype(np.int64) * N + cols)  # (row, column) keys are distinct
    ptr = np.zeros(M + 1, np.int64)
    ptr[1:] = np.cumsum(np.bincount(rows, minlength=M))
    r2 = synth.Ratings(r.name + "-relabelled", M, N, ptr, cols[o].astype(np.int32),
                       r.csr_val[o], iu[r.test_row], iv[r.test_col], r.test_val, r.K)
    return r2, ou, ov, iu, iv
