"""The numpy relabelling the GPU tests compare the library's reorder option
against (CPU only): it must be exactly P R Q^T with users and movies in
descending degree order, ties by id, and a valid CSR."""
import numpy as np
import pytest
import scipy.sparse

import synth
from relabel import relabel


@pytest.mark.parametrize("r", [synth.planted(seed=21, M=1200, N=700, nnz=30000, K=10),
                               synth.random_small(22, 400, 300, 6000, 8, empty_rows=9)],
                         ids=["planted", "empty-rows"])
def test_relabel_is_degree_ordered_permutation(r):
    r2, ou, ov, iu, iv = relabel(r)
    M, N = r.M, r.N
    assert np.array_equal(np.sort(ou), np.arange(M)) and np.array_equal(np.sort(ov), np.arange(N))
    assert np.array_equal(iu[ou], np.arange(M)) and np.array_equal(iv[ov], np.arange(N))
    A = scipy.sparse.csr_matrix((r.csr_val, r.csr_col, r.csr_ptr), shape=(M, N))
    B = scipy.sparse.csr_matrix((r2.csr_val, r2.csr_col, r2.csr_ptr), shape=(M, N))
    assert (A[ou][:, ov] != B).nnz == 0
    # valid CSR: columns strictly increasing within each row
    for i in range(M):
        assert np.all(np.diff(r2.csr_col[r2.csr_ptr[i]:r2.csr_ptr[i + 1]]) > 0)
    # degrees descend, ties by the old id
    du, dv = np.diff(r.csr_ptr), np.bincount(r.csr_col, minlength=N)
    for d, o in ((du, ou), (dv, ov)):
        assert np.all(np.diff(d[o]) <= 0)
        same = np.diff(d[o]) == 0
        assert np.all(np.diff(o)[same] > 0)
    # test pairs keep their order and values
    assert np.array_equal(ou[r2.test_row], r.test_row) and np.array_equal(ov[r2.test_col], r.test_col)
    assert np.array_equal(r2.test_val, r.test_val)
