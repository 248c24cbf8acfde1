"""The allocation-free forward loss (spai_loss_fwd_noalloc) against the allocating
spai_loss_fwd, through the C ABI: two calls in a row on one GPU, the second with a
smaller input, each bitwise equal to the allocating entry point and within 1e-12 of
the oracle's loss; sizes beyond the scratch and host inputs are refused."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import spai_oracle as O
from paper_2511_09753_amd import workloads as W
from tests.helpers import require_gpu

pytestmark = pytest.mark.gpu

SPAI_ERR_ARG = -1            # include/spai.h status codes


def _dev_csr(S, torch, X):
    X = sp.csr_matrix(X)
    rp = torch.from_numpy(np.ascontiguousarray(X.indptr, dtype=np.int64)).cuda()
    ci = torch.from_numpy(np.ascontiguousarray(X.indices, dtype=np.int32)).cuda()
    va = torch.from_numpy(np.ascontiguousarray(X.data, dtype=np.float64)).cuda()
    return S.CsrT(X.shape[0], X.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), 1), (rp, ci, va)


def test_loss_fwd_noalloc_matches_allocating_entry_point():
    require_gpu()
    import torch
    from paper_2511_09753_amd import spai as S
    lib = S.load()
    f = lib.spai_loss_fwd_noalloc
    f.argtypes = [C.POINTER(S.CsrT), C.POINTER(S.CsrT), C.c_void_p, C.c_void_p,
                  C.POINTER(S.OptsT)]
    f.restype = C.c_int
    opts = S.Options().c()
    L_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    err = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    for N, seed in ((96, 41), (40, 42)):          # the second call is smaller
        A = W.grid9(N, seed)
        M = W.loss_m_values(A, W.square_pattern(A), seed + 1)
        cA, keepA = _dev_csr(S, torch, A)
        cM, keepM = _dev_csr(S, torch, M)
        want = O.loss(A, M)
        ref = C.c_double()
        assert lib.spai_loss_fwd(C.byref(cA), C.byref(cM), C.byref(ref), C.byref(opts)) == S.SPAI_OK
        rc = f(C.byref(cA), C.byref(cM), L_dev.data_ptr(), err.data_ptr(), C.byref(opts))
        torch.cuda.synchronize()
        assert rc == S.SPAI_OK, S.load().spai_last_error()
        assert int(err.item()) == 0
        got = float(L_dev.item())
        print(N, got, ref.value, want)
        assert got == ref.value                    # same kernels, same summation order
        assert abs(got - want) <= 1e-12 * want
    # refused before any launch: too many rows for the scratch, host inputs, mixed values
    big = S.CsrT(cA.n, cA.nnz, cA.rowptr, cA.colind, cA.val, 1)
    big.n = (1 << 21) + 1
    assert f(C.byref(big), C.byref(big), L_dev.data_ptr(), err.data_ptr(), C.byref(opts)) == SPAI_ERR_ARG
    host = S.CsrT(cA.n, cA.nnz, cA.rowptr, cA.colind, cA.val, 0)
    assert f(C.byref(host), C.byref(cM), L_dev.data_ptr(), err.data_ptr(), C.byref(opts)) == SPAI_ERR_ARG
    mixed = S.Options(precision="mixed").c()
    assert f(C.byref(cA), C.byref(cM), L_dev.data_ptr(), err.data_ptr(), C.byref(mixed)) == SPAI_ERR_ARG
    del keepA, keepM
