"""Shared test helpers: drop rules from workloads, GPU availability, comparisons."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import spai_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

# tolerances stated for the hot path: ||I - A M||_F relative, FP64 and mixed paths
TOL_F64 = 1e-10
TOL_MIXED = 1e-5


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not gpu_available():
        pytest.fail("GPU test run without a GPU")


def oracle_rule(A, mode, value, relative, symmetrize=True):
    if mode == "global":
        return O.DropRule(mode="global", m=O.cap_counts(A, "global", value, relative),
                          symmetrize=symmetrize)
    if mode == "column":
        return O.DropRule(mode="column", k=O.cap_counts(A, "column", value, relative),
                          symmetrize=symmetrize)
    return O.DropRule(mode="none", symmetrize=symmetrize)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def pattern_diff(Mg, Mo):
    """Entries stored in exactly one of the two matrices: (only_gpu, only_oracle) sets."""
    g = sp.csr_matrix(Mg).tocoo()
    o = sp.csr_matrix(Mo).tocoo()
    sg = set(zip(g.row.tolist(), g.col.tolist()))
    so = set(zip(o.row.tolist(), o.col.tolist()))
    return sg - so, so - sg


def value_err(Mg, Mo):
    D = sp.csr_matrix(Mg) - sp.csr_matrix(Mo)
    scale = max(abs(sp.csr_matrix(Mo)).max(), 1e-300)
    return (abs(D).max() if D.nnz else 0.0) / scale
