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


# ----------------------------------------------------------------------------
# handle state buffers (spai_get_state layout: header, per-matrix scalars, lists as CSC)
# ----------------------------------------------------------------------------

_HDR = "<8sii q iiiiii qq 5q"     # StateHeader, natural alignment (104 bytes)
_SEG_BYTES = 152                  # sizeof(SegState)


def parse_state(buf):
    """Split a state buffer into its header fields and lists [(colptr, idx, val), ...]
    (lists: M, then P and P^T for CG and LOMR, then R)."""
    import struct
    hsz = struct.calcsize(_HDR)
    f = struct.unpack_from(_HDR, buf, 0)
    hd = {"value_bytes": f[2], "n": f[3], "nseg": f[4], "method": f[5], "nlists": f[9],
          "iters_host": f[10], "nnz": list(f[12:17])}
    n = hd["n"]
    vt = np.float32 if hd["value_bytes"] == 4 else np.float64
    o = hsz + _SEG_BYTES * hd["nseg"]
    lists, offs = [], []
    for l in range(hd["nlists"]):
        nz = hd["nnz"][l]
        cp = np.frombuffer(buf, dtype=np.int64, count=n + 1, offset=o)
        offs.append(o)
        o += 8 * (n + 1)
        ix = np.frombuffer(buf, dtype=np.int32, count=nz, offset=o)
        o += 4 * nz
        vl = np.frombuffer(buf, dtype=vt, count=nz, offset=o)
        o += vt().itemsize * nz
        lists.append((cp, ix, vl))
    hd["list_offsets"] = offs
    return hd, lists


def state_matrix(lst, n):
    """A state list as a float64 CSC matrix."""
    cp, ix, vl = lst
    return sp.csc_matrix((vl.astype(np.float64), ix.copy(), cp.copy()), shape=(n, n))


def history_from_oracle(ref):
    """The oracle's per-iteration drop record in spai_history's layout (iters x 6)."""
    rows = []
    for d in ref.drops:
        m, p = d["M"], d["P"]
        rows.append([m["kept"], m["cand"] - m["kept"], m["band"],
                     p["kept"] if p else 0, (p["cand"] - p["kept"]) if p else 0,
                     p["band"] if p else 0])
    return np.array(rows, dtype=np.int64).reshape(-1, 6)


def history_array(h):
    """spai_history of a handle as an (iters x 6) array."""
    d = h.history()
    names = ["nnz_m", "dropped_m", "band_m", "nnz_p", "dropped_p", "band_p"]
    return np.stack([d[k] for k in names], axis=1) if len(d["nnz_m"]) else np.zeros((0, 6), np.int64)


def far_from_cut(entries, info, eta, rtol):
    """The entries (a set of (row, col)) whose oracle candidate magnitude lies farther
    than rtol (relative) from its keep threshold thr (1 + eta), or that were not a
    candidate at all: a pattern difference there is not explained by the rounding of
    the candidate values near the cut."""
    rows, cols, vals, thr = info["candidates"]
    pos = {(int(r), int(c)): i for i, (r, c) in enumerate(zip(rows, cols))}
    bad = []
    for e in entries:
        i = pos.get(e)
        if i is None or thr is None:
            bad.append(e)
            continue
        cut = thr[i] * (1.0 + eta)
        if not abs(abs(vals[i]) - cut) <= rtol * cut:
            bad.append(e)
    return bad
