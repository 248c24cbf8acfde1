"""Write the stored expected values of the full-size parity tests.

Calls only the CPU oracle (and the seeded input generators); nothing here comes from
the HIP library.  Usage: python tests/golden/make_golden.py [aniso256] [lognormal96]
Output: tests/golden/<name>.json with, per method, the residual history
||I - A M_i||_F (i = 0..iters), nnz(M_i), nnz(P_i), the step sizes, the per-iteration
record of the drop rule (candidates, kept, tie band, global cut) and SHA-256 digests of
the final patterns of M and P (CSC, rows ascending in each column).
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import spai_oracle as O                      # noqa: E402
from paper_2511_09753_amd import workloads as W           # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def pattern_digest(X):
    """SHA-256 of a sparse pattern: CSC column pointers (int64) then row indices (int32),
    little-endian, rows ascending within each column."""
    import numpy as np
    import scipy.sparse as sp
    C = sp.csc_matrix(X)
    C.sort_indices()
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(C.indptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(C.indices, dtype="<i4").tobytes())
    return h.hexdigest()


def record(res):
    return {
        "resid": res.resid,
        "nnz_m": res.nnz_m,
        "nnz_p": res.nnz_p,
        "iters": res.iters,
        "status": res.status,
        "steps": [{k: v for k, v in s.items() if isinstance(v, float)} for s in res.scalars],
        "drops": res.drops,
        "pattern_m": pattern_digest(res.M),
        "pattern_p": pattern_digest(res.P) if res.P is not None else None,
    }


def run(name, methods):
    wl = W.workload(name)
    A = wl.A
    if wl.cap_mode == "global":
        rule = O.DropRule(mode="global", m=O.cap_counts(A, "global", wl.cap_value, wl.cap_relative))
    else:
        rule = O.DropRule(mode="column", k=O.cap_counts(A, "column", wl.cap_value, wl.cap_relative))
    out = {"workload": name, "n": A.shape[0], "nnz": A.nnz, "iters": wl.iters,
           "cap_mode": wl.cap_mode, "cap_value": wl.cap_value, "cap_relative": wl.cap_relative,
           "methods": {}}
    for m in methods:
        t = time.time()
        res = O.run(m, A, rule, wl.iters)
        out["methods"][m] = record(res)
        print(name, m, f"{time.time() - t:.1f}s", res.resid[-1], flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["aniso256", "lognormal96"]
    if "aniso256" in todo:
        run("aniso256", ["mr", "cg", "lomr"])
    if "lognormal96" in todo:
        run("lognormal96", ["lomr"])
