"""Host-side logic of bench.py: the byte accounting behind its GB/s figures, the
traffic-profile lookup, and the one-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _counts(iters):
    # per iteration: R 42, kept M/P/PT 14, candidates M 42, P and PT 56 entries per column
    # of a 100-column problem, accumulated over `iters` iterations as the device counters are
    per = {"resid": 4200, "kept_m": 1400, "kept_p": 1400, "kept_pt": 1400,
           "cand_m": 4200, "cand_p": 5600, "cand_pt": 5600}
    return {k: v * iters for k, v in per.items()}


def test_whole_iteration_bytes_by_hand():
    # E(X) = nnz (s + 4) + 8 (n + 1) with s = 4: E(A) = 700*8 + 808 = 6408,
    # E(R) = 4200*8 + 808 = 34408, E(P) = E(M) = 1400*8 + 808 = 12008
    c = _counts(10)
    EA, ER, EP, EM = 6408, 34408, 12008, 12008
    assert bench.lomr_alg_bytes(c, 100, 700, 4, 4, 10) == pytest.approx(2 * EA + 3 * ER + 3 * EP + 3 * EM)
    assert bench.lomr_alg_bytes(c, 100, 700, 4, 4, 10, with_p=False) == pytest.approx(2 * EA + 3 * ER + 3 * EM)
    assert bench.state_min_bytes(c, 100, 700, 4, 4, 10) == pytest.approx(EA + 2 * EM + 2 * EP)
    # float64 values: every entry is 12 bytes instead of 8
    assert bench.state_min_bytes(c, 100, 700, 8, 8, 10) == pytest.approx(
        (700 * 12 + 808) + 2 * (1400 * 12 + 808) + 2 * (1400 * 12 + 808))


def test_phase_bytes_by_hand():
    c = _counts(4)
    n, nnzA = 100, 700
    e, col, EA = 8, 1200, 700 * 8 + 808
    alg = bench.algorithmic_bytes(c, n, nnzA, 4, 4, 4)
    assert alg["dots"] == pytest.approx((4200 + 1400) * e + 2 * col + EA + 48 * n)
    assert alg["resid"] == pytest.approx(1400 * e + col + EA + 4200 * e + col + 8 * n)
    assert alg["update"] == pytest.approx((1400 + 4200 + 1400 + 1400) * e + 4 * col + EA
                                          + (4200 + 5600 + 5600) * e + 3 * col)
    assert alg["compact"] == pytest.approx((4200 + 5600 + 5600) * e + (1400 * 3) * e + 6 * col)


def test_traffic_lookup_needs_a_matching_profile():
    # a kernel with no committed profile reports no traffic
    assert bench.measured_traffic("no_such_kernel") is None
    # the committed profiles name the source file hash they were taken on; each
    # reported figure is positive
    for k in ("k_update_lean", "k_dots_lean", "k_resid_lean", "k_spmm_pair_mx", "k_spmm_pair_ax"):
        t = bench.measured_traffic(k)
        assert t is None or t > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_state_lists_parses_the_state_layout():
    """bench.state_lists reads the documented spai_get_state layout: a 104-byte header,
    152 bytes of scalars per matrix, then each list as CSC (int64 pointers, int32 rows,
    values of value_bytes)."""
    import struct
    import numpy as np
    import bench
    n = 3
    lists = [(np.array([0, 1, 3, 4]), np.array([0, 0, 2, 1]), np.array([1.5, -2.0, 0.25, 3.0])),
             (np.array([0, 0, 1, 1]), np.array([2]), np.array([7.0]))]
    for vb, vt in ((8, np.float64), (4, np.float32)):
        hdr = struct.pack("<8sii q iiiiii qq 5q", b"SPAISTAT", 1, vb, n, 1, 2, 0, 0, 1, 2, 5, 5,
                          4, 1, 0, 0, 0)
        buf = hdr + bytes(152)
        for cp, ix, vl in lists:
            buf += cp.astype("<i8").tobytes() + ix.astype("<i4").tobytes() + vl.astype(vt).tobytes()
        got = bench.state_lists(buf)
        assert len(got) == 2
        for G, (cp, ix, vl) in zip(got, lists):
            assert np.array_equal(G.indptr, cp) and np.array_equal(G.indices, ix)
            assert np.array_equal(G.data, vl.astype(vt).astype(np.float64))


def test_state_parsers_agree():
    """The tests' parse_state and bench.state_lists read the same header fields."""
    import struct
    import numpy as np
    import bench
    from tests.helpers import parse_state
    cp, ix, vl = np.array([0, 2, 2]), np.array([0, 1]), np.array([1.0, 2.0])
    hdr = struct.pack("<8sii q iiiiii qq 5q", b"SPAISTAT", 1, 8, 2, 1, 0, 0, 0, 1, 1, 7, 9,
                      2, 0, 0, 0, 0)
    buf = hdr + bytes(152) + cp.astype("<i8").tobytes() + ix.astype("<i4").tobytes() + \
        vl.astype("<f8").tobytes()
    hd, lists = parse_state(buf)
    assert hd["nlists"] == 1 and hd["iters_host"] == 7 and hd["nnz"][0] == 2 and hd["n"] == 2
    assert np.array_equal(lists[0][1], ix)
    assert np.array_equal(bench.state_lists(buf)[0].toarray(), np.array([[1.0, 0.0], [2.0, 0.0]]))
