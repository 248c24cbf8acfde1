"""The C ABI without a GPU: the library loads, exports every declared entry point,
and rejects bad inputs on the host before touching the device."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from tests.helpers import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "spai.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def S():
    from paper_2511_09753_amd import spai as S
    if not os.path.exists(S.LIB_PATH):
        from paper_2511_09753_amd import build
        build.build()
    S.load()
    return S


def test_exports_every_declared_symbol(S):
    names = _declared()
    assert len(names) >= 13
    lib = S.load()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(S.EXPORTS)


def test_status_strings(S):
    lib = S.load()
    assert lib.spai_status_string(0) == b"SPAI_OK"
    assert lib.spai_status_string(-2) == b"SPAI_ERR_NOT_SYMMETRIC"


def _expect(S, code, fn):
    with pytest.raises(S.SpaiError) as e:
        fn()
    assert e.value.code == code


def test_host_side_errors(S):
    A = sp.csr_matrix(np.array([[2.0, 1.0], [0.5, 2.0]]))
    _expect(S, -2, lambda: S.SPAI(A, "mr"))                            # not symmetric
    B = sp.csr_matrix(np.array([[-1.0, 0.0], [0.0, 2.0]]))
    _expect(S, -3, lambda: S.SPAI(B, "mr"))                            # not SPD diagonal
    Cm = sp.csr_matrix(np.array([[2.0, np.nan], [np.nan, 2.0]]))
    _expect(S, -4, lambda: S.SPAI(Cm, "mr"))                           # non-finite
    D = sp.identity(4, format="csr") * 2.0
    _expect(S, -1, lambda: S.SPAI(D, "mr", "global", 3, False))        # cap below diagonal count
    _expect(S, -1, lambda: S.SPAI(D, "mr", "column", 0.2, False))      # column cap below one
    _expect(S, -1, lambda: S.SPAI(D, "lomr", "global", 0.0, False))


def test_degenerate_shapes_and_options(S):
    E = sp.csr_matrix((0, 0))
    _expect(S, -1, lambda: S.SPAI(E, "mr"))                            # empty matrix
    D = sp.identity(4, format="csr") * 2.0
    _expect(S, -1, lambda: S.SPAI(D, "mr", options=S.Options(drop_tol=-1.0)))
    _expect(S, -1, lambda: S.SPAI(D, "mr", max_iter=-1))
    _expect(S, -1, lambda: S.SPAI(None, "mr", "global", 2.0, True, batch=[D, D]))
    # the implicit residual update only without dropping
    impl = dict(symmetrize=False, drop_tol=0.0, explicit_residual=False)
    _expect(S, -1, lambda: S.SPAI(D, "mr", "global", 8, False, options=S.Options(**impl)))
    _expect(S, -1, lambda: S.SPAI(D, "mr", options=S.Options(**{**impl, "symmetrize": True})))
    _expect(S, -1, lambda: S.SPAI(D, "mr", options=S.Options(**{**impl, "drop_tol": 1e-16})))
    _expect(S, -1, lambda: S.SPAI(None, "mr", batch=[D, D], options=S.Options(**impl)))


def test_c_level_option_checks(S):
    """Option fields the Python wrapper always normalizes, set out of range directly."""
    import ctypes as C
    lib = S.load()
    D = sp.identity(4, format="csr") * 2.0
    a = S._Csr(D)
    for field, bad in (("jacobi", 2), ("a_format", 7), ("precision", 9),
                       ("explicit_residual", 3)):
        o = S.Options().c()
        setattr(o, field, bad)
        h = C.c_void_p()
        rc = lib.spai_create(C.byref(a.c), S.METHODS["mr"], S.cap("none", 0.0, False), 10, 0.0,
                             C.byref(o), C.byref(h))
        assert rc == -1, field


def test_spectrum_rejects_unsymmetric_matrix_on_host(S):
    A = sp.csr_matrix(np.array([[2.0, 1.0], [0.5, 2.0]]))
    _expect(S, -2, lambda: S.spectrum(A, np.ones(2), steps=2))


def test_score_drop_needs_global_cap_and_symmetrize(S):
    D = sp.identity(4, format="csr") * 2.0
    _expect(S, -1, lambda: S.SPAI(D, "mr", "column", 2, False, options=S.Options(drop_score=True)))
    _expect(S, -1, lambda: S.SPAI(D, "mr", "none", 0, False, options=S.Options(drop_score=True)))
    _expect(S, -1, lambda: S.SPAI(D, "mr", "global", 8, False,
                                  options=S.Options(drop_score=True, symmetrize=False)))


def test_floor_frac_must_be_finite_and_nonnegative(S):
    D = sp.identity(4, format="csr") * 2.0
    for bad in (-0.5, float("nan"), float("inf")):
        _expect(S, -1, lambda: S.SPAI(D, "lomr", "global", 8, False,
                                      options=S.Options(floor_frac=bad)))


def test_oracle_and_product_path_are_separate():
    """The oracle imports nothing from the package and the package nothing from the
    oracle; bench.py uses the oracle only in its cpu_baseline leg (and the worker
    processes that leg starts)."""
    import ast
    import glob

    def imports(path):
        tree = ast.parse(open(path).read())
        out = []
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                out += [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom) and node.module:
                out.append(node.module)
        return out

    for f in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        assert not any(m.startswith("paper_2511_09753_amd") for m in imports(f)), f
    for f in glob.glob(os.path.join(ROOT, "paper_2511_09753_amd", "**", "*.py"), recursive=True):
        assert not any(m.split(".")[0] == "oracle" for m in imports(f)), f
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = {fn.name for fn in ast.walk(tree) if isinstance(fn, ast.FunctionDef)
             for node in ast.walk(fn)
             if isinstance(node, ast.ImportFrom) and node.module and node.module.startswith("oracle")}
    # the cpu_baseline leg and the per-core worker it starts (a top-level function, so
    # that a spawned process can find it); nothing else in bench.py calls the worker
    assert users == {"cpu_baseline", "_oracle_worker"}
    callers = {fn.name for fn in ast.walk(tree) if isinstance(fn, ast.FunctionDef)
               for node in ast.walk(fn)
               if isinstance(node, ast.Name) and node.id == "_oracle_worker"}
    assert callers == {"cpu_baseline"}
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    assert not any(isinstance(n, ast.ImportFrom) and n.module and n.module.startswith("oracle")
                   for n in top)


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2511_09753_amd import spai as S
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libspai.so"))
    with pytest.raises(RuntimeError):
        S.load()
    with pytest.raises(RuntimeError):
        S.SPAI(sp.identity(3, format="csr") * 2.0, "mr")


def test_phase_and_counter_tables_match_the_header(S):
    text = open(os.path.join(ROOT, "include", "spai.h")).read()
    nph = int(re.search(r"SPAI_NPHASES\s*=\s*(\d+)", text).group(1))
    ncnt = int(re.search(r"SPAI_NCOUNTS\s*=\s*(\d+)", text).group(1))
    assert len(S.PHASES) == nph and len(S.COUNTS) == ncnt
