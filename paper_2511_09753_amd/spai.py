"""Python binding of libspai: argument marshalling only.

Every step of the method runs in the HIP library; this module turns scipy / torch
matrices into the C structs of ``include/spai.h``, calls the entry point of the
same name and raises :class:`SpaiError` on an error status.  It fails loudly when
the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspai.so")

SPAI_OK, SPAI_CONVERGED, SPAI_MAXITER, SPAI_BREAKDOWN, PCG_INDEFINITE = 0, 1, 2, 3, 4
METHODS = {"mr": 0, "cg": 1, "lomr": 2}
CAP_MODES = {"none": 0, "global": 1, "column": 2}
PRECISIONS = {"f64": 0, "mixed": 1}


class SpaiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class CsrT(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p), ("on_device", C.c_int)]


class CsrOutT(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("capacity", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("val", C.c_void_p),
                ("on_device", C.c_int)]


class CapT(C.Structure):
    _fields_ = [("mode", C.c_int), ("relative", C.c_int), ("value", C.c_double)]


class OptsT(C.Structure):
    _fields_ = [("precision", C.c_int), ("symmetrize", C.c_int), ("drop_tol", C.c_double),
                ("tie_eta", C.c_double), ("stream", C.c_void_p),
                ("device_pool_limit", C.c_int64), ("profile", C.c_int), ("a_format", C.c_int),
                ("jacobi", C.c_int), ("explicit_residual", C.c_int), ("drop_score", C.c_int),
                ("floor_frac", C.c_double)]


EXPORTS = [
    "spai_default_opts", "spai_create", "spai_iterate", "spai_get", "spai_stats",
    "spai_destroy", "pcg_solve", "spai_loss_fwd", "spai_loss_bwd", "spai_create_batched",
    "spai_batched_resid", "spai_last_error", "spai_status_string", "spai_reset", "spai_pcg",
    "spai_profile", "spai_spectrum", "spai_csr_spectrum", "spai_autotune", "spai_get_state",
    "spai_set_state", "spai_set_tiles", "spai_loss_fwd_noalloc", "spai_history",
]
A_FORMATS = {"auto": 0, "csr": 1, "ell": 2}
PHASES = ["dots", "update", "resid", "select", "compact", "bounds", "scalar", "pcg", "pcg_ax",
          "pcg_mx"]
COUNTS = ["cand_m", "cand_p", "cand_pt", "kept_m", "kept_p", "kept_pt", "resid", "iters"]

_lib = None


def load():
    """Load libspai.so (built by ``paper_2511_09753_amd.build``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libspai.so is not built ({LIB_PATH}); run paper_2511_09753_amd/build.py")
    # torch ships its own HIP runtime under the same soname; load it first so that
    # libspai binds to that one and the process holds a single HIP runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.spai_default_opts.argtypes = [C.POINTER(OptsT)]
    lib.spai_default_opts.restype = None
    lib.spai_create.argtypes = [C.POINTER(CsrT), C.c_int, CapT, C.c_int, C.c_double,
                                C.POINTER(OptsT), C.POINTER(P)]
    lib.spai_create_batched.argtypes = [C.POINTER(CsrT), C.c_int, C.c_int, CapT, C.c_int,
                                        C.c_double, C.POINTER(OptsT), C.POINTER(P)]
    lib.spai_iterate.argtypes = [P, C.c_int, C.POINTER(C.c_int), P]
    lib.spai_get.argtypes = [P, C.POINTER(CsrOutT)]
    lib.spai_stats.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_double),
                               C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                               C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.spai_destroy.argtypes = [P]
    lib.spai_batched_resid.argtypes = [P, P]
    lib.pcg_solve.argtypes = [C.POINTER(CsrT), C.POINTER(CsrT), C.c_int, P, P, C.c_double,
                              C.c_int, P, P, C.POINTER(OptsT)]
    lib.spai_loss_fwd.argtypes = [C.POINTER(CsrT), C.POINTER(CsrT), C.POINTER(C.c_double),
                                  C.POINTER(OptsT)]
    lib.spai_loss_bwd.argtypes = [C.POINTER(CsrT), C.POINTER(CsrT), C.c_double, P, P,
                                  C.POINTER(OptsT)]
    lib.spai_loss_fwd_noalloc.argtypes = [C.POINTER(CsrT), C.POINTER(CsrT), P, P,
                                          C.POINTER(OptsT)]
    lib.spai_reset.argtypes = [P]
    lib.spai_pcg.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int, P, P, C.c_int]
    lib.spai_profile.argtypes = [P, P, P, P]
    lib.spai_spectrum.argtypes = [P, C.c_int, P, C.c_int, P, C.POINTER(C.c_int)]
    lib.spai_autotune.argtypes = [P, C.c_int, C.c_int, P, P]
    lib.spai_set_tiles.argtypes = [P, P]
    lib.spai_history.argtypes = [P, P, C.c_int, C.POINTER(C.c_int)]
    lib.spai_get_state.argtypes = [P, P, C.POINTER(C.c_size_t)]
    lib.spai_set_state.argtypes = [P, P, C.c_size_t]
    lib.spai_csr_spectrum.argtypes = [C.POINTER(CsrT), C.c_int, P, P, C.POINTER(C.c_int),
                                      C.POINTER(OptsT)]
    lib.spai_last_error.restype = C.c_char_p
    lib.spai_status_string.restype = C.c_char_p
    lib.spai_status_string.argtypes = [C.c_int]
    for name in EXPORTS:
        if name not in ("spai_default_opts", "spai_last_error", "spai_status_string"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc, allowed=(SPAI_OK,)):
    if rc in allowed:
        return rc
    lib = load()
    raise SpaiError(rc, f"{lib.spai_status_string(rc).decode()}: {lib.spai_last_error().decode()}")


# ----------------------------------------------------------------------------
# argument marshalling
# ----------------------------------------------------------------------------

class _Csr:
    """Keeps the arrays of a CsrT alive for the duration of a call."""

    def __init__(self, A):
        import scipy.sparse as sp
        self.keep = []
        if _is_torch_csr(A):
            rp = A.crow_indices().to(dtype=_torch().int64).contiguous()
            ci = A.col_indices().to(dtype=_torch().int32).contiguous()
            va = A.values().to(dtype=_torch().float64).contiguous()
            self.keep = [rp, ci, va]
            self.c = CsrT(A.shape[0], va.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr(),
                          1 if A.is_cuda else 0)
            self.device = A.is_cuda
        else:
            A = sp.csr_matrix(A)
            rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
            ci = np.ascontiguousarray(A.indices, dtype=np.int32)
            va = np.ascontiguousarray(A.data, dtype=np.float64)
            self.keep = [rp, ci, va]
            self.c = CsrT(A.shape[0], A.nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, 0)
            self.device = False


def _torch():
    import torch
    return torch


def _is_torch_csr(A):
    try:
        import torch
    except ImportError:
        return False
    return isinstance(A, torch.Tensor) and A.layout == torch.sparse_csr


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    return C.c_void_p(getattr(stream, "cuda_stream", stream))


@dataclass
class Options:
    precision: str = "f64"
    symmetrize: bool = True
    drop_tol: float = 2.0 ** -53
    tie_eta: float = 1e-9
    stream: object = None
    device_pool_limit: int = 0
    profile: bool = False
    a_format: str = "auto"      # layout of A on the device: "auto", "csr" or "ell"
    jacobi: bool = False        # Pi = D_A^{-1}-weighted variants (Algorithms 5, 7, 8)
    explicit_residual: bool = True   # False: the update formulas, no dropping (Section 6.2)
    drop_score: bool = False    # global cap of M by the heuristic score of Appendix A
    floor_frac: float = 0.75    # candidates below this fraction of the last cut are not written

    def c(self):
        o = OptsT()
        load().spai_default_opts(C.byref(o))
        o.precision = PRECISIONS[self.precision]
        o.symmetrize = 1 if self.symmetrize else 0
        o.drop_tol = self.drop_tol
        o.tie_eta = self.tie_eta
        o.stream = _stream_ptr(self.stream)
        o.device_pool_limit = int(self.device_pool_limit)
        o.profile = 1 if self.profile else 0
        o.a_format = A_FORMATS[self.a_format]
        o.jacobi = 1 if self.jacobi else 0
        o.explicit_residual = 1 if self.explicit_residual else 0
        o.drop_score = 1 if self.drop_score else 0
        o.floor_frac = float(self.floor_frac)
        return o


def cap(mode="none", value=0.0, relative=False):
    return CapT(CAP_MODES[mode], 1 if relative else 0, float(value))


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------

class SPAI:
    """Handle over ``spai_create`` / ``spai_iterate`` / ``spai_get`` / ``spai_destroy``."""

    def __init__(self, A, method="lomr", cap_mode="none", cap_value=0.0, cap_relative=False,
                 max_iter=100, tol=0.0, options: Options | None = None, batch=None):
        lib = load()
        self.options = options or Options()
        self._opts = self.options.c()
        h = C.c_void_p()
        c = cap(cap_mode, cap_value, cap_relative)
        if batch is None:
            a = _Csr(A)
            self.n = a.c.n
            rc = lib.spai_create(C.byref(a.c), METHODS[method], c, int(max_iter), float(tol),
                                 C.byref(self._opts), C.byref(h))
            self.nseg = 1
        else:
            mats = [_Csr(x) for x in batch]
            arr = (CsrT * len(mats))(*[m.c for m in mats])
            self.n = sum(m.c.n for m in mats)
            rc = lib.spai_create_batched(arr, len(mats), METHODS[method], c, int(max_iter),
                                         float(tol), C.byref(self._opts), C.byref(h))
            self.nseg = len(mats)
        _check(rc)
        self.h = h
        self.method = method

    def iterate(self, k):
        """Run up to k iterations; returns (iterations run, residual history, status)."""
        done = C.c_int(0)
        hist = np.zeros(max(int(k), 1), dtype=np.float64)
        rc = load().spai_iterate(self.h, int(k), C.byref(done), hist.ctypes.data)
        _check(rc, (SPAI_OK, SPAI_CONVERGED, SPAI_BREAKDOWN))
        return done.value, hist[: done.value].copy(), rc

    def get(self):
        """Current iterate M as scipy CSR (float64)."""
        import scipy.sparse as sp
        out = CsrOutT()
        out.n = self.n
        _check(load().spai_get(self.h, C.byref(out)))
        nnz = out.nnz
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        va = np.zeros(max(nnz, 1), dtype=np.float64)
        out.capacity = nnz
        out.rowptr, out.colind, out.val = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
        out.on_device = 0
        _check(load().spai_get(self.h, C.byref(out)))
        return sp.csr_matrix((va[:nnz], ci[:nnz], rp), shape=(self.n, self.n))

    def stats(self):
        it, fb = C.c_int(), C.c_int()
        res, s1, s2 = C.c_double(), C.c_double(), C.c_double()
        nm, npp = C.c_int64(), C.c_int64()
        _check(load().spai_stats(self.h, C.byref(it), C.byref(res), C.byref(nm), C.byref(npp),
                                 C.byref(s1), C.byref(s2), C.byref(fb)))
        return {"iters": it.value, "resid": res.value, "nnz_m": nm.value, "nnz_p": npp.value,
                "step1": s1.value, "step2": s2.value, "mr_fallbacks": fb.value}

    def history(self):
        """Per-iteration drop record: dict of arrays nnz_m, dropped_m, band_m, nnz_p,
        dropped_p, band_p (one entry per iteration run since create/reset)."""
        cnt = C.c_int()
        _check(load().spai_history(self.h, None, 0, C.byref(cnt)))
        rec = np.zeros((max(cnt.value, 1), 6), dtype=np.int64)
        _check(load().spai_history(self.h, rec.ctypes.data, cnt.value, C.byref(cnt)))
        rec = rec[:cnt.value]
        names = ["nnz_m", "dropped_m", "band_m", "nnz_p", "dropped_p", "band_p"]
        return {k: rec[:, c].copy() for c, k in enumerate(names)}

    def reset(self):
        """Restart from M_0 with the same A, method, cap and options."""
        _check(load().spai_reset(self.h))

    def pcg(self, B, rtol=1e-8, max_iter=10000):
        """PCG with this handle's A and current M (both already on the device).

        B: numpy (n x nrhs, host) or a torch CUDA tensor (device).  Returns
        (X, iterations, true relative residuals, status).
        """
        torch_in = not isinstance(B, np.ndarray)
        if torch_in:
            torch = _torch()
            Bt = B.to(dtype=torch.float64).contiguous()
            if Bt.dim() == 1:
                Bt = Bt[:, None]
            X = torch.empty_like(Bt)
            nrhs, bptr, xptr = Bt.shape[1], Bt.data_ptr(), X.data_ptr()
        else:
            Bn = np.ascontiguousarray(B, dtype=np.float64)
            if Bn.ndim == 1:
                Bn = Bn[:, None]
            X = np.zeros_like(Bn)
            nrhs, bptr, xptr = Bn.shape[1], Bn.ctypes.data, X.ctypes.data
        iters = np.zeros(nrhs, dtype=np.int32)
        relres = np.zeros(nrhs, dtype=np.float64)
        rc = load().spai_pcg(self.h, int(nrhs), bptr, xptr, float(rtol), int(max_iter),
                             iters.ctypes.data, relres.ctypes.data, 1 if torch_in else 0)
        _check(rc, (SPAI_OK, SPAI_MAXITER, PCG_INDEFINITE))
        return X, iters, relres, rc

    def profile(self):
        """Per-phase milliseconds / launches (opts.profile) and traffic counters."""
        ms = np.zeros(len(PHASES), dtype=np.float64)
        calls = np.zeros(len(PHASES), dtype=np.int64)
        counts = np.zeros(len(COUNTS), dtype=np.int64)
        _check(load().spai_profile(self.h, ms.ctypes.data, calls.ctypes.data, counts.ctypes.data))
        return ({k: float(v) for k, v in zip(PHASES, ms)},
                {k: int(v) for k, v in zip(PHASES, calls)},
                {k: int(v) for k, v in zip(COUNTS, counts)})

    def spectrum(self, v0, steps=100):
        """Extreme Ritz values of the current M after up to `steps` Lanczos steps from v0
        (numpy on the host or a torch CUDA tensor): (theta_min, theta_max, res_min,
        res_max, steps taken); each theta is within its res of an eigenvalue of M."""
        out = np.zeros(4, dtype=np.float64)
        done = C.c_int(0)
        if isinstance(v0, np.ndarray):
            v = np.ascontiguousarray(v0, dtype=np.float64)
            ptr, dev = v.ctypes.data, 0
        else:
            v = v0.to(dtype=_torch().float64).contiguous()
            ptr, dev = v.data_ptr(), 1
        _check(load().spai_spectrum(self.h, int(steps), ptr, dev, out.ctypes.data,
                                    C.byref(done)))
        return float(out[0]), float(out[1]), float(out[2]), float(out[3]), done.value

    def get_state(self) -> bytes:
        """Checkpoint: the handle's iterate, directions, residual and scalars as bytes."""
        size = C.c_size_t(0)
        _check(load().spai_get_state(self.h, None, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        _check(load().spai_get_state(self.h, buf, C.byref(size)))
        return buf.raw[: size.value]

    def set_state(self, state: bytes):
        """Resume from a checkpoint of a handle with the same problem and configuration."""
        buf = C.create_string_buffer(bytes(state), len(state))
        _check(load().spai_set_state(self.h, buf, len(state)))

    def autotune(self, warm_iters=5, reps=2):
        """Pick the per-column tiles for this workload (see spai_autotune) and restart from
        M_0.  Returns {"resid": (L, H), "dots": (L, H, waves), "update": (L, H, waves)}
        (waves: 5 when that kernel's resident tier runs capped at five waves per SIMD, else
        0) and the best launch times in ms."""
        ch = np.zeros(8, dtype=np.int32)
        ms = np.zeros(3, dtype=np.float64)
        _check(load().spai_autotune(self.h, int(warm_iters), int(reps), ch.ctypes.data,
                                    ms.ctypes.data))
        tiles = {"resid": (int(ch[0]), int(ch[1])), "dots": (int(ch[2]), int(ch[3]), int(ch[7])),
                 "update": (int(ch[4]), int(ch[5]), int(ch[6]))}
        return tiles, {"resid": float(ms[0]), "dots": float(ms[1]), "update": float(ms[2])}

    def set_tiles(self, tiles):
        """Use the given tiles (the dict autotune returns) from the next launch on."""
        r, d, u = tiles["resid"], tiles["dots"], tiles["update"]
        ch = np.array([r[0], r[1], d[0], d[1], u[0], u[1], u[2] if len(u) > 2 else 0,
                       d[2] if len(d) > 2 else 0], dtype=np.int32)
        _check(load().spai_set_tiles(self.h, ch.ctypes.data))

    def batched_resid(self):
        out = np.zeros(self.nseg, dtype=np.float64)
        _check(load().spai_batched_resid(self.h, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "h", None):
            load().spai_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_solve(A, M, B, rtol=1e-8, max_iter=10000, options: Options | None = None):
    """PCG with preconditioner M on every column of B (n x nrhs).

    Host numpy B -> host X; a torch CUDA tensor B (with torch CSR A, M on the device)
    -> a torch CUDA X.  Returns (X, iterations, true relative residuals, status).
    """
    lib = load()
    opts = (options or Options()).c()
    a, m = _Csr(A), _Csr(M)
    torch_in = _is_torch_csr(A)
    if torch_in:
        torch = _torch()
        Bt = B.to(dtype=torch.float64).contiguous()
        if Bt.dim() == 1:
            Bt = Bt[:, None]
        X = torch.empty_like(Bt)
        nrhs = Bt.shape[1]
        bptr, xptr = Bt.data_ptr(), X.data_ptr()
    else:
        Bn = np.ascontiguousarray(B, dtype=np.float64)
        if Bn.ndim == 1:
            Bn = Bn[:, None]
        X = np.zeros_like(Bn)
        nrhs = Bn.shape[1]
        bptr, xptr = Bn.ctypes.data, X.ctypes.data
    iters = np.zeros(nrhs, dtype=np.int32)
    relres = np.zeros(nrhs, dtype=np.float64)
    rc = lib.pcg_solve(C.byref(a.c), C.byref(m.c), int(nrhs), bptr, xptr, float(rtol),
                       int(max_iter), iters.ctypes.data, relres.ctypes.data, C.byref(opts))
    _check(rc, (SPAI_OK, SPAI_MAXITER, PCG_INDEFINITE))
    return X, iters, relres, rc


def spectrum(S, v0, steps=100, options: Options | None = None):
    """Extreme Ritz values of an exactly symmetric CSR matrix S (scipy on the host with a
    numpy v0, or torch CSR on the device with a device v0); returns as SPAI.spectrum."""
    opts = (options or Options()).c()
    s = _Csr(S)
    out = np.zeros(4, dtype=np.float64)
    done = C.c_int(0)
    if s.device:
        v = v0.to(dtype=_torch().float64).contiguous()
        ptr = v.data_ptr()
    else:
        v = np.ascontiguousarray(v0, dtype=np.float64)
        ptr = v.ctypes.data
    _check(load().spai_csr_spectrum(C.byref(s.c), int(steps), ptr, out.ctypes.data,
                                    C.byref(done), C.byref(opts)))
    return float(out[0]), float(out[1]), float(out[2]), float(out[3]), done.value


def loss_fwd(A, M, options: Options | None = None) -> float:
    """f(M) = ||I - A M||_F^2 (A, M: scipy CSR on the host or torch CSR on the device)."""
    out = C.c_double()
    opts = (options or Options()).c()
    a, m = _Csr(A), _Csr(M)
    _check(load().spai_loss_fwd(C.byref(a.c), C.byref(m.c), C.byref(out), C.byref(opts)))
    return out.value


def loss_fwd_noalloc(A, M, L, err, options: Options | None = None) -> None:
    """f(M) into the device tensors L (one float64) and err (one int32) without any
    allocation or host synchronisation (A, M: torch CSR on the device, float64)."""
    opts = (options or Options()).c()
    a, m = _Csr(A), _Csr(M)
    _check(load().spai_loss_fwd_noalloc(C.byref(a.c), C.byref(m.c), L.data_ptr(),
                                        err.data_ptr(), C.byref(opts)))


def loss_bwd(A, M, dL=1.0, want_a=True, want_m=True, options: Options | None = None):
    """Gradients of f in the stored values of A and M (arrays in their CSR order)."""
    opts = (options or Options()).c()
    a, m = _Csr(A), _Csr(M)
    if a.device:
        torch = _torch()
        dev = A.values().device
        gA = torch.empty(a.c.nnz, dtype=torch.float64, device=dev) if want_a else None
        gM = torch.empty(m.c.nnz, dtype=torch.float64, device=dev) if want_m else None
        pa = gA.data_ptr() if want_a else None
        pm = gM.data_ptr() if want_m else None
    else:
        gA = np.zeros(a.c.nnz) if want_a else None
        gM = np.zeros(m.c.nnz) if want_m else None
        pa = gA.ctypes.data if want_a else None
        pm = gM.ctypes.data if want_m else None
    _check(load().spai_loss_bwd(C.byref(a.c), C.byref(m.c), float(dL), pa, pm, C.byref(opts)))
    return gA, gM


def fro_loss_function():
    """torch.autograd.Function for f = ||I - A M||_F^2 over the values of A and M.

    ``FroLoss.apply(a_vals, m_vals, A_pattern, M_pattern, options)`` where the patterns
    are torch CSR tensors on the device (their values are ignored) and a_vals, m_vals
    are 1-D tensors of the stored values in CSR order.
    """
    torch = _torch()

    def _with(pattern, vals):
        return torch.sparse_csr_tensor(pattern.crow_indices(), pattern.col_indices(),
                                       vals.detach().to(torch.float64), size=pattern.shape)

    class FroLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, a_vals, m_vals, A_pattern, M_pattern, options=None):
            A = _with(A_pattern, a_vals)
            M = _with(M_pattern, m_vals)
            ctx.save_for_backward(a_vals, m_vals)
            ctx.pats = (A_pattern, M_pattern, options)
            return torch.tensor(loss_fwd(A, M, options), dtype=torch.float64,
                                device=a_vals.device)

        @staticmethod
        def backward(ctx, grad):
            a_vals, m_vals = ctx.saved_tensors
            A_pattern, M_pattern, options = ctx.pats
            A = _with(A_pattern, a_vals)
            M = _with(M_pattern, m_vals)
            gA, gM = loss_bwd(A, M, float(grad), ctx.needs_input_grad[0],
                              ctx.needs_input_grad[1], options)
            out_a = gA.to(a_vals.dtype) if gA is not None else None
            out_m = gM.to(m_vals.dtype) if gM is not None else None
            return out_a, out_m, None, None, None

    return FroLoss
