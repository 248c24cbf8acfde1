#!/usr/bin/env python3
"""Benchmark of the SPAI hot path on one MI355X.

A step is one pass of the whole path on the 96^3 lognormal-diffusion workload
(n = 884,736): restart from M_0 = (tr A / tr A^2) I, 30 LOMR iterations (float32
iterate values, float64 sums, global cap 2 nnz(A)), then PCG with the resulting M on
64 right-hand sides to 1e-8.  A, the handle's pools and B are resident in device
memory before the timed region.  Prints one JSON line (rank 0).

Extra legs (not timed as steps): the float64 path on the same workload and the
mixed-vs-float64 time to equal ||I - A M||_F, the Pi-weighted LOMR, the Appendix A
heuristic drop score under the same cap, Lanczos extremes of the final M, the batched
form on 256 random geometric-graph matrices, the loss and its gradients on the
512 x 512 9-point grid, and the CPU oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(c, n, nnzA, s_val, s_aval, iters):
    """Bytes each phase must move per iteration if every operand is read once and
    every output written once (LOMR), from the traffic counters.

    Padded column storage: entry = 4-byte row index + value; column = 8-byte start +
    4-byte length.  A: CSR with 8-byte row pointers, 4-byte column indices.
    """
    e = 4 + s_val
    col = 12 * n
    EA = nnzA * (4 + s_aval) + 8 * (n + 1)
    nR = c["resid"] / max(iters, 1)
    nM = c["kept_m"] / max(iters, 1)
    nP = c["kept_p"] / max(iters, 1)
    nPT = c["kept_pt"] / max(iters, 1)
    cM = c["cand_m"] / max(iters, 1)
    cP = c["cand_p"] / max(iters, 1)
    cPT = c["cand_pt"] / max(iters, 1)
    return {
        "dots": (nR + nP) * e + 2 * col + EA + 48 * n,
        "update": (nM + nR + nP + nPT) * e + 4 * col + EA + (cM + cP + cPT) * e + 3 * col,
        "resid": nM * e + col + EA + nR * e + col + 8 * n,
        "compact": (cM + cP + cPT) * e * 1 + (nM + nP + nPT) * e + 6 * col,
    }


def lomr_alg_bytes(c, n, nnzA, s_val, s_aval, iters, with_p=True):
    """Whole-iteration algorithmic bytes of LOMR (each operand of the iteration read once,
    each output written once): 2E(A) + 3E(R) + 3E(P) + 3E(M), E(X) = nnz(X)(s + 4) + 8(n + 1);
    MR (with_p False) has no P term."""
    def E(nnz, s):
        return nnz * (s + 4) + 8 * (n + 1)
    it = max(iters, 1)
    return (2 * E(nnzA, s_aval) + 3 * E(c["resid"] / it, s_val)
            + (3 * E(c["kept_p"] / it, s_val) if with_p else 0) + 3 * E(c["kept_m"] / it, s_val))


# kernel of each timed phase (its resident tier; the lean tiers when A is held in ELL),
# and the source file its code lives in
PHASE_KERNEL = {"dots": "k_dots", "update": "k_update", "resid": "k_resid", "compact": "k_compact",
                "pcg_mx": "k_spmm_pair_mx", "pcg_ax": "k_spmm_pair_ax"}
KERNEL_SOURCE = {"k_dots": "spai_kernels.hip", "k_update": "spai_kernels.hip",
                 "k_resid": "spai_kernels.hip", "k_compact": "spai_kernels.hip",
                 "k_dots_lean": "spai_kernels.hip", "k_update_lean": "spai_kernels.hip",
                 "k_resid_lean": "spai_kernels.hip",
                 "k_spmm_pair_mx": "spai_pcg.hip", "k_spmm_pair_ax": "spai_pcg.hip"}


def phase_kernels(tiles, ell):
    """PHASE_KERNEL with the resident-tier variants a handle runs: the lean residual when A
    is held in ELL (ell: its padded row width, 0 for CSR), the lean dots and update when
    their tile variant is 1."""
    out = dict(PHASE_KERNEL)
    if ell:
        out["resid"] = "k_resid_lean"
    if tiles is None:                 # the defaults: lean tiers with A in ELL
        tiles = {"dots": (0, 0, 1 if ell else 0), "update": (0, 0, 1 if ell else 0)}
    if tiles["dots"][2] == 1:
        out["dots"] = "k_dots_lean"
    if tiles["update"][2] == 1:
        out["update"] = "k_update_lean"
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, or None when that summary is missing or was taken on other kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_lognormal96.md")
    if kernel not in KERNEL_SOURCE or not os.path.exists(path):
        return None
    src = os.path.join(ROOT, "paper_2511_09753_amd", "csrc", KERNEL_SOURCE[kernel])
    want = hashlib.sha256(open(src, "rb").read()).hexdigest()
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != want:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calib_copy(nbytes):
    """A plain device-to-device copy of nbytes (the reference the HBM counters are
    scaled by): reads nbytes, writes nbytes."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": nbytes, "launches": 3}), flush=True)


def exp05():
    """The protocol of Experiments 05 and 06 (Section 7.2, Tables 5-6) on the paper's own
    matrices rebuilt from their recipes: the Pi-weighted MR, matrix CG and LOMR
    (Pi = D_A^{-1}) with a 3% density cap, snapshots after 5, 20 and 100 iterations unless
    ||I - AM||_F / sqrt(n) <= 1e-6 comes first; per snapshot lambda_min(M), lambda_max(M)
    as the extreme Ritz values of up to 300 Lanczos steps on the GPU (each with its
    residual bound; a negative theta_min proves M indefinite), ||I - AM||_F, iterations,
    nnz(M)/n^2, and vector PCG iterations with M (one RHS, to 1e-8) beside Jacobi's.  The realisations differ from the authors', so the comparison
    with the tables is qualitative."""
    import numpy as np
    import scipy.sparse as sp
    from paper_2511_09753_amd import spai as S
    from paper_2511_09753_amd import workloads as W
    S.load()
    rows = []
    names = {"mr": "PMR_SPD", "cg": "PCG (matrix)", "lomr": "LOPMR_SPD"}
    for k, name in enumerate(W.PAPER_RECIPES):
        A = W.paper_recipe(name, W.seed_for(6, k))
        n = A.shape[0]
        b = W.rhs(n, 1, W.seed_for(6, 10 + k))
        m = int(round(0.03 * n * n))
        _, itj, _, rcj = S.pcg_solve(A, sp.diags(1.0 / A.diagonal()).tocsr(), b, rtol=1e-8,
                                     max_iter=20000)
        log(f"{name}: n={n} nnz={A.nnz}; vector PCG with Jacobi: {int(itj[0])} iterations (status {rcj})")
        for method in ("mr", "cg", "lomr"):
            try:
                h = S.SPAI(A, method, "global", m, False, max_iter=100, tol=1e-6,
                           options=S.Options(jacobi=True))
            except S.SpaiError as e:
                rows.append({"matrix": name, "method": names[method], "error": str(e)})
                continue
            done, t_spai = 0, 0.0
            for target in (5, 20, 100):
                try:
                    t0 = time.perf_counter()
                    d, hist, rc = h.iterate(target - done)
                    t_spai += time.perf_counter() - t0
                except S.SpaiError as e:
                    rows.append({"matrix": name, "method": names[method], "error": str(e)})
                    break
                done += d
                st = h.stats()
                v0 = np.random.default_rng(W.seed_for(6, 20 + k)).standard_normal(n)
                lmin, lmax, rmin, rmax, ksteps = h.spectrum(v0, steps=min(300, n))
                _, itp, relp, rcp = h.pcg(b, rtol=1e-8, max_iter=20000)
                row = {"matrix": name, "method": names[method], "iters": done,
                       "lambda_min": lmin, "lambda_max": lmax, "lambda_min_res": rmin,
                       "lambda_max_res": rmax, "lanczos_steps": ksteps, "resid_fro": st["resid"],
                       "density": st["nnz_m"] / float(n) ** 2,
                       "pcg_iters": int(itp[0]), "pcg_status": int(rcp),
                       "jacobi_pcg_iters": int(itj[0]), "spai_seconds": t_spai}
                rows.append(row)
                log(f"  {names[method]:13s} its {done:3d}  lmin {lmin: .2e} lmax {lmax: .2e}  "
                    f"||I-AM|| {st['resid']:.2e}  nnz/n^2 {row['density']:.2e}  "
                    f"vector PCG {int(itp[0])} (status {int(rcp)})  {t_spai:.2f} s")
                if rc == S.SPAI_CONVERGED or d < target - (done - d):
                    break
            h.close()
    print(json.dumps({"experiment": "Experiments 05/06 protocol, paper recipe matrices",
                      "rows": rows}), flush=True)


def _oracle_worker(path, iters, q):
    """Child process of the all-cores CPU baseline: load the state and time `iters` LOMR
    iterations of the oracle from it (the oracle as it stands, one process per core)."""
    import numpy as np
    import scipy.sparse as sp
    from oracle import spai_oracle as O
    z = np.load(path)
    n = int(z["n"])
    A = sp.csr_matrix((z["a_val"], z["a_idx"], z["a_ptr"]), shape=(n, n))
    M = sp.csc_matrix((z["m_val"], z["m_idx"], z["m_ptr"]), shape=(n, n))
    P = sp.csc_matrix((z["p_val"], z["p_idx"], z["p_ptr"]), shape=(n, n))
    rule = O.DropRule(mode="global", m=int(z["m"]))
    t = time.perf_counter()
    O.lomr(A, rule, iters, M0=M, P0=P)
    q.put(time.perf_counter() - t)


def cpu_baseline(A, M, P, start_iter, procs=16):
    """The oracle (as it stands) on a bounded sample of the workload: LOMR iterations from
    a representative iterate (M_i, P_{i-1} of the device run after start_iter
    iterations, when the columns have their steady size), on one core and then one
    process per core at once (the oracle is single-threaded scipy)."""
    import multiprocessing as mp
    import numpy as np
    from oracle import spai_oracle as O
    m = O.cap_counts(A, "global", 2.0, True)
    rule = O.DropRule(mode="global", m=m)
    its1 = 1
    t = time.perf_counter()
    O.lomr(A, rule, its1, M0=M, P0=P)
    dt1 = time.perf_counter() - t
    procs = max(1, min(procs, os.cpu_count() or 1))
    path = os.path.join("/dev/shm" if os.path.isdir("/dev/shm") else "/tmp",
                        f"spai_cpu_baseline_{os.getpid()}.npz")
    Ac = A.tocsr()
    np.savez(path, n=A.shape[0], m=m, a_val=Ac.data, a_idx=Ac.indices, a_ptr=Ac.indptr,
             m_val=M.data, m_idx=M.indices, m_ptr=M.indptr,
             p_val=P.data, p_idx=P.indices, p_ptr=P.indptr)
    try:
        ctx = mp.get_context("spawn")
        q = ctx.Queue()
        ps = [ctx.Process(target=_oracle_worker, args=(path, 1, q)) for _ in range(procs)]
        t = time.perf_counter()
        for p in ps:
            p.start()
        times = [q.get() for _ in ps]
        wall = time.perf_counter() - t
        for p in ps:
            p.join()
    finally:
        os.remove(path)
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         model)
    except OSError:
        pass
    # aggregate throughput of the all-core run: iterations done / the slowest process's
    # time (start-up and loading excluded, as the single-core figure excludes them)
    return {"value": procs / max(times), "unit": "SPAI iters/s", "cores": procs, "kind": "oracle",
            "single_core_value": its1 / dt1,
            "sample": f"FP64 LOMR iterations of the oracle from the iterate after {start_iter} "
                      f"device iterations on the 96^3 lognormal matrix (global cap 2 nnz(A)): "
                      f"{procs} processes x 1 iteration at once ({max(times):.1f} s the slowest, "
                      f"{wall:.1f} s wall with start-up), and {its1} iterations on one core "
                      f"({dt1:.1f} s); scipy, single-threaded per process, {os.cpu_count()} "
                      f"logical cores ({model})"}


def state_min_bytes(c, n, nnzA, s_val, s_aval, iters):
    """State-only lower bound of a LOMR iteration: A once, M and P read and written once,
    R recomputed per column and never stored: E(A) + 2E(M) + 2E(P)."""
    def E(nnz, s):
        return nnz * (s + 4) + 8 * (n + 1)
    it = max(iters, 1)
    return E(nnzA, s_aval) + 2 * E(c["kept_m"] / it, s_val) + 2 * E(c["kept_p"] / it, s_val)


def state_lists(buf):
    """The column lists of a spai_get_state buffer (header, per-matrix scalars, then the
    lists as compact CSC: M, P, P^T for CG and LOMR, R), as float64 scipy CSC matrices."""
    import struct
    import numpy as np
    import scipy.sparse as sp
    hdr = "<8sii q iiiiii qq 5q"
    f = struct.unpack_from(hdr, buf, 0)
    vb, n, nseg, nl, nnz = f[2], f[3], f[4], f[9], f[12:17]
    vt = np.float32 if vb == 4 else np.float64
    o = struct.calcsize(hdr) + 152 * nseg          # SegState is 152 bytes
    out = []
    for l in range(nl):
        cp = np.frombuffer(buf, dtype=np.int64, count=n + 1, offset=o)
        o += 8 * (n + 1)
        ix = np.frombuffer(buf, dtype=np.int32, count=nnz[l], offset=o)
        o += 4 * nnz[l]
        vl = np.frombuffer(buf, dtype=vt, count=nnz[l], offset=o).astype(np.float64)
        o += vb * nnz[l]
        out.append(sp.csc_matrix((vl, ix.copy(), cp.copy()), shape=(n, n)))
    return out


def small_configs_leg(S, W, torch, np):
    """The two float64 configurations beside the benchmark: the 32 x 32 Laplacian (MR,
    global cap nnz(A), 20 iterations, PCG on one right-hand side) and the 256 x 256
    anisotropic stencil (MR, LOMR and CG, column cap 3 nnz(A e_j), 50 iterations each,
    PCG on four right-hand sides), with per-iteration times, final ||I - A M||_F and the
    PCG iteration counts (the method comparison of Tables 5-6)."""
    out = {}
    for name, methods, cfg in (("laplace32", ["mr"], 1), ("aniso256", ["mr", "lomr", "cg"], 2)):
        wl = W.workload(name)
        A = wl.A
        B = W.rhs(A.shape[0], wl.nrhs, W.seed_for(cfg, 1))
        for method in methods:
            h = S.SPAI(A, method, wl.cap_mode, wl.cap_value, wl.cap_relative, max_iter=wl.iters)
            h.iterate(wl.iters)                    # warm-up
            h.reset()
            torch.cuda.synchronize()
            t = time.perf_counter()
            done, hist, _ = h.iterate(wl.iters)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3 / max(done, 1)
            X, it, rel, rc = h.pcg(B, rtol=wl.rtol)
            st = h.stats()
            h.close()
            out[f"{name}_{method}"] = {
                "iters": int(done), "ms_per_iter": ms, "resid_fro": float(hist[-1]),
                "nnz_m": st["nnz_m"], "pcg_iters": [int(x) for x in it],
                "pcg_max_true_relres": float(rel.max()), "pcg_status": int(rc)}
    return out


def batched_leg(S, W, torch, np, iters=20, nrhs=8):
    """The batched form on random-graph SPD matrices: 256 geometric-graph Laplacians with
    diagonal shifts (n ~ U{500..20000}) as one handle, MR, column cap 4, float32 values
    with float64 sums, tiles autotuned, 20 iterations from M_0 replayed from the handle's
    HIP graph and timed as a whole (a batched handle has no per-phase events); then PCG
    with the block-diagonal A and M on nrhs right-hand sides."""
    wl = W.workload("geo256")
    mats = wl.A
    n = sum(A.shape[0] for A in mats)
    nnz = sum(A.nnz for A in mats)
    log(f"batched: {len(mats)} geometric-graph matrices, n={n}, nnz={nnz}")
    h = S.SPAI(None, "mr", "column", 4.0, False, max_iter=iters,
               options=S.Options(precision="mixed"), batch=mats)
    tiles, _ = h.autotune(warm_iters=3, reps=2)
    h.reset()
    h.iterate(iters)                                  # warm-up (graph capture)
    _, _, k0 = h.profile()
    h.reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    done, _, _ = h.iterate(iters)
    torch.cuda.synchronize()
    T = time.perf_counter() - t
    _, _, k1 = h.profile()
    res = h.batched_resid()
    its = max(k1["iters"] - k0["iters"], 1)
    cnt = {k: k1[k] - k0[k] for k in k1}
    it_bytes = lomr_alg_bytes(cnt, n, nnz, 4, 4, its, with_p=False)
    ms_it = T / max(done, 1) * 1e3
    got = it_bytes / (ms_it * 1e-3) / 1e9
    B = torch.from_numpy(W.rhs(n, nrhs, W.seed_for(4, 1))).cuda()
    h.pcg(B, rtol=1e-8, max_iter=10000)               # warm-up (graph capture)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, pit, rel, rc = h.pcg(B, rtol=1e-8, max_iter=10000)
    torch.cuda.synchronize()
    Tp = time.perf_counter() - t
    h.close()
    out = {
        "workload": f"{len(mats)} random geometric-graph Laplacians + shift, n={n}, nnz={nnz}; "
                    f"MR, column cap 4, float32 values, float64 sums, {iters} iterations",
        "iters": done, "iters_per_s": done / T, "ms_per_iter": ms_it,
        "tiles": tiles,
        "iteration_alg_bytes": it_bytes,
        "roofline": {"bound": "hbm", "kernel": "whole iteration (graph replay)", "achieved": got,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": got / HBM_PEAK_GBS},
        "resid_fro_max": float(res.max()), "resid_fro_median": float(np.median(res)),
        "pcg": {"nrhs": nrhs, "iters_max": int(pit.max()), "iters_min": int(pit.min()),
                "max_true_rel_res": float(rel.max()), "status": int(rc), "seconds": Tp},
    }
    log("batched:", json.dumps(out))
    return out


def loss_leg(S, W, torch, np, reps=5):
    """The differentiation form: f = ||I - A M||_F^2 and its gradients in the values of A
    and M through the autograd function, on the 512 x 512 9-point grid graph with M on
    the pattern of A^2 (n = 262,144), inputs resident on the device; FP64 and the FP32
    form (float64 sums).  Median of reps calls; algorithmic bytes: A and M read once
    (index 4 + value 8 bytes, 8-byte row pointers), the two gradients written once."""
    import scipy.sparse as sp
    wl = W.workload("grid9_512")
    A = sp.csr_matrix(wl.A)
    M = sp.csr_matrix(W.loss_m_values(A, wl.extra["pattern"], W.seed_for(5, 1)))
    n = A.shape[0]
    dev = torch.device("cuda")

    def pattern(X):
        return torch.sparse_csr_tensor(torch.from_numpy(X.indptr.astype(np.int64)),
                                       torch.from_numpy(X.indices.astype(np.int64)),
                                       torch.from_numpy(X.data), size=X.shape).to(dev)
    Ap, Mp = pattern(A), pattern(M)
    FroLoss = S.fro_loss_function()
    read = A.nnz * 12 + M.nnz * 12 + 16 * (n + 1)
    out = {"workload": f"9-point grid graph 512x512 (n={n}, nnz(A)={A.nnz}), M on pattern(A^2) "
                       f"(nnz={M.nnz})", "alg_bytes_fwd": read,
           "alg_bytes_fwd_bwd": 2 * read + 8 * (A.nnz + M.nnz)}
    for prec in ("f64", "mixed"):
        opts = S.Options(precision=prec)
        fwd, both = [], []
        for r in range(reps + 1):
            a = torch.tensor(A.data, device=dev, requires_grad=True)
            m = torch.tensor(M.data, device=dev, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L = FroLoss.apply(a, m, Ap, Mp, opts)
            float(L.detach())
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if r:                                   # the first call warms up
                fwd.append(t1 - t0)
                both.append(t2 - t0)
        f, b = float(np.median(fwd)), float(np.median(both))
        out[prec] = {"loss": float(L.detach()), "fwd_ms": f * 1e3, "fwd_bwd_ms": b * 1e3,
                     "fwd_gbs": read / f / 1e9, "fwd_bwd_gbs": out["alg_bytes_fwd_bwd"] / b / 1e9}
    log("loss:", json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--grid", type=int, default=96)
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pcg", action="store_true", help="(diagnostics only) skip the PCG leg")
    ap.add_argument("--no-jacobi", action="store_true", help="skip the Pi-weighted LOMR leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles")
    ap.add_argument("--tiles", default="", metavar="JSON",
                    help='use these tiles instead of tuning, as the tuner reports them, e.g. '
                         '\'{"resid": [128, 1024], "dots": [256, 1024, 1], "update": [128, 256, 1]}\'')
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the heuristic-score and spectrum legs")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched random-graph leg")
    ap.add_argument("--exp05", action="store_true",
                    help="run the Experiment 05/06 protocol on the paper's recipe matrices and exit")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.calib_copy:
        calib_copy(args.calib_copy)
        return
    if args.exp05:
        exp05()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU column sharding is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import scipy.sparse as sp
    import torch
    from paper_2511_09753_amd import spai as S
    from paper_2511_09753_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    S.load()
    N = args.grid
    A = W.lognormal3d(N, W.seed_for(3))
    n, nnzA = A.shape[0], A.nnz
    deg = int(np.diff(sp.csr_matrix(A).indptr).max())
    ell = 0 if deg > 64 else 1 << max(0, (deg - 1).bit_length())   # the ELL row width
    log(f"workload: 3D lognormal 7-point {N}^3, n={n}, nnz={nnzA}")
    B = torch.from_numpy(W.rhs(n, args.nrhs, W.seed_for(3, 1))).cuda()

    def make(prec, profile, jacobi=False, score=False):
        return S.SPAI(A, "lomr", "global", 2.0, True, max_iter=max(args.iters, 60),
                      options=S.Options(precision=prec, profile=profile, jacobi=jacobi,
                                        drop_score=score))

    def step(h, its):
        h.reset()
        done, hist, _ = h.iterate(its)
        pcg = None
        if not args.no_pcg:
            X, pit, rel, rc = h.pcg(B, rtol=1e-8, max_iter=10000)
            pcg = (pit, rel, rc)
        return done, hist, pcg

    # ---------------- mixed path: the timed steps
    t0 = time.perf_counter()
    h = make("mixed", True)
    log(f"create (validate + upload + pools): {time.perf_counter() - t0:.2f} s")
    tuned = None
    if args.tiles:                            # tiles given (e.g. a stored tuner result)
        tiles = {k: tuple(v) for k, v in json.loads(args.tiles).items()}
        h.set_tiles(tiles)
        tuned = {"tiles": tiles, "given": True}
    elif not args.no_autotune:                # per-column tiles for this workload (setup)
        # tuned on the state halfway through the run: the columns have their steady
        # size there (after 5 iterations they are still small, and a tile that is best
        # there can be slower over the run)
        t0 = time.perf_counter()
        tiles, tms = h.autotune(warm_iters=max(5, args.iters // 2), reps=2)
        tuned = {"tiles": tiles, "launch_ms": tms, "seconds": time.perf_counter() - t0}
    if tuned:
        log("tiles:", json.dumps(tuned))
    for _ in range(args.warmup):
        step(h, args.iters)
    ms0, calls0, cnt0 = h.profile()
    torch.cuda.synchronize()
    t = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = step(h, args.iters)
    torch.cuda.synchronize()
    T = time.perf_counter() - t
    ms1, calls1, cnt1 = h.profile()
    done, hist, pcg = last
    cpu_state = None
    if not args.no_cpu:                     # a representative iterate for the CPU oracle
        h.reset()
        h.iterate(10)
        lists = state_lists(h.get_state())
        cpu_state = (lists[0], lists[1], 10)
        h.reset()
        h.iterate(args.iters)               # leave the handle at the timed steps' end state
    iters_timed = cnt1["iters"] - cnt0["iters"]
    ph_ms = {k: ms1[k] - ms0[k] for k in ms1}
    ph_calls = {k: calls1[k] - calls0[k] for k in calls1}
    cnt = {k: cnt1[k] - cnt0[k] for k in cnt1}
    spai_ms = sum(v for k, v in ph_ms.items() if not k.startswith("pcg"))
    log(f"phases (ms over {args.steps} steps): " + ", ".join(f"{k}={v:.1f}" for k, v in ph_ms.items()))
    alg = algorithmic_bytes(cnt, n, nnzA, 4, 4, iters_timed)
    per_iter_ms = {k: ph_ms[k] / max(iters_timed, 1) for k in alg}
    stats = h.stats()

    pk = phase_kernels(tuned["tiles"] if tuned else None, ell)

    def roofline(phase, bytes_per_launch):
        launch_ms = ph_ms[phase] / max(ph_calls[phase], 1)
        got = bytes_per_launch / (launch_ms * 1e-3) / 1e9
        kern = pk[phase]
        return {"bound": "hbm", "kernel": kern, "achieved": got, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": got / HBM_PEAK_GBS, "traffic": measured_traffic(kern),
                "alg_bytes_per_launch": bytes_per_launch, "avg_launch_ms": launch_ms,
                "ms_per_step": ph_ms[phase] / args.steps}

    # The SPAI iteration's kernels against their shares of the iteration's algorithmic
    # bytes 2E(A) + 3E(R) + 3E(P) + 3E(M) (each operand read once, each output written
    # once): the dots read A, R, P; the update reads M, R, P and writes M, P (the new
    # iterate and direction before the drop); the residual reads A, M and writes R.
    # Selection and compaction (the drop's second pass over the update's candidates)
    # carry no share of their own: they are this design's cost of the drop.  A phase's
    # time per iteration is its launch on the resident tier plus the launches for
    # deferred columns (none on this workload once the lean tiers hold every column).
    def E(nnz, sv):
        return nnz * (sv + 4) + 8 * (n + 1)
    itc = max(iters_timed, 1)
    eA, eR = E(nnzA, 4), E(cnt["resid"] / itc, 4)
    eM, eP = E(cnt["kept_m"] / itc, 4), E(cnt["kept_p"] / itc, 4)
    share = {"dots": eA + eR + eP, "update": eR + 2 * eP + 2 * eM, "resid": eA + eM + eR}
    spai_kernels = {}
    for k, b in share.items():
        t_ms = per_iter_ms[k]
        got = b / (t_ms * 1e-3) / 1e9
        spai_kernels[k] = {"bound": "hbm", "kernel": pk[k], "achieved": got,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": got / HBM_PEAK_GBS,
                           "traffic": measured_traffic(pk[k]),
                           "alg_bytes_per_launch": b, "avg_launch_ms": t_ms,
                           "launches_per_iter": ph_calls[k] / itc,
                           "ms_per_step": ph_ms[k] / args.steps}
    spai_kernels["select_compact"] = {
        "kernel": "k_sel_* + k_compact (the drop's selection and compaction)",
        "ms_per_iter": (ph_ms.get("select", 0.0) + ph_ms.get("compact", 0.0)) / itc}
    # the headline: the SPAI step's dominant kernel (most time per iteration)
    dom = max(share, key=lambda k: spai_kernels[k]["avg_launch_ms"])
    roof_spai = dict(spai_kernels[dom])
    # the PCG products (event-timed inside the solve): read the matrix and X once, write Y
    # once, X and Y n x nrhs float64; M in padded columns (4-byte index + 4-byte value,
    # 12-byte descriptor), A as CSR with float64 values
    roofs = {"spai": roof_spai}
    if ph_calls.get("pcg_mx"):
        vec = 2 * n * args.nrhs * 8
        roofs["pcg_mx"] = roofline("pcg_mx", stats["nnz_m"] * 8 + 12 * n + vec)
        roofs["pcg_ax"] = roofline("pcg_ax", nnzA * 12 + 8 * (n + 1) + vec)
    it_bytes = lomr_alg_bytes(cnt, n, nnzA, 4, 4, iters_timed)
    it_gbs = it_bytes / (spai_ms / max(iters_timed, 1) * 1e-3) / 1e9
    roof_iter = {"bound": "hbm", "kernel": "LOMR iteration (dots, update, select, compact, "
                 "residual, scalars)", "achieved": it_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": it_gbs / HBM_PEAK_GBS, "alg_bytes_per_iter": it_bytes,
                 "ms_per_iter": spai_ms / max(iters_timed, 1),
                 "traffic": None}
    min_bytes = state_min_bytes(cnt, n, nnzA, 4, 4, iters_timed)
    min_gbs = min_bytes / (spai_ms / max(iters_timed, 1) * 1e-3) / 1e9
    r_mixed = float(hist[-1])
    log(f"mixed: ||I-AM||_F after {done} its = {r_mixed:.6e}, nnz(M)={stats['nnz_m']}, "
        f"nnz(P)={stats['nnz_p']}; SPAI {spai_ms / max(iters_timed, 1):.3f} ms/it")
    if pcg:
        log(f"PCG 64 RHS: iterations min/max {pcg[0].min()}/{pcg[0].max()}, "
            f"max true rel res {pcg[1].max():.2e}, status {pcg[2]}")

    # ---------------- spectrum of the final M: Lanczos on the device (Tables 4-6 columns)
    spec = None
    if not args.no_extras:
        v0 = torch.from_numpy(np.random.default_rng(W.seed_for(3, 2)).standard_normal(n)).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        lo, hi, rlo, rhi, ks = h.spectrum(v0, steps=100)
        torch.cuda.synchronize()
        spec = {"lanczos_steps": ks, "theta_min": lo, "theta_max": hi, "res_min": rlo,
                "res_max": rhi, "seconds": time.perf_counter() - t}
        log("spectrum of M:", json.dumps(spec))

    # ---------------- float64 path and time to equal residual
    f64 = None
    if not args.no_f64:
        M_mixed = h.get()                           # the mixed path's final iterate
        h.close()
        h64 = make("f64", True)
        tiles64 = None
        if tuned and not tuned.get("given"):        # each precision with its own tiles
            tiles64, _ = h64.autotune(warm_iters=max(5, args.iters // 2), reps=2)
        step(h64, args.iters)                       # warm-up
        m0, c0, k0 = h64.profile()
        torch.cuda.synchronize()
        t = time.perf_counter()
        d64, hist64, pcg64 = step(h64, args.iters)
        torch.cuda.synchronize()
        T64 = time.perf_counter() - t
        m1, c1, k1 = h64.profile()
        spai64 = sum(m1[k] - m0[k] for k in m1 if not k.startswith("pcg"))
        r64 = float(hist64[-1])
        M_f64 = h64.get()
        h64.close()
        # both final iterates' ||I - A M||_F evaluated in float64 (the loss entry point)
        ev_mixed = math.sqrt(S.loss_fwd(A, M_mixed))
        ev_f64 = math.sqrt(S.loss_fwd(A, M_f64))
        del M_mixed, M_f64
        # mixed until ||I - A M||_F <= r64 (1 + 1e-5), at most 60 iterations
        hm = make("mixed", True)
        a0, _, q0 = hm.profile()
        hm.reset()
        dn, histm, _ = hm.iterate(60)
        a1, _, q1 = hm.profile()
        reach = next((i + 1 for i, r in enumerate(histm) if r <= r64 * (1 + 1e-5)), None)
        mixed_ms_per_it = sum(a1[k] - a0[k] for k in a1 if not k.startswith("pcg")) / max(q1["iters"] - q0["iters"], 1)
        f64_ms_per_it = spai64 / max(k1["iters"] - k0["iters"], 1)
        hm.close()
        f64 = {
            "f64_resid_fro_30": r64, "mixed_resid_fro_30": r_mixed,
            "f64_evaluated_resid_fro_30": {"f64_path": ev_f64, "mixed_path": ev_mixed},
            "rel_diff_30": abs(r_mixed - r64) / r64,
            "f64_spai_ms_per_iter": f64_ms_per_it, "mixed_spai_ms_per_iter": mixed_ms_per_it,
            "per_iter_speedup": f64_ms_per_it / mixed_ms_per_it,
            "mixed_iters_to_f64_resid": reach,
            "time_to_equal_resid_speedup": (f64_ms_per_it * args.iters) / (mixed_ms_per_it * reach)
            if reach else None,
            "f64_step_s": T64, "f64_pcg_iters_max": int(pcg64[0].max()) if pcg64 else None,
            "f64_tiles": tiles64,
        }
        log("f64 comparison:", json.dumps(f64))
    else:
        h.close()

    # ---------------- Pi-weighted LOMR (Algorithm 8, Pi = D_A^{-1}), same workload and cap
    jac = None
    if not args.no_jacobi:
        hj = make("mixed", True, jacobi=True)
        hj.reset()
        hj.iterate(args.iters)                       # warm-up
        j0, _, k0 = hj.profile()
        hj.reset()
        _, histj, _ = hj.iterate(args.iters)
        j1, _, k1 = hj.profile()
        jms = sum(j1[k] - j0[k] for k in j1 if not k.startswith("pcg")) / max(k1["iters"] - k0["iters"], 1)
        hj.close()
        jac = {"method": "LOMR_SPD (Pi = D_A^-1), mixed", "spai_ms_per_iter": jms,
               "resid_fro": float(histj[-1]), "iters": args.iters}
        log("jacobi-weighted LOMR:", json.dumps(jac))

    # ---------------- Appendix A heuristic drop score under the same cap (LOMR, mixed)
    score = None
    if not args.no_extras:
        hs = make("mixed", True, score=True)
        hs.reset()
        hs.iterate(args.iters)                       # warm-up
        s0, _, q0 = hs.profile()
        hs.reset()
        _, hists, _ = hs.iterate(args.iters)
        s1, _, q1 = hs.profile()
        its = max(q1["iters"] - q0["iters"], 1)
        score = {"method": "LOMR, Appendix A score in the global cap, mixed",
                 "spai_ms_per_iter": sum(s1[k] - s0[k] for k in s1 if not k.startswith("pcg")) / its,
                 "select_ms_per_iter": (s1["select"] - s0["select"]) / its,
                 "resid_fro": float(hists[-1]), "resid_fro_magnitude_rule": r_mixed,
                 "iters": args.iters}
        hs.close()
        log("score drop:", json.dumps(score))

    # ---------------- batched form: 256 random geometric-graph Laplacians in one handle
    batched = None if args.no_batched else batched_leg(S, W, torch, np)

    # ---------------- differentiation form: the loss and its gradients
    loss = None if args.no_extras else loss_leg(S, W, torch, np)

    small = None if args.no_extras else small_configs_leg(S, W, torch, np)
    if small:
        log("small configurations:", json.dumps(small))

    cpu = None if args.no_cpu else cpu_baseline(A, cpu_state[0], cpu_state[1], cpu_state[2])
    if cpu:
        log("cpu baseline:", json.dumps(cpu))

    value = args.iters * args.steps / T
    out = {
        "metric": "SPAI iters/s & HBM GB/s (n=885k), mixed vs FP64 at same ‖I−AM‖_F",
        "value": value,
        "unit": "SPAI iters/s",
        "value_definition": "LOMR iterations per second of whole steps: the iterations of a "
                            "step divided by the step's time, PCG included; the iteration "
                            "rate alone is spai_iters_per_s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed: fp32 values, fp64 reductions",
        "data": "synthetic",
        "config": {
            "workload": f"lognormal{N}: 3D 7-point diffusion, lognormal face coefficients, {N}^3 "
                        f"(n={n}, nnz={nnzA}); LOMR, float32 values with float64 sums, global cap "
                        f"2 nnz(A), {args.iters} iterations, then PCG with {args.nrhs} RHS to 1e-8",
            "global_batch": args.nrhs, "seq_len": 0, "parallelism": "none (1 GPU)",
        },
        "roofline": roof_spai,
        "roofline_spai_iteration": roof_iter,
        "roofline_per_kernel": roofs,
        "roofline_spai_kernels": spai_kernels,
        "iteration_alg_bytes": it_bytes,
        "iteration_alg_gbs": it_gbs,
        "iteration_min_bytes": min_bytes,
        "iteration_min_gbs": min_gbs,
        "cpu_baseline": cpu,
        "spai_ms_per_iter": spai_ms / max(iters_timed, 1),
        "spai_iters_per_s": 1e3 / max(spai_ms / max(iters_timed, 1), 1e-9),
        "pcg_ms_per_step": ph_ms["pcg"] / args.steps,
        "phase_ms_per_iter": {k: v / max(iters_timed, 1) for k, v in ph_ms.items()
                              if not k.startswith("pcg")},
        # bytes each phase of this design moves (its own candidate lists included), from
        # the device counters; not the iteration's algorithmic bytes above
        "design_gbs_per_phase": {k: alg[k] / (per_iter_ms[k] * 1e-3) / 1e9
                                 if per_iter_ms[k] > 0 else None for k in alg},
        "design_bytes_per_phase": alg,
        "phase_calls_per_iter": {k: ph_calls[k] / max(iters_timed, 1) for k in alg},
        "resid_fro": r_mixed,
        "pcg_iters_max": int(pcg[0].max()) if pcg else None,
        "mixed_vs_f64": f64,
        "jacobi_lomr": jac,
        "autotune": tuned,
        "score_lomr": score,
        "spectrum_of_m": spec,
        "batched_geo256": batched,
        "loss_grid9_512": loss,
        "small_configs_f64": small,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
