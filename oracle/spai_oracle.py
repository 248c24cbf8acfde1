"""Plain FP64 CPU oracle for the global SPAI iterations and the SPAI-preconditioned CG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check of ``__graft_entry__`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and imports nothing from the package.

Everything is float64 with ``scipy.sparse`` matrices.  Library primitives
(sparse product, sparse sum, transpose, sort) serve as single steps; there is no
blocking, fusion or reordering beyond the algorithms as the paper states them.
Iterates are kept column-compressed (CSC) because columns are the independent
unit of the objective (Section 2).  Support means the set of nonzero entries,
as in the definitions of supp(P) and supp(M) (Section 6.1, Appendix A): stored
zeros are removed.

Every function here is pinned by tests/test_oracle_pins.py against what the paper
and the mathematics fix (closed forms, the theorems of Sections 2-5, brute force on
small inputs, library routines for special cases).  Whole MR trajectories with
dropping are pinned where they have a closed form (a constant-diagonal A under a cap
that leaves room for the diagonal only: every iterate is a multiple of I).  Parity
unpinned: trajectories with dropping that keep off-diagonal entries (the drop rules and
the steps are pinned one by one, their composition over many iterations has no
independent reference).

Readings of points the paper leaves open (each is an argument, shared with the
GPU library's options):

* M_0 = (tr A / tr A^2) I, the Frobenius-optimal multiple of the identity
  (Section 2 says only "given an initial iterate").
* Explicit residual R_{i+1} = I - A M_{i+1} whenever dropping is active
  (Section 6.2); the implicit update is available for dropping-free runs.
* Drop rule on M (Appendix A, steps 1-3, with the cap of step 3 taken as the
  hard thresholding of Section 6.1, which is what the dropping experiments of
  Section 7.2 use): symmetrize, remove off-diagonal |m| < u, then cap.  The
  diagonal is never dropped and counts toward the cap.
* Drop rule on P (Section 6.1): hard thresholding with the same cap, no
  diagonal exemption.  MR's search direction P = R is not dropped.
* Ties: eq. (hard thresholding) has no unique minimiser when magnitudes tie at
  the cut.  With t the (b+1)-th largest candidate magnitude (b = budget), keep
  exactly the entries with |x| > t (1 + eta).  This never exceeds the budget,
  keeps symmetric pairs together and equals the textbook top-b whenever the
  b-th largest magnitude exceeds t (1 + eta).
* Per-column cap (not in the paper, whose caps are global): column j keeps at
  most k_j entries; on the symmetrized M an off-diagonal (r, c) survives only if
  it passes both column thresholds, which keeps M symmetric.
* LOMR degeneracy: when c_i <= 1e-14 (AR,AR)(AP,AP) (Theorem 4.2's c_i is a
  2x2 Gram determinant) take the MR step (gamma = 0).
* Stop when ||I - A M_i||_F / sqrt(n) <= tol (the "backward error" of
  Section 7.2; Tables 5-6 are consistent with this scaling).
* Heuristic drop score (Appendix A, optional, global cap only): the entries of
  the symmetrized, small-dropped M~ are ranked by the effect of dropping them on
  ||I - A M~||_F^2, s_kl = m_kl^2 ||A e_k||^2 + 2 m_kl (A R~)_kl with R~ = I - A M~
  (the derivation's square kept; the printed rule lacks it), and since M stays
  symmetric they are dropped in symmetric pairs ranked by s_kl + s_lk, which is
  exactly the effect of dropping that pair alone.  Ties as above with the band
  sigma > t + eta |t| (scores may be negative).
* Pi-weighted variants (Section 5): the MR step of Algorithm 5 has numerator
  (Z, A Z), the one the Pi^{-1}-weighted product gives and Algorithm 8 uses at
  i = 0 (the printed (Z, Pi A Z) is read as a typo); their drop rules are the
  ones above with Z in R's place.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "frob", "fnorm", "initial_iterate", "residual", "DropRule", "cap_counts",
    "drop_main", "drop_direction", "mr", "cg", "lomr", "run", "pcg", "pcg_block",
    "loss", "loss_grad", "OracleBreakdown", "column_residual", "row_residual",
    "grad_m_entry", "grad_a_entry", "jacobi", "mr_spd", "cg_spd", "lomr_spd", "run_spd",
    "extreme_eigenvalues", "lanczos", "heuristic_scores", "pair_scores",
]

UNIT_ROUNDOFF = 2.0 ** -53
LOMR_DEGENERACY = 1e-14


class OracleBreakdown(RuntimeError):
    """Raised when a step size is undefined (e.g. (P, AP)_F <= 0 in CG)."""


# ----------------------------------------------------------------------------
# basic operations (Section 2)
# ----------------------------------------------------------------------------

def _csc(X) -> sp.csc_matrix:
    X = sp.csc_matrix(X, dtype=np.float64)
    X.sum_duplicates()
    X.eliminate_zeros()
    X.sort_indices()
    return X


def frob(X, Y) -> float:
    """Frobenius inner product (X, Y)_F = tr(X^T Y) (Section 2)."""
    return float(sp.csc_matrix(X).multiply(sp.csc_matrix(Y)).sum())


def fnorm(X) -> float:
    """Frobenius norm ||X||_F = (X, X)_F^(1/2) (Section 2)."""
    return math.sqrt(frob(X, X))


def initial_iterate(A) -> tuple[float, sp.csc_matrix]:
    """M_0 = c I with c = tr(A) / tr(A^2), i.e. argmin_c ||I - c A||_F."""
    A = sp.csr_matrix(A)
    t1 = float(A.diagonal().sum())
    t2 = float(A.multiply(A.T).sum())          # tr(A A) = sum_ij a_ij a_ji
    c = t1 / t2
    n = A.shape[0]
    return c, _csc(c * sp.identity(n, format="csc"))


def residual(A, M) -> sp.csc_matrix:
    """R = I - A M (the objective's residual, Section 2; explicit update, Section 6.2)."""
    n = A.shape[0]
    return _csc(sp.identity(n, format="csc") - sp.csr_matrix(A) @ sp.csc_matrix(M))


# ----------------------------------------------------------------------------
# dropping (Section 6.1 hard thresholding; Appendix A steps 1-3)
# ----------------------------------------------------------------------------

@dataclass
class DropRule:
    """What the drop operators D_M and D_P do.

    mode: "none" | "global" | "column".  ``m`` is the global count cap and
    ``k`` the per-column caps (array of length n), as produced by
    :func:`cap_counts`.  ``u`` is the small-entry threshold of Appendix A
    step 2 (0 disables it), ``eta`` the tie band, ``symmetrize`` Appendix A
    step 1.  ``score`` (global cap only): rank the entries of M by the heuristic
    of Appendix A (:func:`heuristic_scores`, :func:`pair_scores`) instead of by
    magnitude; the drop of P stays hard thresholding.
    """
    mode: str = "none"
    m: int = 0
    k: np.ndarray | None = None
    u: float = UNIT_ROUNDOFF
    eta: float = 1e-9
    symmetrize: bool = True
    score: bool = False

    @staticmethod
    def no_drop() -> "DropRule":
        return DropRule(mode="none", u=0.0, symmetrize=False)


def cap_counts(A, mode: str, value: float, relative: bool):
    """Turn a cap spec into counts: global m, or per-column k_j.

    relative global: m = round(value * nnz(A)); relative column:
    k_j = round(value * nnz(A e_j)); otherwise the value itself.
    """
    A = sp.csc_matrix(A)
    if mode == "global":
        return int(round(value * A.nnz)) if relative else int(round(value))
    if mode == "column":
        counts = np.diff(A.indptr).astype(np.float64)
        if relative:
            return np.rint(value * counts).astype(np.int64)
        return np.full(A.shape[1], int(round(value)), dtype=np.int64)
    return None


def _entries(X: sp.csc_matrix):
    cols = np.repeat(np.arange(X.shape[1]), np.diff(X.indptr))
    return X.indices.astype(np.int64), cols, X.data.copy()


def _kth_largest_per_column(cols, mags, ncols, kk):
    """t_c = (kk_c + 1)-th largest of mags in column c, or 0 if there are <= kk_c."""
    t = np.zeros(ncols)
    if len(mags) == 0:
        return t
    # scatter each column's magnitudes into one row of a padded table, sort rows
    order = np.argsort(cols, kind="stable")
    sc, sm = cols[order], mags[order]
    count = np.bincount(sc, minlength=ncols)
    start = np.concatenate(([0], np.cumsum(count)[:-1]))
    pos = np.arange(len(sc)) - start[sc]
    table = np.full((ncols, int(count.max())), -np.inf)
    table[sc, pos] = sm
    table = -np.sort(-table, axis=1)                 # each row in descending order
    has = count > kk
    t[has] = table[np.nonzero(has)[0], kk[has]]
    return t


def _from_entries(rows, cols, vals, shape):
    return _csc(sp.csc_matrix((vals, (rows, cols)), shape=shape))


def heuristic_scores(A, X) -> sp.csc_matrix:
    """The effect on ||R||_F^2 of dropping each stored entry of X alone (Appendix A):
    s_kl = m_kl^2 ||A e_k||_2^2 + 2 m_kl (A R)_kl with R = I - A X, on X's pattern.
    The square on m_kl is the one the derivation carries (the printed selection rule
    omits it).  Dropping one entry per column changes ||R||_F^2 by exactly the sum of
    these; entries of one column also couple through (A e_k)^T (A e_r)."""
    A = sp.csr_matrix(A)
    X = _csc(X)
    R = residual(A, X)
    AR = sp.csr_matrix(A @ R)
    colnorm2 = np.asarray(A.multiply(A).sum(axis=0)).ravel()      # ||A e_k||_2^2
    rows, cols, vals = _entries(X)
    ar = np.asarray(AR[rows, cols]).ravel()
    return _csc(sp.csc_matrix((vals * vals * colnorm2[rows] + 2.0 * vals * ar, (rows, cols)),
                              shape=X.shape))


def pair_scores(A, X) -> sp.csc_matrix:
    """For a symmetric X: sigma_kl = s_kl + s_lk, the effect on ||R||_F^2 of dropping the
    symmetric pair {(k, l), (l, k)} alone (its two entries lie in different columns, so
    they do not couple); on the diagonal, s_kk itself."""
    Sc = heuristic_scores(A, X)
    P = _csc(Sc + Sc.T)
    P.setdiag(Sc.diagonal())
    return _csc(P)


def _record(info, cand, keep, band, t, rows=None, cols=None, vals=None, thr=None):
    """What a drop did (diagnostics only, no effect on the result): the candidates it
    saw, the entries it kept, the band (candidates dropped within the tie band of the
    cut, |x| >= t (1 - eta) for the threshold t before the tie factor: entries that a
    last-bit difference in the values cannot move across its edge) and the global
    threshold t (None otherwise).
    With info["keep_candidates"] set, also the candidate entries (rows, cols, vals) and
    each one's threshold before the tie factor (the global t, or the column threshold)."""
    if info is not None:
        info.update({"cand": int(cand.sum()), "kept": int(keep.sum()), "band": int(band),
                     "t": None if t is None else float(t)})
        if info.get("keep_candidates") and rows is not None:
            info["candidates"] = (rows[cand], cols[cand], vals[cand],
                                  None if thr is None else np.asarray(thr)[cand])


def drop_main(X, rule: DropRule, A=None, info=None) -> sp.csc_matrix:
    """D_M: the drop rule on the main iterate (Appendix A steps 1-3 + Section 6.1).
    With rule.score the cap of step 3 ranks by the pair scores of Appendix A (A needed).
    info (optional dict): receives the counts of _record."""
    X = _csc(X)
    n = X.shape[0]
    if rule.symmetrize:                                  # step 1: M := (M + M^T) / 2
        X = _csc((X + X.T.tocsc()) * 0.5)
    rows, cols, vals = _entries(X)
    diag = rows == cols
    keep = vals != 0.0
    if rule.u > 0.0:                                     # step 2: off-diagonal |m| < u
        keep &= diag | (np.abs(vals) >= rule.u)
    cand = keep.copy()
    band, tcut = 0, None
    if rule.mode == "global":                            # step 3: cap |supp(M)| <= m
        if keep.sum() > rule.m:
            ndiag = int((keep & diag).sum())
            b = rule.m - ndiag
            if b < 0:
                raise ValueError("cap below the number of diagonal entries")
            if rule.score:
                if not rule.symmetrize:
                    raise ValueError("the score drops symmetric pairs: symmetrize first")
                Xk = _from_entries(rows[keep], cols[keep], vals[keep], X.shape)
                Sg = pair_scores(A, Xk)
                sig = np.asarray(Sg[rows, cols]).ravel()
                cand_s = sig[keep & ~diag]
                if len(cand_s) > b:
                    t = np.sort(cand_s)[::-1][b]
                    keep &= diag | (sig > t + rule.eta * abs(t))
                    band = int((cand & ~keep & (sig >= t - rule.eta * abs(t))).sum())
                    tcut = t
            else:
                mags = np.abs(vals[keep & ~diag])
                if len(mags) > b:
                    t = np.sort(mags)[::-1][b]
                    keep &= diag | (np.abs(vals) > t * (1.0 + rule.eta))
                    band = int((cand & ~keep & (np.abs(vals) >= t * (1.0 - rule.eta))).sum())
                    tcut = t
        thr = None if tcut is None else np.full(len(vals), tcut)
    elif rule.mode == "column":
        k = np.asarray(rule.k, dtype=np.int64)
        if np.any(k < 1):
            raise ValueError("column cap below one (the diagonal)")
        off = keep & ~diag
        t = _kth_largest_per_column(cols[off], np.abs(vals[off]), n, k - 1)
        thr = np.maximum(t[rows], t[cols]) if rule.symmetrize else t[cols]
        keep &= diag | (np.abs(vals) > thr * (1.0 + rule.eta))
        band = int((cand & ~keep & (thr > 0) & (np.abs(vals) >= thr * (1.0 - rule.eta))).sum())
    else:
        thr = None
    _record(info, cand, keep, band, tcut, rows, cols, vals, thr)
    return _from_entries(rows[keep], cols[keep], vals[keep], X.shape)


def drop_direction(X, rule: DropRule, info=None) -> sp.csc_matrix:
    """D_P: hard thresholding of a search direction (Section 6.1), no diagonal exemption.
    info (optional dict): receives the counts of _record."""
    X = _csc(X)
    rows, cols, vals = _entries(X)
    keep = vals != 0.0
    cand = keep.copy()
    band, tcut, thr = 0, None, None
    if rule.mode == "global":
        if keep.sum() > rule.m:
            mags = np.abs(vals[keep])
            t = np.sort(mags)[::-1][rule.m]
            keep &= np.abs(vals) > t * (1.0 + rule.eta)
            band = int((cand & ~keep & (np.abs(vals) >= t * (1.0 - rule.eta))).sum())
            tcut = t
            thr = np.full(len(vals), t)
    elif rule.mode == "column":
        k = np.asarray(rule.k, dtype=np.int64)
        t = _kth_largest_per_column(cols[keep], np.abs(vals[keep]), X.shape[1], k)
        thr = t[cols]
        keep &= np.abs(vals) > thr * (1.0 + rule.eta)
        band = int((cand & ~keep & (thr > 0) & (np.abs(vals) >= thr * (1.0 - rule.eta))).sum())
    _record(info, cand, keep, band, tcut, rows, cols, vals, thr)
    return _from_entries(rows[keep], cols[keep], vals[keep], X.shape)


# ----------------------------------------------------------------------------
# the three global iterations
# ----------------------------------------------------------------------------

@dataclass
class Result:
    M: sp.csc_matrix
    P: sp.csc_matrix | None
    resid: list = field(default_factory=list)     # ||R_i||_F, i = 0..iters
    scalars: list = field(default_factory=list)   # per iteration dict
    nnz_m: list = field(default_factory=list)
    nnz_p: list = field(default_factory=list)
    drops: list = field(default_factory=list)     # per iteration {"M": info, "P": info}
    iters: int = 0
    status: str = "maxiter"
    c: float = 0.0


def _converged(rnorm, n, tol):
    return tol > 0.0 and rnorm / math.sqrt(n) <= tol


def mr(A, rule: DropRule, max_iter: int, tol: float = 0.0, explicit: bool = True,
       M0=None, keep_candidates: bool = False) -> Result:
    """Minimal residual with matrix iterates (Algorithm 1).

    alpha_i = (R_i, A R_i)_F / ||A R_i||_F^2 ; M_{i+1} = D_M(M_i + alpha_i R_i).
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    c, Minit = initial_iterate(A)
    M = Minit if M0 is None else _csc(M0)
    R = residual(A, M)
    out = Result(M, None, c=c)
    out.resid.append(fnorm(R))
    out.nnz_m.append(M.nnz)
    if _converged(out.resid[-1], n, tol):
        out.status = "converged"
        return out
    for i in range(max_iter):
        AR = _csc(A @ R)
        ar_ar = frob(AR, AR)
        if ar_ar == 0.0:
            out.status = "converged"
            break
        r_ar = frob(R, AR)
        alpha = r_ar / ar_ar
        dm = {"keep_candidates": keep_candidates}
        M = drop_main(M + alpha * R, rule, A, info=dm)
        R = residual(A, M) if explicit else _csc(R - alpha * AR)
        out.scalars.append({"alpha": alpha, "r_ar": r_ar, "ar_ar": ar_ar})
        out.drops.append({"M": dm, "P": None})
        out.resid.append(fnorm(R))
        out.nnz_m.append(M.nnz)
        out.iters = i + 1
        if _converged(out.resid[-1], n, tol):
            out.status = "converged"
            break
    out.M = M
    return out


def cg(A, rule: DropRule, max_iter: int, tol: float = 0.0, explicit: bool = True,
       M0=None) -> Result:
    """Conjugate gradient with matrix iterates (Algorithm 3).

    P_0 = D_P(R_0); alpha_i = ||R_i||^2 / (P_i, A P_i); M_{i+1} = D_M(M_i + alpha_i P_i);
    beta_{i+1} = ||R_{i+1}||^2 / ||R_i||^2; P_{i+1} = D_P(R_{i+1} + beta_{i+1} P_i).
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    c, Minit = initial_iterate(A)
    M = Minit if M0 is None else _csc(M0)
    R = residual(A, M)
    P = drop_direction(R, rule)
    rr = frob(R, R)
    out = Result(M, P, c=c)
    out.resid.append(math.sqrt(rr))
    out.nnz_m.append(M.nnz)
    out.nnz_p.append(P.nnz)
    if _converged(out.resid[-1], n, tol):
        out.status = "converged"
        return out
    for i in range(max_iter):
        if rr == 0.0:
            out.status = "converged"
            break
        AP = _csc(A @ P)
        p_ap = frob(P, AP)
        if not p_ap > 0.0:
            out.status = "breakdown"
            break
        alpha = rr / p_ap
        dm, dp = {}, {}
        M = drop_main(M + alpha * P, rule, A, info=dm)
        R = residual(A, M) if explicit else _csc(R - alpha * AP)
        rr_new = frob(R, R)
        beta = rr_new / rr
        P = drop_direction(R + beta * P, rule, info=dp)
        out.scalars.append({"alpha": alpha, "beta": beta, "p_ap": p_ap, "rr": rr})
        out.drops.append({"M": dm, "P": dp})
        rr = rr_new
        out.resid.append(math.sqrt(rr))
        out.nnz_m.append(M.nnz)
        out.nnz_p.append(P.nnz)
        out.iters = i + 1
        if _converged(out.resid[-1], n, tol):
            out.status = "converged"
            break
    out.M, out.P = M, P
    return out


def lomr_coefficients(r_ar, ar_ar, ar_ap, r_ap, ap_ap, first: bool):
    """(delta_i, gamma_i) of Theorem 4.2 / Algorithm 4, with the MR step when degenerate."""
    if first:
        return r_ar / ar_ar, 1.0, False
    c = ar_ar * ap_ap - ar_ap * ar_ap
    if not c > LOMR_DEGENERACY * ar_ar * ap_ap:
        return r_ar / ar_ar, 0.0, True
    delta = (ap_ap * r_ar - ar_ap * r_ap) / c
    gamma = (ar_ar * r_ap - ar_ap * r_ar) / c
    return delta, gamma, False


def lomr(A, rule: DropRule, max_iter: int, tol: float = 0.0, explicit: bool = True,
         M0=None, P0=None, keep_candidates: bool = False) -> Result:
    """Locally optimal minimal residual (Definition 4.1, Theorem 4.2, Algorithm 4).

    M_{i+1} = D_M(M_i + delta_i R_i + gamma_i P_{i-1}), P_i = D_P(delta_i R_i + gamma_i P_{i-1}),
    with P_{-1} = 0 and the MR step at i = 0.  Given P0 (the direction P_{i-1} of a run
    in progress, with M0 its iterate M_i), the run continues from there instead: its
    first step is a LOMR step over span{R_i, P0}.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    c, Minit = initial_iterate(A)
    M = Minit if M0 is None else _csc(M0)
    R = residual(A, M)
    P = _csc(sp.csc_matrix((n, n))) if P0 is None else _csc(P0)
    out = Result(M, P, c=c)
    out.resid.append(fnorm(R))
    out.nnz_m.append(M.nnz)
    out.nnz_p.append(P.nnz)
    if _converged(out.resid[-1], n, tol):
        out.status = "converged"
        return out
    for i in range(max_iter):
        AR = _csc(A @ R)
        AP = _csc(A @ P)
        ar_ar = frob(AR, AR)
        if ar_ar == 0.0:
            out.status = "converged"
            break
        r_ar = frob(R, AR)
        ar_ap = frob(AR, AP)
        r_ap = frob(R, AP)
        ap_ap = frob(AP, AP)
        first = i == 0 and P0 is None
        delta, gamma, fell_back = lomr_coefficients(r_ar, ar_ar, ar_ap, r_ap, ap_ap, first)
        dm, dp = {"keep_candidates": keep_candidates}, {"keep_candidates": keep_candidates}
        M = drop_main(M + delta * R + gamma * P, rule, A, info=dm)
        Rnew = residual(A, M) if explicit else _csc(R - delta * AR - gamma * AP)
        P = drop_direction(delta * R + gamma * P, rule, info=dp)
        R = Rnew
        out.scalars.append({"delta": delta, "gamma": gamma, "r_ar": r_ar, "ar_ar": ar_ar,
                            "ar_ap": ar_ap, "r_ap": r_ap, "ap_ap": ap_ap,
                            "mr_fallback": fell_back})
        out.drops.append({"M": dm, "P": dp})
        out.resid.append(fnorm(R))
        out.nnz_m.append(M.nnz)
        out.nnz_p.append(P.nnz)
        out.iters = i + 1
        if _converged(out.resid[-1], n, tol):
            out.status = "converged"
            break
    out.M, out.P = M, P
    return out


# ----------------------------------------------------------------------------
# Pi-weighted variants (Section 5, Algorithms 5, 7 and 8)
# ----------------------------------------------------------------------------

def jacobi(A) -> sp.csr_matrix:
    """Pi = D_A^{-1}, the preconditioner of Section 5 and of the experiments of Section 7."""
    return sp.diags(1.0 / sp.csr_matrix(A).diagonal()).tocsr()


def mr_spd(A, Pi, rule: DropRule, max_iter: int, tol: float = 0.0, explicit: bool = True,
           M0=None) -> Result:
    """MR with Pi-weighted inner products (Algorithm 5).

    Z_i = Pi R_i; alpha_i = (Z_i, A Z_i)_F / (A Z_i, Pi A Z_i)_F;
    M_{i+1} = D_M(M_i + alpha_i Z_i).  Section 5 weights the Frobenius product by Pi^{-1}
    so that Pi A is self-adjoint; in that product the MR step for Pi A with residual Z
    has numerator (Z, A Z) (it minimises (R_{i+1}, Pi R_{i+1})), and Algorithm 8 takes
    the same numerator at i = 0, so the printed (Z_i, Pi A Z_i) is read as (Z_i, A Z_i).
    Z, like MR's R, is not dropped.
    """
    A = sp.csr_matrix(A)
    Pi = sp.csr_matrix(Pi)
    n = A.shape[0]
    c, Minit = initial_iterate(A)
    M = Minit if M0 is None else _csc(M0)
    R = residual(A, M)
    out = Result(M, None, c=c)
    out.resid.append(fnorm(R))
    out.nnz_m.append(M.nnz)
    if _converged(out.resid[-1], n, tol):
        out.status = "converged"
        return out
    for i in range(max_iter):
        Z = _csc(Pi @ R)
        AZ = _csc(A @ Z)
        az_paz = frob(AZ, _csc(Pi @ AZ))
        if az_paz == 0.0:
            out.status = "converged"
            break
        z_az = frob(Z, AZ)
        alpha = z_az / az_paz
        M = drop_main(M + alpha * Z, rule, A)
        R = residual(A, M) if explicit else _csc(R - alpha * AZ)
        out.scalars.append({"alpha": alpha, "z_az": z_az, "az_paz": az_paz})
        out.resid.append(fnorm(R))
        out.nnz_m.append(M.nnz)
        out.iters = i + 1
        if _converged(out.resid[-1], n, tol):
            out.status = "converged"
            break
    out.M = M
    return out


def cg_spd(A, Pi, rule: DropRule, max_iter: int, tol: float = 0.0, explicit: bool = True,
           M0=None) -> Result:
    """Matrix CG preconditioned by Pi (Algorithm 7).

    Z_0 = Pi R_0, P_0 = D_P(Z_0); alpha_i = (R_i, Z_i)_F / (P_i, A P_i)_F;
    M_{i+1} = D_M(M_i + alpha_i P_i); Z_{i+1} = Pi R_{i+1};
    beta_{i+1} = (R_{i+1}, Z_{i+1})_F / (R_i, Z_i)_F; P_{i+1} = D_P(Z_{i+1} + beta_{i+1} P_i).
    """
    A = sp.csr_matrix(A)
    Pi = sp.csr_matrix(Pi)
    n = A.shape[0]
    c, Minit = initial_iterate(A)
    M = Minit if M0 is None else _csc(M0)
    R = residual(A, M)
    Z = _csc(Pi @ R)
    P = drop_direction(Z, rule)
    rz = frob(R, Z)
    out = Result(M, P, c=c)
    out.resid.append(fnorm(R))
    out.nnz_m.append(M.nnz)
    out.nnz_p.append(P.nnz)
    if _converged(out.resid[-1], n, tol):
        out.status = "converged"
        return out
    for i in range(max_iter):
        if rz == 0.0:
            out.status = "converged"
            break
        AP = _csc(A @ P)
        p_ap = frob(P, AP)
        if not p_ap > 0.0:
            out.status = "breakdown"
            break
        alpha = rz / p_ap
        M = drop_main(M + alpha * P, rule, A)
        R = residual(A, M) if explicit else _csc(R - alpha * AP)
        Z = _csc(Pi @ R)
        rz_new = frob(R, Z)
        beta = rz_new / rz
        P = drop_direction(Z + beta * P, rule)
        out.scalars.append({"alpha": alpha, "beta": beta, "p_ap": p_ap, "rz": rz})
        rz = rz_new
        out.resid.append(fnorm(R))
        out.nnz_m.append(M.nnz)
        out.nnz_p.append(P.nnz)
        out.iters = i + 1
        if _converged(out.resid[-1], n, tol):
            out.status = "converged"
            break
    out.M, out.P = M, P
    return out


def lomr_spd(A, Pi, rule: DropRule, max_iter: int, tol: float = 0.0, explicit: bool = True,
             M0=None) -> Result:
    """Locally optimal MR with Pi-weighted inner products (Algorithm 8).

    Z_i = Pi R_i; (delta_i, gamma_i) from the five products (Z, AZ), (AZ, Pi AZ),
    (AZ, Pi AP), (Z, AP), (AP, Pi AP) in the roles Theorem 4.2 gives (R, AR), (AR, AR),
    (AR, AP), (R, AP), (AP, AP); M_{i+1} = D_M(M_i + delta_i Z_i + gamma_i P_{i-1}),
    P_i = D_P(delta_i Z_i + gamma_i P_{i-1}), P_{-1} = 0, the MR step at i = 0.
    """
    A = sp.csr_matrix(A)
    Pi = sp.csr_matrix(Pi)
    n = A.shape[0]
    c, Minit = initial_iterate(A)
    M = Minit if M0 is None else _csc(M0)
    R = residual(A, M)
    P = _csc(sp.csc_matrix((n, n)))
    out = Result(M, P, c=c)
    out.resid.append(fnorm(R))
    out.nnz_m.append(M.nnz)
    out.nnz_p.append(0)
    if _converged(out.resid[-1], n, tol):
        out.status = "converged"
        return out
    for i in range(max_iter):
        Z = _csc(Pi @ R)
        AZ = _csc(A @ Z)
        AP = _csc(A @ P)
        PAZ = _csc(Pi @ AZ)
        PAP = _csc(Pi @ AP)
        az_paz = frob(AZ, PAZ)
        if az_paz == 0.0:
            out.status = "converged"
            break
        z_az = frob(Z, AZ)
        az_pap = frob(AZ, PAP)
        z_ap = frob(Z, AP)
        ap_pap = frob(AP, PAP)
        delta, gamma, fell_back = lomr_coefficients(z_az, az_paz, az_pap, z_ap, ap_pap, i == 0)
        M = drop_main(M + delta * Z + gamma * P, rule, A)
        Rnew = residual(A, M) if explicit else _csc(R - delta * AZ - gamma * AP)
        P = drop_direction(delta * Z + gamma * P, rule)
        R = Rnew
        out.scalars.append({"delta": delta, "gamma": gamma, "z_az": z_az, "az_paz": az_paz,
                            "az_pap": az_pap, "z_ap": z_ap, "ap_pap": ap_pap,
                            "mr_fallback": fell_back})
        out.resid.append(fnorm(R))
        out.nnz_m.append(M.nnz)
        out.nnz_p.append(P.nnz)
        out.iters = i + 1
        if _converged(out.resid[-1], n, tol):
            out.status = "converged"
            break
    out.M, out.P = M, P
    return out


def run(method: str, A, rule: DropRule, max_iter: int, tol: float = 0.0, **kw) -> Result:
    return {"mr": mr, "cg": cg, "lomr": lomr}[method](A, rule, max_iter, tol, **kw)


def run_spd(method: str, A, Pi, rule: DropRule, max_iter: int, tol: float = 0.0,
            **kw) -> Result:
    """The Pi-weighted variant of `method` (Algorithms 5, 7, 8)."""
    return {"mr": mr_spd, "cg": cg_spd, "lomr": lomr_spd}[method](A, Pi, rule, max_iter, tol,
                                                                   **kw)


# ----------------------------------------------------------------------------
# vector PCG with the SPAI as preconditioner (Sections 1 and 7, Experiments 04/06)
# ----------------------------------------------------------------------------

def pcg(A, M, b, rtol: float = 1e-8, max_iter: int = 10000):
    """Textbook preconditioned CG for one right-hand side, z = M r, x_0 = 0.

    Stops when ||r||_2 <= rtol ||b||_2 on the recursively updated residual.
    Returns (x, iterations, status) with status "converged", "maxiter" or
    "indefinite" ((r, z) <= 0 or (p, A p) <= 0).
    """
    A = sp.csr_matrix(A)
    M = sp.csr_matrix(M)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.sqrt(b @ b))
    if bnorm == 0.0:
        return x, 0, "converged"
    r = b.copy()
    z = M @ r
    rz = float(r @ z)
    p = z.copy()
    for it in range(1, max_iter + 1):
        if not rz > 0.0:
            return x, it - 1, "indefinite"
        q = A @ p
        pq = float(p @ q)
        if not pq > 0.0:
            return x, it - 1, "indefinite"
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        if float(np.sqrt(r @ r)) <= rtol * bnorm:
            return x, it, "converged"
        z = M @ r
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, max_iter, "maxiter"


def pcg_block(A, M, B, rtol: float = 1e-8, max_iter: int = 10000):
    """Run :func:`pcg` independently on each column of B (shape n x nrhs)."""
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B)
    iters, status = [], []
    for j in range(B.shape[1]):
        x, it, st = pcg(A, M, B[:, j], rtol, max_iter)
        X[:, j] = x
        iters.append(it)
        status.append(st)
    return X, np.array(iters), status


# ----------------------------------------------------------------------------
# spectrum of a symmetric iterate (the lambda_min / lambda_max of Tables 4-6; whether a
# SPAI is positive definite, Section 7.1)
# ----------------------------------------------------------------------------

LANCZOS_INVARIANT = 1e-12


def extreme_eigenvalues(S) -> tuple[float, float]:
    """(lambda_min, lambda_max) of a symmetric matrix: the definition, through a dense
    symmetric eigensolver (small matrices only)."""
    w = np.linalg.eigvalsh(sp.csr_matrix(S).toarray())
    return float(w[0]), float(w[-1])


def lanczos(S, steps: int, v0):
    """The Lanczos process with full reorthogonalisation, written from its textbook
    definition (Golub and Van Loan, Matrix Computations, Section 10.1): v_0 = v0/||v0||;
    per step w = S v_j, Gram-Schmidt against all previous v twice, alpha_j = v_j^T S v_j
    (the sum of the two projections on v_j), beta_j = ||w||, v_{j+1} = w / beta_j; stop
    early when beta_j <= 1e-12 max_{i<=j}(|alpha_i| + beta_i).  At most min(steps, n)
    steps.  Returns (theta_min, theta_max, res_min, res_max, steps taken): the extreme
    eigenvalues of T_k = tridiag(beta, alpha, beta) and beta_k |y_k| for their unit
    eigenvectors y (the distance to the nearest eigenvalue of S is at most res)."""
    S = sp.csr_matrix(S)
    n = S.shape[0]
    K = min(int(steps), n)
    v0 = np.asarray(v0, dtype=np.float64)
    V = np.zeros((n, K + 1))
    V[:, 0] = v0 / np.linalg.norm(v0)
    alpha, beta = [], []
    scale = 0.0
    for j in range(K):
        w = S @ V[:, j]
        Vj = V[:, :j + 1]
        h1 = Vj.T @ w
        w = w - Vj @ h1
        h2 = Vj.T @ w
        w = w - Vj @ h2
        a = float(h1[j] + h2[j])
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        scale = max(scale, abs(a) + b)
        if b <= LANCZOS_INVARIANT * scale:
            break
        if j + 1 < K:
            V[:, j + 1] = w / b
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    theta, Y = np.linalg.eigh(T)
    res = beta[k - 1] * np.abs(Y[k - 1, :])
    return float(theta[0]), float(theta[-1]), float(res[0]), float(res[-1]), k


# ----------------------------------------------------------------------------
# differentiable objective f(M) = ||I - A M||_F^2 (Section 2 and its gradient)
# ----------------------------------------------------------------------------

def loss(A, M) -> float:
    """f(M) = ||I - A M||_F^2 (the objective of Section 2)."""
    return frob(residual(A, M), residual(A, M))


def loss_grad(A, M):
    """Gradients of f in the stored values of M and of A.

    With R = I - A M: df = -2 (R, dA M + A dM)_F, so df/dM = -2 A^T R and
    df/dA = -2 R M^T; each is restricted to the pattern of its argument and
    returned as a CSR matrix on that pattern (A's and M's patterns as given).
    For symmetric A the first is the gradient of Section 2.
    """
    A = sp.csr_matrix(A)
    M = sp.csr_matrix(M)
    R = residual(A, M)
    GM = -2.0 * (A.T @ R)
    GA = -2.0 * (R @ M.T)
    return _on_pattern(GA, A), _on_pattern(GM, M)


def _on_pattern(G, P):
    P = sp.csr_matrix(P)
    P.sort_indices()
    G = sp.csr_matrix(G)
    rows = np.repeat(np.arange(P.shape[0]), np.diff(P.indptr))
    vals = np.asarray(G[rows, P.indices]).ravel()
    return sp.csr_matrix((vals, P.indices.copy(), P.indptr.copy()), shape=P.shape)


# ----------------------------------------------------------------------------
# single entries of the gradients, from one column / one row of R (for sampling
# full-size results: perturbing m_kj changes only column j of R, perturbing a_ik only
# row i)
# ----------------------------------------------------------------------------

def column_residual(A, M, j):
    """r_j = e_j - A m_j as a dense float64 vector (column j of R = I - A M).

    Pass A as CSR and M as CSC to avoid format conversions."""
    A = A if sp.isspmatrix_csr(A) else sp.csr_matrix(A)
    M = M if sp.isspmatrix_csc(M) else sp.csc_matrix(M)
    r = -(A @ M[:, j]).toarray().ravel()
    r[j] += 1.0
    return r


def row_residual(A, M, i):
    """R(i, :) = e_i^T - A(i, :) M as a dense float64 vector (A, M as CSR)."""
    A = A if sp.isspmatrix_csr(A) else sp.csr_matrix(A)
    M = M if sp.isspmatrix_csr(M) else sp.csr_matrix(M)
    row = -(A[i, :] @ M).toarray().ravel()
    row[i] += 1.0
    return row


def grad_m_entry(A, M, k, j, A_csc=None):
    """d f / d m_kj = -2 (A^T r_j)_k = -2 sum_u a_uk r_j(u) (A as CSR, M as CSC)."""
    A_csc = A_csc if A_csc is not None else sp.csc_matrix(A)
    r = column_residual(A, M, j)
    col = A_csc[:, k]
    return float(-2.0 * (col.T @ r)[0])


def grad_a_entry(A, M, i, k):
    """d f / d a_ik = -2 (R M^T)_ik = -2 sum_j R(i, j) m_kj (A, M as CSR)."""
    M = M if sp.isspmatrix_csr(M) else sp.csr_matrix(M)
    row = row_residual(A, M, i)
    return float(-2.0 * (M[k, :] @ row)[0])
