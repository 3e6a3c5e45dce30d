"""Leave-one-out jackknife of CP models, one submodel at a time, in float64
(test infrastructure only).

The fitting loop is Alg. 2's: remove slice p of the sampled mode from the
tensor, remove row p from the sampled mode's initial factor, and run CP-ALS
(Alg. 1) on what is left.  JK-CALS (Alg. 3) must reproduce exactly these
iterates up to rounding (Sec. 4.1, Case I and Case II), which is what the
parity tests check.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import cp


@dataclasses.dataclass
class ModelResult:
    """Outcome of one submodel fit.  Factors are stored reduced (row p of the
    sampled mode absent) unless produced by ``padded``."""

    left_out: object        # -1, one index, or a tuple of d indices (delete-d)
    sampled_mode: int
    U: List[np.ndarray]
    lam: np.ndarray
    normT2: float
    iters: int = 0
    converged: bool = False
    fallbacks: int = 0
    e_hist: List[float] = dataclasses.field(default_factory=list)
    fit_hist: List[float] = dataclasses.field(default_factory=list)
    lam_hist: List[np.ndarray] = dataclasses.field(default_factory=list)
    U_hist: Dict[int, List[np.ndarray]] = dataclasses.field(default_factory=dict)
    H_last: Optional[np.ndarray] = None
    M_last: Optional[np.ndarray] = None

    def padded(self, U: Optional[Sequence[np.ndarray]] = None) -> List[np.ndarray]:
        """Factors with zero rows re-inserted at the left-out indices of the
        sampled mode, matching the zero-padded multi-factor of Alg. 3."""
        U = self.U if U is None else U
        out = [u.copy() for u in U]
        rows = left_out_rows(self.left_out)
        if rows:
            n = self.sampled_mode
            I = out[n].shape[0] + len(rows)
            full = np.zeros((I, out[n].shape[1]))
            full[np.setdiff1d(np.arange(I), rows)] = out[n]
            out[n] = full
        return out


def left_out_rows(p) -> List[int]:
    """The samples a model leaves out: none for -1 (or a list of -1), one
    for an index, d for a list of d indices (delete-d jackknife)."""
    rows = [int(x) for x in np.atleast_1d(np.asarray(p)).ravel()]
    return sorted(x for x in rows if x >= 0)


def reduce_tensor(T: np.ndarray, sampled_mode: int, p) -> np.ndarray:
    """T_{-P}: T with the slices P of the sampled mode deleted (Alg. 2,
    slice removal; d slices for delete-d); the full tensor when P is empty
    (p = -1)."""
    T = np.asarray(T, dtype=np.float64)
    rows = left_out_rows(p)
    if not rows:
        return T
    return np.delete(T, rows, axis=sampled_mode)


def reduce_init(U_init: np.ndarray, p) -> np.ndarray:
    """The sampled mode's factor with the rows P deleted (Alg. 2, row
    removal)."""
    rows = left_out_rows(p)
    if not rows:
        return np.array(U_init, dtype=np.float64)
    return np.delete(np.asarray(U_init, dtype=np.float64), rows, axis=0)


def cp_als(T: np.ndarray, U0: Sequence[np.ndarray], sweeps: int, tol: float = 0.0,
           record_factors: Sequence[int] = (), sampled_mode: int = 0,
           left_out=-1) -> ModelResult:
    """CP-ALS (Alg. 1) on tensor T from factors U0, in float64.

    One sweep updates modes 0..N-1 in order; each update is MTTKRP, the
    Hadamard product of the other modes' Gramians, the normal-equation
    update, then column normalisation (lambda) and a Gram refresh.  After
    the last mode the squared error comes from the fast identity and
    fit = 1 - sqrt(max(e, 0)) / ||T||.  With tol > 0 the model stops after
    sweep t >= 2 once |fit_t - fit_{t-1}| < tol; tol = 0 runs exactly
    ``sweeps`` sweeps (the fixed-iteration protocol of Sec. 5.1).
    ``record_factors`` lists the sweep numbers (1-based) whose factors are
    kept in ``U_hist``.
    """
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    U = [np.array(u, dtype=np.float64) for u in U0]
    R = U[0].shape[1]
    unf = [cp.unfold(T, n) for n in range(N)]
    normT2 = float(np.sum(T * T))
    G = [cp.gram(u) for u in U]
    lam = np.ones(R)
    res = ModelResult(left_out, sampled_mode, U, lam, normT2)
    want = set(int(s) for s in record_factors)
    for t in range(1, sweeps + 1):
        H = M = None
        for n in range(N):
            M = unf[n] @ cp.krp_excluding(U, n)
            H = cp.hadamard_of_grams(G, n)
            Un, fb = cp.solve_normal(M, H)
            res.fallbacks += int(fb)
            U[n], lam = cp.normalise_columns(Un)
            G[n] = cp.gram(U[n])
        e = cp.error_fast(normT2, H, G[N - 1], U[N - 1], M, lam)
        fit = 1.0 - np.sqrt(max(e, 0.0)) / np.sqrt(normT2)
        res.e_hist.append(e)
        res.fit_hist.append(fit)
        res.lam_hist.append(lam.copy())
        if t in want:
            res.U_hist[t] = [u.copy() for u in U]
        res.iters = t
        res.H_last, res.M_last = H, M
        if tol > 0.0 and t >= 2 and abs(res.fit_hist[-1] - res.fit_hist[-2]) < tol:
            res.converged = True
            break
    res.U, res.lam = U, lam
    return res


def model_offsets(ranks: Sequence[int]) -> np.ndarray:
    ranks = np.asarray(ranks, dtype=np.int64)
    off = np.zeros(len(ranks), dtype=np.int64)
    off[1:] = np.cumsum(ranks[:-1])
    return off


def jk_als(T: np.ndarray, sampled_mode: int, ranks: Sequence[int],
           left_out: Sequence[int], init: Sequence[np.ndarray], sweeps: int,
           tol: float = 0.0, models: Optional[Sequence[int]] = None,
           record_factors: Sequence[int] = ()) -> Dict[int, ModelResult]:
    """Jackknife by independent submodel fits (the fitting loop of Alg. 2).

    Model k takes columns [off_k, off_k + ranks[k]) of every initial
    multi-factor ``init[n]`` (I_n x C), deletes row(s) left_out[k] of the
    sampled mode's block and the same slice(s) of T, and runs ``cp_als``.
    left_out[k] is one index (or -1) for leave-one-out, or a list of d
    indices for delete-d jackknife (Sec. 4.1, closing remark).
    ``models`` restricts the run to a subset (the results of the others are
    unaffected, since submodels never interact).
    """
    off = model_offsets(ranks)
    todo = range(len(ranks)) if models is None else models
    out = {}
    for k in todo:
        k = int(k)
        p = left_out[k]
        p = int(p) if np.ndim(p) == 0 else tuple(int(x) for x in p)
        cols = slice(int(off[k]), int(off[k] + ranks[k]))
        U0 = [np.array(init[n][:, cols], dtype=np.float64) for n in range(len(init))]
        U0[sampled_mode] = reduce_init(U0[sampled_mode], p)
        Tk = reduce_tensor(T, sampled_mode, p)
        out[k] = cp_als(Tk, U0, sweeps, tol, record_factors, sampled_mode, p)
    return out


# ---------------------------------------------------------------------------
# CP least-squares loss and its gradient (all-at-once CP, cited in Sec. 2).
# ---------------------------------------------------------------------------

def loss(T: np.ndarray, U: Sequence[np.ndarray]) -> float:
    """f = 1/2 ||T - [[U]]||_F^2, the model formed densely."""
    return 0.5 * cp.residual_explicit(T, U)


def grad(T: np.ndarray, U: Sequence[np.ndarray]) -> List[np.ndarray]:
    """df/dU_n = U_n H_n - M_n with H_n = *_{m != n} U_m^T U_m and M_n the
    MTTKRP of T at the same factors, for every mode n."""
    G = [u.T @ u for u in U]
    out = []
    for n in range(len(U)):
        H = cp.hadamard_of_grams(G, n)
        out.append(U[n] @ H - cp.mttkrp(T, U, n))
    return out


def loss_and_grad(T: np.ndarray, U: Sequence[np.ndarray]):
    return loss(T, U), grad(T, U)


def fd_grad(T: np.ndarray, U: Sequence[np.ndarray], h: float = 1e-3,
            entries: Optional[Sequence[tuple]] = None) -> Dict[tuple, float]:
    """Central differences (f(U + h e) - f(U - h e)) / (2 h) of ``loss`` for
    the listed (mode, row, col) entries (all entries when None)."""
    U = [np.array(u, dtype=np.float64) for u in U]
    if entries is None:
        entries = [(n, i, r) for n, u in enumerate(U)
                   for i in range(u.shape[0]) for r in range(u.shape[1])]
    out = {}
    for (n, i, r) in entries:
        keep = U[n][i, r]
        U[n][i, r] = keep + h
        fp = loss(T, U)
        U[n][i, r] = keep - h
        fm = loss(T, U)
        U[n][i, r] = keep
        out[(n, i, r)] = (fp - fm) / (2.0 * h)
    return out


def gd_refine(T: np.ndarray, U0: Sequence[np.ndarray], steps: int) -> List[np.ndarray]:
    """Gradient refinement of one submodel (reading; not in the paper, which
    only cites gradient-based all-at-once CP in Sec. 2):
    U_n <- U_n - eta * df/dU_n for all modes at once, with the step
    eta = 1 / sum_n ||H_n||_F fixed from the factors at step 0.  Pinned
    against central differences of the dense loss and an explicitly formed
    Khatri-Rao Gram (one step, three steps with the frozen step size, the
    fixed point at an exact decomposition)."""
    U = [np.array(u, dtype=np.float64) for u in U0]
    G = [u.T @ u for u in U]
    eta = 1.0 / sum(np.linalg.norm(cp.hadamard_of_grams(G, n)) for n in range(len(U)))
    for _ in range(steps):
        g = grad(T, U)
        U = [u - eta * gn for u, gn in zip(U, g)]
    return U


# ---------------------------------------------------------------------------
# Flop counts of Sec. 4.2.
# ---------------------------------------------------------------------------

def flops_jk_als(dims: Sequence[int], sampled_mode: int, R: int, d: int = 1) -> float:
    """MTTKRP flops of one mode summed over all I/d submodels of JK-ALS:
    (I/d) * 2 R (I - d) * prod_{i != n-hat} I_i."""
    I = dims[sampled_mode]
    rest = float(np.prod([x for m, x in enumerate(dims) if m != sampled_mode]))
    return (I / d) * (2.0 * R * (I - d) * rest)


def flops_jk_cals(dims: Sequence[int], sampled_mode: int, R: int, d: int = 1) -> float:
    """Flops of the one fused MTTKRP of JK-CALS: 2 (I/d) R prod_i I_i."""
    I = dims[sampled_mode]
    return 2.0 * (I / d) * R * float(np.prod(dims))


def flop_ratio(I: int, d: int = 1) -> float:
    """JK-CALS over JK-ALS flops: I / (I - d), at most 2 for d <= I/2."""
    return I / (I - d)
