"""CP-ALS building blocks in plain float64 numpy (test infrastructure only).

Every function follows one passage of the paper; no blocking, fusion or
reordering beyond what that passage states.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence, Tuple

import numpy as np
import scipy.linalg

EPS = np.finfo(np.float64).eps


def unfold(T: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding T_(n) (Sec. 3.1 notation; index map Eq. (3)).

    Element T(i_1, ..., i_N) lands in row i_n and column
    j = sum_{k != n} i_k * prod_{m < k, m != n} I_m (0-based), i.e. the
    remaining modes are laid out with the lowest mode varying fastest.
    """
    T = np.asarray(T, dtype=np.float64)
    return np.reshape(np.moveaxis(T, n, 0), (T.shape[n], -1), order="F")


def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Column-wise Kronecker product A (.) B (.) ... of the listed matrices
    (Sec. 3.1).  In column r the row index of the last-listed matrix varies
    fastest, as for kron(a, b)."""
    out = np.asarray(mats[0], dtype=np.float64)
    R = out.shape[1]
    for B in mats[1:]:
        B = np.asarray(B, dtype=np.float64)
        out = (out[:, None, :] * B[None, :, :]).reshape(-1, R)
    return out


def krp_excluding(U: Sequence[np.ndarray], n: int) -> np.ndarray:
    """U_N (.) ... (.) U_{n+1} (.) U_{n-1} (.) ... (.) U_1, the order of Eq. (1)."""
    order = [U[m] for m in reversed(range(len(U))) if m != n]
    return khatri_rao(order)


def mttkrp(T: np.ndarray, U: Sequence[np.ndarray], n: int) -> np.ndarray:
    """M_n = T_(n) (U_N (.) ... (.) U_{n+1} (.) U_{n-1} (.) ... (.) U_1)
    (Alg. 1 MTTKRP step; Eq. (1)).  Pinned by brute force in the tests."""
    return unfold(T, n) @ krp_excluding(U, n)


def mttkrp_bruteforce(T: np.ndarray, U: Sequence[np.ndarray], n: int) -> np.ndarray:
    """The defining sum M_n(i_n, r) = sum_i T(i) prod_{m != n} U_m(i_m, r),
    in pure-Python loops.  Only for tiny tensors."""
    T = np.asarray(T, dtype=np.float64)
    R = U[0].shape[1]
    M = np.zeros((T.shape[n], R))
    for idx in itertools.product(*[range(s) for s in T.shape]):
        t = float(T[idx])
        for r in range(R):
            prod = t
            for m, im in enumerate(idx):
                if m != n:
                    prod *= float(U[m][im, r])
            M[idx[n], r] += prod
    return M


def gram(U: np.ndarray) -> np.ndarray:
    """U^T U with the upper triangle mirrored, so G is exactly symmetric."""
    G = np.asarray(U, dtype=np.float64).T @ np.asarray(U, dtype=np.float64)
    upper = np.triu(G)
    return upper + np.triu(G, 1).T


def hadamard_of_grams(G: Sequence[np.ndarray], n: int) -> np.ndarray:
    """H_n = *_{i != n} U_i^T U_i (Alg. 1 Hadamard step)."""
    H = None
    for i, Gi in enumerate(G):
        if i == n:
            continue
        H = Gi.copy() if H is None else H * Gi
    return H


PIVOT_TOL = 64.0 * EPS     # times R: relative pivot / eigenvalue cutoff


def solve_normal(M: np.ndarray, H: np.ndarray) -> Tuple[np.ndarray, bool]:
    """U = M H^+ (Alg. 1 update step; normal equations of Sec. 3.2).

    Reading of the pseudoinverse: when H is numerically positive definite
    the product is formed through the Cholesky factorisation H = L L^T and
    two triangular solves.  H counts as positive definite when every pivot
    L_jj^2 exceeds tau * max_j H_jj with tau = 64 R eps, and everything is
    finite.  Otherwise the eigen-decomposition pseudoinverse is used, with
    eigenvalues at or below tau * lambda_max(H) treated as zero.  Returns
    (U, used_fallback).
    """
    R = H.shape[0]
    tau = PIVOT_TOL * R
    scale = float(np.max(np.diag(H))) if R else 0.0
    if np.all(np.isfinite(H)) and np.all(np.isfinite(M)) and scale > 0.0:
        try:
            L = scipy.linalg.cholesky(H, lower=True)
            if float(np.min(np.diag(L))) ** 2 > tau * scale:
                Y = scipy.linalg.solve_triangular(L, M.T, lower=True)
                X = scipy.linalg.solve_triangular(L.T, Y, lower=False)
                if np.all(np.isfinite(X)):
                    return X.T, False
        except np.linalg.LinAlgError:
            pass
    if not np.all(np.isfinite(H)):
        return np.full_like(M, np.nan), True
    w, V = np.linalg.eigh(H)
    cutoff = tau * max(float(np.max(w)), 0.0)
    winv = np.array([1.0 / x if x > cutoff else 0.0 for x in w])
    Hpinv = (V * winv[None, :]) @ V.T
    return M @ Hpinv, True


def normalise_columns(U: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """lambda_r = ||U(:, r)||_2 and U(:, r) / lambda_r where lambda_r > 0.
    Not in the paper (standard CP-ALS practice); it leaves the fitted model
    unchanged because the next mode update absorbs the scale."""
    lam = np.sqrt(np.sum(U * U, axis=0))
    V = U.copy()
    for r in range(U.shape[1]):
        if lam[r] > 0.0:
            V[:, r] = U[:, r] / lam[r]
    return V, lam


def error_fast(normT2: float, H_last: np.ndarray, G_last: np.ndarray,
               U_last: np.ndarray, M_last: np.ndarray, lam: np.ndarray) -> float:
    """Squared error ||T - [[lambda; U]]||^2 from the last mode's quantities
    (Alg. 1 error step, Alg. 3 error step).

    Reading: ||T||^2 + ||[[lambda; U]]||^2 - 2 <T, [[lambda; U]]>, with
    ||[[lambda; U]]||^2 = lambda^T (H_N * G_N) lambda and
    <T, [[lambda; U]]> = sum_r lambda_r sum_i U_N(i, r) M_N(i, r).  The
    printed minus sign in front of the second term is read as a plus.
    """
    quad = float(lam @ ((H_last * G_last) @ lam))
    inner = float(np.sum(lam[None, :] * U_last * M_last))
    return normT2 + quad - 2.0 * inner


def reconstruct(U: Sequence[np.ndarray], lam: np.ndarray | None = None) -> np.ndarray:
    """Dense [[lambda; U_1, ..., U_N]], built element by element from the
    definition (sum of R scaled rank-one outer products)."""
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    shape = tuple(u.shape[0] for u in U)
    out = np.zeros(shape)
    for r in range(R):
        term = np.asarray(lam[r], dtype=np.float64)
        for u in U:
            term = np.multiply.outer(term, u[:, r])
        out += term
    return out


def residual_explicit(T: np.ndarray, U: Sequence[np.ndarray],
                      lam: np.ndarray | None = None) -> float:
    """||T - [[lambda; U]]||_F^2 with the model formed densely."""
    D = np.asarray(T, dtype=np.float64) - reconstruct(U, lam)
    return float(np.sum(D * D))
