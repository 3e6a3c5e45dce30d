"""Jackknife post-processing of fitted submodels (test infrastructure only).

Alg. 2 ends with two steps the paper leaves to its citation on jackknife of
multi-way models: every fitted submodel is brought into the component order
and scaling of the overall model P (the permutation and scale adjustment),
and then the standard deviation of every factor matrix except the sampled
mode's is taken over the set of submodels.  Readings (flagged, repeated in
the design notes):

* matching: the congruence of submodel component r with reference component
  s is the product over the non-sampled modes of the cosine between their
  loading vectors (Tucker's congruence coefficient); the assignment maximises
  the sum of the absolute congruences of matched pairs over all permutations
  (an assignment problem, solved exactly);
* scale adjustment: every loading vector of a non-sampled mode is scaled to
  unit 2-norm and its sign chosen so that its inner product with the matched
  reference vector is not negative; the sampled mode (whose rows differ
  between submodels) absorbs the scales and signs and is not reported;
* standard deviation: the jackknife formula
  S = sqrt((K-1)/K * sum_k (theta_k - theta_bar)^2) over the K submodels of
  the set, theta_bar their mean, element by element.

Parity status: ``match_components`` is pinned against exhaustive search over
all permutations and against planted permutations; ``jackknife_std`` against
planted copies of the reference (S = 0), against the classical identity that
the jackknife standard error of a sample mean is the sample standard
deviation over sqrt(n), and against the two-submodel closed form |a - b| / 2
(tests/test_oracle_postprocess.py).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np
from scipy.optimize import linear_sum_assignment


def congruence(U: Sequence[np.ndarray], V: Sequence[np.ndarray], modes: Sequence[int]) -> np.ndarray:
    """phi[r, s] = prod over ``modes`` of cos(U_n[:, r], V_n[:, s]), the
    product taken in ascending mode order.  A zero vector has cosine 0."""
    R = U[modes[0]].shape[1]
    phi = np.ones((R, V[modes[0]].shape[1]))
    for n in modes:
        a, b = U[n], V[n]
        na = np.sqrt(np.sum(a * a, axis=0))
        nb = np.sqrt(np.sum(b * b, axis=0))
        d = a.T @ b
        den = np.outer(na, nb)
        phi = phi * np.where(den > 0, d / np.where(den > 0, den, 1.0), 0.0)
    return phi


def match_components(U: Sequence[np.ndarray], V: Sequence[np.ndarray],
                     sampled_mode: int) -> Tuple[np.ndarray, Dict[int, np.ndarray]]:
    """Permutation and signs that bring submodel factors U into the component
    order of the reference V (Alg. 2, permutation and scale adjustment).

    Returns perm with perm[s] = the component of U matched to reference
    component s, and for every non-sampled mode n the signs sign[n][s] in
    {+1, -1} of U_n[:, perm[s]] against V_n[:, s] (+1 for a zero product)."""
    N = len(U)
    modes = [n for n in range(N) if n != sampled_mode]
    phi = congruence(U, V, modes)
    rows, cols = linear_sum_assignment(-np.abs(phi))
    perm = np.empty(phi.shape[1], dtype=np.int64)
    perm[cols] = rows
    signs = {}
    for n in modes:
        d = np.sum(U[n][:, perm] * V[n], axis=0)
        signs[n] = np.where(d < 0, -1.0, 1.0)
    return perm, signs


def aligned_factors(U: Sequence[np.ndarray], V: Sequence[np.ndarray],
                    sampled_mode: int) -> Dict[int, np.ndarray]:
    """The non-sampled factors of U in the reference's component order, each
    column scaled to unit 2-norm with the matched sign (scale adjustment)."""
    perm, signs = match_components(U, V, sampled_mode)
    out = {}
    for n, sg in signs.items():
        A = U[n][:, perm]
        nrm = np.sqrt(np.sum(A * A, axis=0))
        out[n] = A * np.where(nrm > 0, sg / np.where(nrm > 0, nrm, 1.0), 0.0)
    return out


def jackknife_std(subs: Sequence[Sequence[np.ndarray]], ref: Sequence[np.ndarray],
                  sampled_mode: int) -> Dict[int, np.ndarray]:
    """S_n for every mode n except the sampled one (Alg. 2, standard deviation
    step): the jackknife standard deviation, element by element, of the
    aligned factors of the K submodels in ``subs``."""
    K = len(subs)
    al = [aligned_factors(U, ref, sampled_mode) for U in subs]
    S = {}
    for n in al[0]:
        th = np.stack([a[n] for a in al])          # K x I_n x R
        mean = th.sum(axis=0) / K
        S[n] = np.sqrt((K - 1) / K * np.sum((th - mean) ** 2, axis=0))
    return S
