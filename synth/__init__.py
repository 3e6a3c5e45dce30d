"""Seeded synthetic inputs for the JK-CALS workloads.

This module only draws random numbers and lays them out. It holds none of the
fitting method's arithmetic (no unfolding, no Khatri-Rao product, no MTTKRP, no
Gram, no solve): the oracle and the HIP path both take its outputs as plain
inputs, and neither is imported here.

Layout conventions shared by every consumer:

* a tensor of shape (I_1, ..., I_N) is returned as a numpy array in Fortran
  order, so ``T.ravel(order="F")`` is the column-major, i_1-fastest storage
  of Eq. (3) (element (i_1, ..., i_N) at offset i_1 + I_1*(i_2 + I_2*(...)));
* a model table is two int32 arrays ``ranks[K]`` and ``left_out[K]``
  (``-1`` marks a full model that keeps every sample), or ``left_out[K, d]``
  for delete-d jackknife (row k lists the d samples model k leaves out, a row
  of ``-1`` a full model); model k owns the
  columns ``[off_k, off_k + ranks[k])`` of every multi-factor, with offsets
  taken in model order;
* an initial multi-factor for mode n is an ``I_n x C`` float64 array in C
  order (C contiguous), with C = sum(ranks).  It is *not* pre-zeroed: the
  consumer removes (oracle) or zeroes (GPU path) the left-out rows of the
  sampled mode itself.

Random streams: ``SeedSequence(211203985 + config_index).spawn(3)`` gives the
[factors, noise, init] generators (PCG64), so every draw is reproducible.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 211203985


@dataclasses.dataclass
class Workload:
    """One synthetic jackknife problem."""

    name: str
    T: np.ndarray                 # Fortran-ordered tensor (I_1, ..., I_N)
    sampled_mode: int             # the paper's n-hat, 0-based
    ranks: np.ndarray             # int32 [K]
    left_out: np.ndarray          # int32 [K] or [K, d] (delete-d), -1 = full model
    init: List[np.ndarray]        # per mode, I_n x C float64, C-contiguous
    sweeps: int                   # iteration budget of the configuration
    truth: Optional[List[np.ndarray]] = None   # generating factors (for pins)

    @property
    def dims(self):
        return tuple(int(d) for d in self.T.shape)

    @property
    def C(self):
        return int(np.sum(self.ranks))

    @property
    def K(self):
        return int(len(self.ranks))

    def offsets(self):
        off = np.zeros(len(self.ranks), dtype=np.int64)
        if len(self.ranks) > 1:
            off[1:] = np.cumsum(self.ranks[:-1])
        return off


def streams(config_index: int):
    ss = np.random.SeedSequence(BASE_SEED + int(config_index)).spawn(3)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def dense_from_factors(factors: Sequence[np.ndarray]) -> np.ndarray:
    """Sum of R rank-one outer products, built with einsum, Fortran order."""
    N = len(factors)
    letters = "abcdefgh"[:N]
    if N <= 3:
        spec = ",".join(f"{c}z" for c in letters) + "->" + letters
        out = np.einsum(spec, *factors, optimize=True)
    else:
        # pairwise outer products keep the intermediate small for 4-way data
        R = factors[0].shape[1]
        left = np.einsum("az,bz->abz", factors[0], factors[1]).reshape(-1, R)
        right = np.einsum("cz,dz->cdz", factors[2], factors[3]).reshape(-1, R)
        out = (left @ right.T).reshape([f.shape[0] for f in factors])
    return np.asfortranarray(out)


def add_noise(T0: np.ndarray, rng: np.random.Generator, level: float) -> np.ndarray:
    """T0 + E with E ~ N(0,1) rescaled so that ||E||_F = level * ||T0||_F."""
    if level <= 0.0:
        return np.asfortranarray(T0)
    E = rng.standard_normal(T0.shape)
    E *= level * np.linalg.norm(T0.ravel()) / np.linalg.norm(E.ravel())
    return np.asfortranarray(T0 + E)


def loo_table(I: int, R: int, include_full: bool = False):
    """Leave-one-out models over I samples, all of rank R (full model first)."""
    lo = list(range(I))
    if include_full:
        lo = [-1] + lo
    ranks = np.full(len(lo), R, dtype=np.int32)
    return ranks, np.asarray(lo, dtype=np.int32)


def delete_d_table(I: int, d: int, R: int, include_full: bool = False):
    """Delete-d jackknife over I samples in groups of d consecutive samples
    (the last group smaller when d does not divide I is dropped), all models
    of rank R: left_out is [K, d] (full model first, as a row of -1)."""
    groups = [list(range(g * d, g * d + d)) for g in range(I // d)]
    if include_full:
        groups = [[-1] * d] + groups
    ranks = np.full(len(groups), R, dtype=np.int32)
    return ranks, np.asarray(groups, dtype=np.int32).reshape(len(groups), d)


def shared_parent_init(rng: np.random.Generator, dims, parents_R: Sequence[int],
                       children: Sequence[int]):
    """One N(0,1) parent init per entry of ``parents_R``; parent q is repeated
    ``children[q]`` times, side by side, to form each mode's multi-factor."""
    parents = [[rng.standard_normal((I, R)) for I in dims] for R in parents_R]
    init = []
    for n, _ in enumerate(dims):
        blocks = []
        for q, par in enumerate(parents):
            blocks.extend([par[n]] * int(children[q]))
        init.append(np.ascontiguousarray(np.concatenate(blocks, axis=1)))
    return init


def gaussian_peaks(rng: np.random.Generator, I: int, R: int) -> np.ndarray:
    """Columns exp(-(i-mu)^2 / (2 sigma^2)) with mu ~ U(0.1 I, 0.9 I) and
    FWHM ~ U(10, 30) bins, sigma = FWHM / (2 sqrt(2 ln 2))."""
    i = np.arange(I, dtype=np.float64)[:, None]
    mu = rng.uniform(0.1 * I, 0.9 * I, size=R)[None, :]
    fwhm = rng.uniform(10.0, 30.0, size=R)[None, :]
    sigma = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    return np.exp(-((i - mu) ** 2) / (2.0 * sigma ** 2))


# ---------------------------------------------------------------------------
# The five workloads.  ``scale`` < 1 shrinks a workload's sizes for fast
# tests while keeping its structure; ``scale=1`` is the full configuration.
# ---------------------------------------------------------------------------

def config1() -> Workload:
    """20x30x40, rank-3 N(0,1) factors, 1 % noise; 20 LOO + the full model,
    rank 3 each, from one shared N(0,1) parent init; 50 sweeps."""
    rf, rn, ri = streams(1)
    dims = (20, 30, 40)
    A = [rf.standard_normal((I, 3)) for I in dims]
    T = add_noise(dense_from_factors(A), rn, 0.01)
    ranks, lo = loo_table(dims[0], 3, include_full=True)
    init = shared_parent_init(ri, dims, [3], [len(ranks)])
    return Workload("c1_20x30x40_r3_loo+full", T, 0, ranks, lo, init, 50, A)


def config2(dims=(100, 200, 200), models: Optional[int] = None, delete_d: int = 1) -> Workload:
    """Fluorescence-like 3-way tensor: mode 1 concentrations U(0,1), modes 2
    and 3 Gaussian-peak spectra; rank 5, 2 % noise; leave-one-out over all
    mode-1 samples at rank 5 from a shared N(0,1) parent init; 100 sweeps.
    delete_d > 1: delete-d jackknife over groups of d consecutive samples
    instead (I / d submodels), the same tensor and init."""
    rf, rn, ri = streams(2)
    R0 = 5
    A = [rf.uniform(0.0, 1.0, size=(dims[0], R0))]
    A += [gaussian_peaks(rf, I, R0) for I in dims[1:]]
    T = add_noise(dense_from_factors(A), rn, 0.02)
    ranks, lo = loo_table(dims[0], 5) if delete_d <= 1 else delete_d_table(dims[0], delete_d, 5)
    if models is not None:
        ranks, lo = ranks[:models], lo[:models]
    init = shared_parent_init(ri, dims, [5], [len(ranks)])
    name = "c2_%dx%dx%d_r5_%s" % (tuple(dims) + ("loo" if delete_d <= 1 else "delete%d" % delete_d,))
    return Workload(name, T, 0, ranks, lo, init, 100, A)


def config3(dims=(300, 250, 200), rank_max: int = 10, inits_per_rank: int = 5,
            samples: Optional[Sequence[int]] = None) -> Workload:
    """Random rank-8 noise-free 3-way tensor; for every R in 1..rank_max,
    ``inits_per_rank`` N(0,1) parent inits, each jackknifed over the mode-1
    samples (all of them unless ``samples`` lists a subset); 100 sweeps."""
    rf, rn, ri = streams(3)
    A = [rf.standard_normal((I, 8)) for I in dims]
    T = dense_from_factors(A)
    lo_rows = list(range(dims[0])) if samples is None else [int(s) for s in samples]
    parents_R, ranks, lo = [], [], []
    for R in range(1, rank_max + 1):
        for _ in range(inits_per_rank):
            parents_R.append(R)
            ranks.extend([R] * len(lo_rows))
            lo.extend(lo_rows)
    init = shared_parent_init(ri, dims, parents_R, [len(lo_rows)] * len(parents_R))
    return Workload("c3_%dx%dx%d_r1-10_x%d_loo" % (tuple(dims) + (inits_per_rank,)), T, 0,
                    np.asarray(ranks, np.int32), np.asarray(lo, np.int32), init, 100, A)


def config4(dims=(200, 120, 100, 80), models: Optional[int] = None) -> Workload:
    """4-way random rank-12 tensor with 1 % noise; leave-one-out over mode 1
    at rank 12 from a shared N(0,1) parent init; 100 sweeps (split-BF16)."""
    rf, rn, ri = streams(4)
    A = [rf.standard_normal((I, 12)) for I in dims]
    T = add_noise(dense_from_factors(A), rn, 0.01)
    ranks, lo = loo_table(dims[0], 12)
    if models is not None:
        ranks, lo = ranks[:models], lo[:models]
    init = shared_parent_init(ri, dims, [12], [len(ranks)])
    return Workload("c4_%dx%dx%dx%d_r12_loo" % tuple(dims), T, 0, ranks, lo, init, 100, A)


def config5(dims=(100, 150, 150), models: Optional[int] = None) -> Workload:
    """Random rank-10 noise-free 3-way tensor generated in float64 and
    stored as float32; leave-one-out at rank 10; 20 ALS sweeps followed by
    200 gradient steps."""
    rf, rn, ri = streams(5)
    A = [rf.standard_normal((I, 10)) for I in dims]
    T = np.asfortranarray(dense_from_factors(A).astype(np.float32))
    ranks, lo = loo_table(dims[0], 10)
    if models is not None:
        ranks, lo = ranks[:models], lo[:models]
    init = shared_parent_init(ri, dims, [10], [len(ranks)])
    return Workload("c5_%dx%dx%d_r10_loo_f32" % tuple(dims), T, 0, ranks, lo, init, 20, A)


def random_problem(seed: int, dims, ranks, left_out, noise: float = 0.0,
                   true_rank: int = 3, sampled_mode: int = 0,
                   dtype=np.float64) -> Workload:
    """Small generic problem for tests: N(0,1) factors of ``true_rank``,
    optional noise, and an independent N(0,1) init for every model."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + 1000 + seed)))
    A = [rng.standard_normal((I, true_rank)) for I in dims]
    T = add_noise(dense_from_factors(A), rng, noise)
    if dtype != np.float64:
        T = np.asfortranarray(T.astype(dtype))
    ranks = np.asarray(ranks, np.int32)
    lo = np.asarray(left_out, np.int32)
    C = int(ranks.sum())
    init = [np.ascontiguousarray(rng.standard_normal((I, C))) for I in dims]
    return Workload("random_%d" % seed, T, sampled_mode, ranks, lo, init, 10, A)
