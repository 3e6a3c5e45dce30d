"""Jackknife post-processing on the GPU (Alg. 2, permutation and scale
adjustment and the standard deviation of the factors) against the oracle:
matched components and signs exactly, standard deviations to 1e-10
(relative to the largest) on planted sets, and end to end after fitting the
20-submodel workload with both paths."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import make_ctx, say, to_np

pytestmark = pytest.mark.gpu


def _planted(seed, dims, R, count, noise, nh=0):
    """Reference factors V and `count` submodels: V with permuted columns,
    random signs and scales per mode, plus noise; as a context with the
    reference as model 0 (left_out -1) and the submodels after it."""
    rng = np.random.default_rng(7000 + seed)
    V = [rng.standard_normal((I, R)) for I in dims]
    subs, perms = [], []
    for k in range(count):
        perm = rng.permutation(R)
        U = []
        for n, v in enumerate(V):
            u = np.empty_like(v)
            u[:, perm] = v * rng.choice([-1.0, 1.0], size=R) * rng.uniform(0.3, 3.0, size=R)
            u += noise * rng.standard_normal(u.shape)
            U.append(u)
        U[nh][k % dims[nh], :] = 0.0          # row p of the sampled mode is 0 in the context
        subs.append(U)
        perms.append(perm)
    ranks = [R] * (count + 1)
    left = [-1] + [k % dims[nh] for k in range(count)]
    return V, subs, ranks, left


def _context(dims, nh, ranks, left, V, subs):
    import torch
    init = [np.concatenate([V[n]] + [U[n] for U in subs], axis=1) for n in range(len(dims))]
    wl = synth.Workload("planted", np.zeros(dims, order="F"), nh, np.asarray(ranks, np.int32),
                        np.asarray(left, np.int32), init, 1, None)
    ctx = make_ctx(wl)
    for n in range(len(dims)):
        ctx.set_factors(n, torch.from_numpy(np.ascontiguousarray(init[n])).cuda())
    return ctx


def _compare(S_gpu, S_ref, tol=1e-10):
    assert set(S_gpu) == set(S_ref)
    for n in S_ref:
        g, r = to_np(S_gpu[n]), S_ref[n]
        scale = max(np.max(np.abs(r)), 1e-300)
        assert np.max(np.abs(g - r)) <= tol * scale, (n, np.max(np.abs(g - r)), scale)


@pytest.mark.parametrize("seed,dims,R,count,nh", [
    (1, (12, 15, 11), 4, 9, 0),
    (2, (9, 14, 10, 7), 3, 6, 1),
    (3, (40, 33, 29), 32, 5, 0),       # the largest rank
    (4, (17, 8), 5, 7, 1),
    (7, (100, 200, 200), 5, 99, 0),  # the benchmark shape: 99 submodels of rank 5
])
def test_planted_sets_match_oracle(seed, dims, R, count, nh):
    V, subs, ranks, left = _planted(seed, dims, R, count, 0.05, nh)
    say("jackknife planted", seed, dims, R, count)
    ctx = _context(dims, nh, ranks, left, V, subs)
    S, perm, sign = ctx.jackknife_std(0, 1, count, with_matching=True)
    perm, sign = to_np(perm), to_np(sign)
    for k, U in enumerate(subs):
        p, sg = oracle.match_components(U, V, nh)
        assert np.array_equal(perm[k], p), (k, perm[k], p)
        for n, s in sg.items():
            assert np.array_equal(sign[n, k], s), (k, n)
    _compare(S, oracle.jackknife_std(subs, V, nh))


def test_single_submodel_and_copies_give_zero():
    V, subs, ranks, left = _planted(5, (10, 12, 9), 3, 4, 0.0)
    ctx = _context((10, 12, 9), 0, ranks, left, V, subs)
    S = ctx.jackknife_std(0, 1, 4)
    for n in (1, 2):
        assert np.max(np.abs(to_np(S[n]))) < 1e-14
    S1 = ctx.jackknife_std(0, 2, 1)
    for n in (1, 2):
        assert np.all(to_np(S1[n]) == 0.0)


def test_invalid_sets_are_refused():
    V, subs, ranks, left = _planted(6, (8, 7, 6), 2, 3, 0.1)
    ranks[3] = 2
    ctx = _context((8, 7, 6), 0, ranks, left, V, subs)
    with pytest.raises(jk.JkcError):
        ctx.jackknife_std(0, 1, 4)       # past the last model
    with pytest.raises(jk.JkcError):
        ctx.jackknife_std(0, 0, 0)       # empty set


def test_rank_mismatch_is_refused():
    import torch
    rng = np.random.default_rng(11)
    dims = (6, 5, 4)
    ranks, left = [2, 3, 2], [-1, 0, 1]
    init = [rng.standard_normal((I, 7)) for I in dims]
    wl = synth.Workload("mix", np.zeros(dims, order="F"), 0, np.asarray(ranks, np.int32),
                        np.asarray(left, np.int32), init, 1, None)
    ctx = make_ctx(wl)
    with pytest.raises(jk.JkcError, match="rank"):
        ctx.jackknife_std(0, 1, 2)


def test_end_to_end_after_fitting_the_20_submodel_workload():
    """Config 1 (20x30x40, 1 % noise, 20 leave-one-out submodels + the full
    model as model 0): both paths fit 50 sweeps, then post-process."""
    wl = synth.config1()
    say("c1 jackknife end to end")
    ctx = make_ctx(wl)
    ctx.sweep(wl.sweeps)
    S = ctx.jackknife_std(0, 1, wl.K - 1)
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, wl.sweeps)
    ref = res[0].U
    subs = [res[k].U for k in range(1, wl.K)]
    # the fits agree to ~1e-11; the deviations are differences of nearby
    # values, so the comparison is relative to their size
    _compare(S, oracle.jackknife_std(subs, ref, 0), tol=1e-7)
