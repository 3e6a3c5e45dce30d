"""Delete-d jackknife on the GPU (Sec. 4.1, closing remark: d zero rows per
submodel instead of one) against the oracle's independent fits on the
explicitly reduced tensors: the fused MTTKRP per model (1e-12), every
iteration of the sweeps (1e-11), the loss and gradient, and the benchmark
tensor with groups of 4 samples at full size."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import make_ctx, oracle_model_mttkrp, rel, say, to_np, cols

pytestmark = pytest.mark.gpu

SPECS = [
    # (seed, dims, ranks, left_out [K, d], sampled_mode)
    (51, (17, 13, 11), [3, 2, 4], [[-1, -1], [0, 16], [5, 6]], 0),
    (52, (9, 12, 7, 6), [2, 3], [[8, 0, 4], [1, 2, 3]], 0),
    (53, (15, 24, 10), [3, 3, 5], [[4, 9, 20, 23], [-1, -1, -1, -1], [0, 1, 2, 3]], 1),
    (54, (40, 33), [2, 3], [[39, 38], [7, 1]], 0),
]


def _wl(spec, noise=0.1):
    seed, dims, ranks, lo, nh = spec
    return synth.random_problem(seed, dims, ranks, lo, noise=noise, sampled_mode=nh)


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_fused_mttkrp_matches_per_model(spec):
    wl = _wl(spec)
    say("delete-d mttkrp", spec[0])
    ctx = make_ctx(wl)
    for n in range(len(wl.dims)):
        M = to_np(ctx.mttkrp(n))
        for k in range(wl.K):
            e = rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
            assert e <= 1e-12, (n, k, e)


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_sweeps_match_oracle(spec):
    wl = _wl(spec)
    sweeps = 4
    say("delete-d sweeps", spec[0])
    res = oracle.jk_als(np.asarray(wl.T), wl.sampled_mode, wl.ranks, wl.left_out, wl.init,
                        sweeps, record_factors=range(1, sweeps + 1))
    ctx = make_ctx(wl)
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        err, fit = (to_np(x) for x in ctx.get_status()[:2])
        lam = to_np(ctx.get_factors(0)[1])
        facs = [to_np(ctx.get_factors(n)[0]) for n in range(len(wl.dims))]
        for k, r in res.items():
            c = cols(wl, k)
            ref = r.padded(r.U_hist[t])
            for n in range(len(wl.dims)):
                assert rel(facs[n][:, c], ref[n]) <= 1e-11, (t, k, n)
            assert rel(lam[c], r.lam_hist[t - 1]) <= 1e-11
            assert abs(err[k] - r.e_hist[t - 1]) <= 1e-11 * r.normT2, (t, k)
            assert abs(fit[k] - r.fit_hist[t - 1]) <= 1e-9


def test_loss_and_gradient_match_oracle():
    import torch
    wl = _wl(SPECS[0], noise=0.2)
    ctx = make_ctx(wl)
    facs = [torch.from_numpy(u).cuda().requires_grad_() for u in wl.init]
    loss = jk.JKCPLoss.apply(ctx, *facs)
    grads = torch.autograd.grad(loss.sum(), facs)
    L = to_np(loss)
    G = [to_np(g) for g in grads]
    for k in range(wl.K):
        c = cols(wl, k)
        p = wl.left_out[k]
        U = [np.array(u[:, c]) for u in wl.init]
        U[0] = oracle.reduce_init(U[0], p)
        Tk = oracle.reduce_tensor(np.asarray(wl.T), 0, p)
        f, g = oracle.loss_and_grad(Tk, U)
        assert abs(L[k] - f) <= 1e-11 * max(1.0, 0.5 * np.sum(Tk ** 2)), k
        rows = oracle.left_out_rows(p)
        full = np.zeros((wl.dims[0], len(U[0][0])))
        full[np.setdiff1d(np.arange(wl.dims[0]), rows)] = g[0]
        assert rel(G[0][:, c], full) <= 1e-11, k
        for n in (1, 2):
            assert rel(G[n][:, c], g[n]) <= 1e-11, (k, n)


def test_benchmark_tensor_in_groups_of_four():
    """The benchmark tensor (100x200x200, rank 5) jackknifed in 25 groups of
    4 consecutive samples; sampled models checked per iteration."""
    wl = synth.config2(delete_d=4)
    models = [0, 12, 24]
    say("c2 delete-4")
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 5,
                        models=models, record_factors=range(1, 6))
    ctx = make_ctx(wl)
    for t in range(1, 6):
        ctx.sweep(1)
        facs = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
        err = to_np(ctx.get_status()[0])
        for k in models:
            r = res[k]
            ref = r.padded(r.U_hist[t])
            for n in range(3):
                assert rel(facs[n][:, cols(wl, k)], ref[n]) <= 1e-11, (t, k, n)
            assert abs(err[k] - r.e_hist[t - 1]) <= 1e-11 * r.normT2


def test_fit_with_compaction_and_post_processing():
    """Delete-d submodels of uneven convergence fitted with a tolerance:
    compaction on and off give the same bits, and the jackknife deviations
    of the delete-2 set match the oracle's on the oracle's own fits."""
    rng_dims, R = (24, 15, 12), 3
    groups = [[-1, -1]] + [[2 * g, 2 * g + 1] for g in range(12)]
    wl = synth.random_problem(55, rng_dims, [R] * len(groups), groups, noise=0.05, true_rank=3)
    say("delete-2 fit + jackknife")
    a = make_ctx(wl)
    b = make_ctx(wl)
    b.set_compaction(False)
    ia, fa, sa = a.fit(200, 1e-8)
    ib, fb, sb = b.fit(200, 1e-8)
    assert np.array_equal(ia, ib) and np.array_equal(sa, sb) and np.array_equal(fa, fb)
    for n in range(3):
        assert np.array_equal(to_np(a.get_factors(n)[0]), to_np(b.get_factors(n)[0]))
    # post-processing of fits after a fixed number of sweeps on both paths
    c = make_ctx(wl)
    c.sweep(30)
    S = c.jackknife_std(0, 1, wl.K - 1)
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 30)
    ref = oracle.jackknife_std([res[k].U for k in range(1, wl.K)], res[0].U, 0)
    for n in (1, 2):
        g, r = to_np(S[n]), ref[n]
        assert np.max(np.abs(g - r)) <= 1e-7 * np.max(np.abs(r)), n
