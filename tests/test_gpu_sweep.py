"""Parity of the JK-CALS sweep (Alg. 3) with the oracle's independent
per-submodel ALS on the explicitly reduced tensors (Alg. 2 fitting loop
around Alg. 1), per iteration: factors (zero row re-inserted), lambda,
error and fit, at 1e-11 relative for the float64 path."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import make_ctx, rel, say, to_np, cols, shipped_tilings, apply_tilings

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _compare_iteration(wl, ctx, res, t, models=None, tol=TOL, fit_from_err=False):
    """Compare GPU state after sweep t with the oracle record of sweep t.
    fit_from_err: the fit is 1 - sqrt(e / ||T||^2) of the error e, so it is
    also accepted within sqrt(|e_gpu - e_ref| / ||T||^2), the exact bound
    |sqrt(a) - sqrt(b)| <= sqrt(|a - b|) applied to the error's agreement
    (the binding term only where a model fits its tensor exactly and e is a
    cancellation at rounding level)."""
    err, fit, st, it = (to_np(x) for x in ctx.get_status())
    facs = [to_np(ctx.get_factors(n)[0]) for n in range(len(wl.dims))]
    lam = to_np(ctx.get_factors(0)[1])
    worst = 0.0
    for k in (models if models is not None else res.keys()):
        r = res[k]
        c = cols(wl, k)
        U_ref = r.padded(r.U_hist[t])
        for n in range(len(wl.dims)):
            e = rel(facs[n][:, c], U_ref[n])
            worst = max(worst, e)
            assert e <= tol, ("U", t, k, n, e)
        e = rel(lam[c], r.lam_hist[t - 1])
        assert e <= tol, ("lambda", t, k, e)
        assert abs(err[k] - r.e_hist[t - 1]) <= tol * r.normT2, ("err", t, k)
        ftol = 1e-9
        if fit_from_err:
            ftol = max(ftol, float(np.sqrt(abs(err[k] - r.e_hist[t - 1]) / r.normT2)) + 1e-15)
        assert abs(fit[k] - r.fit_hist[t - 1]) <= ftol, ("fit", t, k)
        worst = max(worst, e)
    return worst


@pytest.mark.parametrize("seed,dims,ranks,lo,nh", [
    (21, (17, 13, 11), [3, 2, 4], [-1, 0, 16], 0),
    (22, (9, 12, 7, 6), [2, 3], [8, -1], 0),
    (23, (15, 24, 10), [3, 3, 5], [4, -1, 23], 1),
    (24, (40, 33), [2, 3], [-1, 7], 0),
    # multi-start CALS without jackknife: every model fitted to all of T
    (31, (20, 15, 12), [2, 3, 4, 5, 3, 2], [-1] * 6, 0),
])
def test_sweeps_match_oracle(seed, dims, ranks, lo, nh):
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, sampled_mode=nh)
    sweeps = 4
    say("sweep parity", seed, dims)
    res = oracle.jk_als(np.asarray(wl.T), nh, wl.ranks, wl.left_out, wl.init, sweeps,
                        record_factors=range(1, sweeps + 1))
    ctx = make_ctx(wl)
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        _compare_iteration(wl, ctx, res, t)


@pytest.mark.parametrize("seed,dims,ranks,lo,true_rank", [
    (32, (14, 12, 10), [1, 1, 1, 1], [-1, 0, 5, 13], 1),     # one rank 1 for every model
    (33, (18, 15, 13), [9, 9, 9], [-1, 4, 17], 9),           # one rank above 8
])
def test_uniform_rank_sweeps_match_oracle(seed, dims, ranks, lo, true_rank):
    """Models that all share one rank take the update's fast path (columns
    and Gram blocks from the model index); rank 1 and a rank above 8 (the
    factorisation in LDS after M is staged) against the oracle per
    iteration."""
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, true_rank=true_rank)
    sweeps = 4
    say("uniform-rank sweep parity", seed, ranks[0])
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, sweeps,
                        record_factors=range(1, sweeps + 1))
    for k in res:
        assert np.linalg.cond(res[k].H_last) <= 1e4, k
    ctx = make_ctx(wl)
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        _compare_iteration(wl, ctx, res, t)


@pytest.mark.parametrize("dims,lo", [
    ((2, 9, 8), [-1, 0, 1]),     # a sampled mode of two: each submodel fits one slice
    ((3, 1, 7), [-1, 0, 2]),     # a mode of size one (two submodels fit exactly)
])
def test_degenerate_shapes_match_oracle(dims, lo):
    """Degenerate shapes per iteration at 1e-11; a submodel that fits its
    reduced tensor exactly has an error at rounding level (the Gram identity
    cancels), so its fit is checked against the bound the error's agreement
    implies."""
    wl = synth.random_problem(51, dims, [2, 2, 2], lo, noise=0.1, true_rank=2)
    sweeps = 3
    say("degenerate shape", dims)
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, sweeps,
                        record_factors=range(1, sweeps + 1))
    ctx = make_ctx(wl)
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        _compare_iteration(wl, ctx, res, t, fit_from_err=True)


def test_config1_trajectory_50_sweeps():
    """Config 1 (20x30x40, rank 3, 1 % noise, 20 leave-one-out + full
    model, 50 sweeps): every iteration of every model."""
    wl = synth.config1()
    say("c1 trajectory")
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, wl.sweeps,
                        record_factors=range(1, wl.sweeps + 1))
    ctx = make_ctx(wl)
    worst = 0.0
    for t in range(1, wl.sweeps + 1):
        ctx.sweep(1)
        worst = max(worst, _compare_iteration(wl, ctx, res, t))
    say("c1 worst rel err", worst)


def test_config2_sampled_models():
    """Benchmark workload (100x200x200, 100 models): sampled submodels
    checked per iteration for 10 sweeps."""
    wl = synth.config2()
    models = [0, 49, 99]
    say("c2 sweep parity")
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 10,
                        models=models, record_factors=range(1, 11))
    ctx = make_ctx(wl)
    for t in range(1, 11):
        ctx.sweep(1)
        _compare_iteration(wl, ctx, res, t, models=models)


def test_config2_bench_tilings_sampled_models():
    """The benchmark workload in the launch configuration bench.py times: the
    tilings of the shipped tuned table (each mode's fused MTTKRP with its
    split count, and the shared contraction W), sampled submodels checked per
    iteration for 10 sweeps."""
    wl = synth.config2()
    models = [0, 50, 99]
    ctx = make_ctx(wl)
    tilings = shipped_tilings(wl)
    assert sorted(tilings) == [0, 1, 2, 3]
    descs = apply_tilings(ctx, tilings)
    say("c2 bench tilings", descs)
    for n in range(3):
        assert (" s%d " % tilings[n][1]) in descs[n], descs[n]
    assert descs[3].startswith("tree ")
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 10,
                        models=models, record_factors=range(1, 11))
    for t in range(1, 11):
        ctx.sweep(1)
        _compare_iteration(wl, ctx, res, t, models=models)


def test_sweeps_bitwise_repeatable_and_resumable():
    wl = synth.random_problem(25, (30, 25, 20), [4, 4, 4], [-1, 3, 29], noise=0.05)
    a = make_ctx(wl)
    a.sweep(6)
    b = make_ctx(wl)
    b.sweep(3)
    # checkpoint b after 3 sweeps into a fresh context, then 3 more sweeps
    c = make_ctx(wl)
    for n in range(3):
        U, lam = b.get_factors(n)
        c.set_factors(n, U, lam)
    c.sweep(3)
    b.sweep(3)
    for n in range(3):
        ua, ub, uc = (to_np(x.get_factors(n)[0]) for x in (a, b, c))
        assert np.array_equal(ua, ub)
        assert np.array_equal(ua, uc)


def test_nan_model_leaves_others_bitwise_unchanged():
    wl = synth.random_problem(26, (20, 15, 10), [3, 3, 3], [-1, 2, 19], noise=0.05)
    ref = make_ctx(wl)
    ref.sweep(3)
    bad = synth.random_problem(26, (20, 15, 10), [3, 3, 3], [-1, 2, 19], noise=0.05)
    bad.init[1][0, 3] = np.nan          # model 1, column 0
    ctx = make_ctx(bad)
    ctx.sweep(3)
    st = to_np(ctx.get_status()[2])
    assert st[1] & jk.JKC_ST_NONFINITE
    for n in range(3):
        a, b = to_np(ref.get_factors(n)[0]), to_np(ctx.get_factors(n)[0])
        for k in (0, 2):
            assert np.array_equal(a[:, cols(wl, k)], b[:, cols(wl, k)])


def test_singular_normal_matrix_uses_pseudoinverse():
    wl = synth.random_problem(27, (12, 10, 9), [3], [-1], noise=0.1)
    for n in (1, 2):
        wl.init[n][:, 2] = wl.init[n][:, 1]
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 1,
                        record_factors=[1])
    assert res[0].fallbacks > 0
    ctx = make_ctx(wl)
    ctx.sweep(1)
    st = to_np(ctx.get_status()[2])
    assert st[0] & jk.JKC_ST_FALLBACK
    U0 = to_np(ctx.get_factors(0)[0])
    # mode 0 used the pseudoinverse; a minimum-norm solution is unique
    assert rel(U0, res[0].U_hist[1][0]) <= 1e-6


def test_fit_with_tolerance_freezes_models():
    wl = synth.random_problem(28, (25, 20, 15), [2, 2, 2], [-1, 0, 24], noise=0.02, true_rank=2)
    say("fit tol")
    ctx = make_ctx(wl)
    iters, fit, status = ctx.fit(500, 1e-7)
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 500, tol=1e-7)
    for k in range(wl.K):
        assert status[k] & jk.JKC_ST_CONVERGED
        assert abs(int(iters[k]) - res[k].iters) <= 1
        assert abs(fit[k] - res[k].fit_hist[-1]) <= 1e-6


def test_uniform_rank_fast_path_matches_table_path():
    """Models of one rank in the canonical column layout take the update's
    fast path (columns and Gram blocks computed from the model index); once
    convergence compaction has moved columns, the same models are updated
    through the model table.  A tolerance fit with compaction must equal one
    without it bit for bit, so both paths compute the same update."""
    wl = synth.random_problem(41, (30, 25, 20), [4] * 12, [-1] + list(range(11)), noise=0.0,
                              true_rank=4)
    say("uniform-rank fast path vs table path")
    a = make_ctx(wl)
    b = make_ctx(wl)
    b.set_compaction(False)
    ia, fa, sa = a.fit(300, 1e-7)
    ib, fb, sb = b.fit(300, 1e-7)
    it = np.sort(np.asarray(ia))
    say("iterations", it.tolist())
    # at least 3 models (12 of 48 columns, past the one-fifth threshold)
    # converged while others were still fitted: compaction moved columns
    assert it[2] < it[-1]
    assert np.array_equal(np.asarray(ia), np.asarray(ib))
    assert np.array_equal(np.asarray(sa), np.asarray(sb))
    assert np.array_equal(np.asarray(fa), np.asarray(fb))
    for n in range(3):
        ua, la = (to_np(x) for x in a.get_factors(n))
        ub, lb = (to_np(x) for x in b.get_factors(n))
        assert np.array_equal(ua, ub) and np.array_equal(la, lb)


def test_remove_slice_bit_exact():
    import torch
    rng = np.random.default_rng(3)
    for dims, nh in (((5, 4, 3), 0), ((5, 4, 3), 1), ((3, 4, 5, 2), 3), ((6, 7), 1)):
        for dt in (np.float64, np.float32):
            T = np.asfortranarray(rng.standard_normal(dims).astype(dt))
            Td = jk.to_device_tensor(T)
            for p in (0, dims[nh] - 1, dims[nh] // 2):
                out = to_np(jk.jk_cals_remove_slice(Td, dims, nh, p))
                ref = np.delete(T, p, axis=nh).ravel(order="F")
                assert out.dtype == ref.dtype and np.array_equal(out, ref)


@pytest.mark.parametrize("dims", [(35, 28, 22), (150, 70, 9)])
def test_update_kernels_agree(dims):
    """The LDS-staged (default), global-memory and row-parallel update kernels
    compute the same update; their fixed summation orders differ, so they agree
    to rounding.  The second shape has a mode of 150 rows (three row chunks)."""
    wl = synth.random_problem(29, dims, [5, 3, 7, 1], [-1, 0, dims[0] - 1, 9], noise=0.05)
    ctxs = [make_ctx(wl) for _ in range(3)]
    ctxs[1].set_update_kernel(1)
    ctxs[2].set_update_kernel(2)
    for c in ctxs:
        c.sweep(4)
    for n in range(3):
        ua, la = (to_np(x) for x in ctxs[0].get_factors(n))
        for c in ctxs[1:]:
            ub, lb = (to_np(x) for x in c.get_factors(n))
            assert rel(ua, ub) <= 1e-13 and rel(la, lb) <= 1e-13
    ea = to_np(ctxs[0].get_status()[0])
    for c in ctxs[1:]:
        assert np.allclose(ea, to_np(c.get_status()[0]), rtol=1e-12, atol=0)


def test_graph_replays_match_direct_launches():
    """Multi-sweep runs replay a captured graph of one sweep; every replay,
    with eager work and synchronisation in between, must give the same bits
    as launching the kernels directly."""
    import torch
    wl = synth.random_problem(30, (33, 26, 21), [4, 2, 5], [-1, 12, 32], noise=0.05)
    g = make_ctx(wl)
    g.set_sweep_graph(True)
    d = make_ctx(wl)
    d.set_sweep_graph(False)
    for rep in range(4):
        g.sweep(2)                       # graph path (two replays)
        d.sweep(1)
        d.sweep(1)                       # direct path
        torch.cuda.synchronize()
        _ = to_np(g.mttkrp(0))           # eager work between replays
        for n in range(3):
            assert np.array_equal(to_np(g.get_factors(n)[0]), to_np(d.get_factors(n)[0])), (rep, n)
        assert np.array_equal(to_np(g.get_status()[1]), to_np(d.get_status()[1]))


def test_convergence_compaction_is_bitwise_neutral():
    """jk_cals_fit moves the models still being fitted to the front once a
    fifth of the columns belong to converged models; every model's sums run
    in the same order wherever its columns sit, so factors, lambda, fits,
    iteration counts and flags are bitwise those of a fit without it.  The
    uneven-batch workload with 10 samples per parent (500 models of ranks
    1..10, which converge after 4 to ~30 sweeps)."""
    wl = synth.config3(samples=list(range(0, 300, 30)))
    say("compaction", wl.K)
    a = make_ctx(wl)
    b = make_ctx(wl)
    b.set_compaction(False)
    ia, fa, sa = a.fit(300, 1e-6)
    ib, fb, sb = b.fit(300, 1e-6)
    assert np.array_equal(np.asarray(ia), np.asarray(ib))
    assert np.array_equal(np.asarray(sa), np.asarray(sb))
    assert np.array_equal(np.asarray(fa), np.asarray(fb))
    assert len(set(np.asarray(ia).tolist())) > 3          # convergence is spread out
    for n in range(3):
        ua, la = (to_np(x) for x in a.get_factors(n))
        ub, lb = (to_np(x) for x in b.get_factors(n))
        assert np.array_equal(ua, ub) and np.array_equal(la, lb)
    # the canonical layout is back: a further sweep matches too
    a.sweep(1)
    b.sweep(1)
    assert np.array_equal(to_np(a.get_factors(2)[0]), to_np(b.get_factors(2)[0]))
