"""Trajectory parity at the iteration budgets the benchmark times (the
fixed-iteration protocol of Sec. 5.1), full-size workloads, sampled models
(columns never interact, so a sample is valid while the GPU still runs the
whole fused launch).  Every result's normwise and elementwise errors are
printed; float64 gate 1e-11 per iteration where kappa(H) <= 1e4 (checked).
Each context runs in the tilings bench.py times (the shipped tuned table)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import apply_tilings, errors, make_ctx, rel, say, shipped_tilings, to_np, cols

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _compare(wl, ctx, recs, t, tol=TOL):
    """GPU factors, lambda and error of the sampled models after sweep t
    against the oracle's records of sweep t; returns the worst error."""
    err = to_np(ctx.get_status()[0])
    facs = [to_np(ctx.get_factors(n)[0]) for n in range(len(wl.dims))]
    lam = to_np(ctx.get_factors(0)[1])
    worst = 0.0
    for k, r in recs.items():
        c = cols(wl, k)
        U_ref = r.padded(r.U_hist[t])
        for n in range(len(wl.dims)):
            fro, mx = errors(facs[n][:, c], U_ref[n])
            worst = max(worst, fro, mx)
            assert max(fro, mx) <= tol, ("U", t, k, n, fro, mx)
        e = rel(lam[c], r.lam_hist[t - 1])
        ee = abs(err[k] - r.e_hist[t - 1]) / r.normT2
        assert e <= tol and ee <= tol, ("lambda/err", t, k, e, ee)
        worst = max(worst, e, ee)
    return worst


@pytest.mark.timeout(900)
def test_config2_100_sweeps_sampled_models():
    """Benchmark workload (100x200x200, 100 leave-one-out models of rank 5):
    three models compared after every one of the 100 sweeps the benchmark
    times."""
    wl = synth.config2()
    models = [0, 49, 99]
    sweeps = 100
    say("c2 100-sweep trajectory: oracle")
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, sweeps,
                        models=models, record_factors=range(1, sweeps + 1))
    say("c2 100-sweep trajectory: GPU")
    ctx = make_ctx(wl)
    say("tilings", apply_tilings(ctx, shipped_tilings(wl)))
    worst = 0.0
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        w = _compare(wl, ctx, res, t)
        worst = max(worst, w)
        if t % 10 == 0:
            say("c2 sweep %d: worst rel err so far %.3e" % (t, worst))
    for k in models:
        kappa = float(np.linalg.cond(res[k].H_last))
        say("c2 model %d: kappa(H) %.2f, fit %.6f" % (k, kappa, res[k].fit_hist[-1]))
        assert kappa <= 1e4


@pytest.mark.timeout(900)
def test_config3_stratified_60_models_5_sweeps():
    """Uneven batch at full size (300x250x200, 15,000 models of ranks 1..10,
    C = 82,500): the stratified sample of all 10 ranks x 2 inits x
    p in {0, 149, 299} (60 models), every one of 5 sweeps."""
    wl = synth.config3()
    sweeps = 5
    per_parent = 300
    models = []
    for R in range(1, 11):
        for init in (0, 3):
            parent = (R - 1) * 5 + init
            for p in (0, 149, 299):
                models.append(parent * per_parent + p)
    assert len(models) == 60
    say("c3 stratified trajectory: oracle (60 models)")
    T = np.asarray(wl.T)
    res = {}
    off = oracle.model_offsets(wl.ranks)
    for p in (0, 149, 299):
        Tk = oracle.reduce_tensor(T, 0, p)
        for k in models:
            if int(wl.left_out[k]) != p:
                continue
            c = slice(int(off[k]), int(off[k] + wl.ranks[k]))
            U0 = [np.array(u[:, c]) for u in wl.init]
            U0[0] = oracle.reduce_init(U0[0], p)
            res[k] = oracle.cp_als(Tk, U0, sweeps, record_factors=range(1, sweeps + 1),
                                   sampled_mode=0, left_out=p)
        say("c3 oracle: p = %d done" % p)
    for k in models:
        assert np.linalg.cond(res[k].H_last) <= 1e4, k
    say("c3 stratified trajectory: GPU")
    ctx = make_ctx(wl)
    say("tilings", apply_tilings(ctx, shipped_tilings(wl)))
    worst = 0.0
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        worst = max(worst, _compare(wl, ctx, res, t))
        say("c3 sweep %d: worst rel err so far %.3e" % (t, worst))


@pytest.mark.timeout(900)
def test_config5_20_sweeps_and_200_refinement_steps():
    """Refinement workload at full size (100x150x150 float32 tensor, rank 10,
    100 leave-one-out models, C = 1000) at its whole budget: 20 ALS sweeps
    (compared every sweep), then 200 gradient steps, then the loss and the
    all-mode gradient, for three sampled models against the oracle running
    the same rule."""
    import torch
    wl = synth.config5()
    models = [0, 57, 99]
    sweeps, steps = 20, 200
    T = np.asarray(wl.T, dtype=np.float64)
    say("c5 budget: oracle ALS")
    res = oracle.jk_als(T, 0, wl.ranks, wl.left_out, wl.init, sweeps, models=models,
                        record_factors=range(1, sweeps + 1))
    ctx = make_ctx(wl)
    say("tilings", apply_tilings(ctx, shipped_tilings(wl)))
    worst = 0.0
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        worst = max(worst, _compare(wl, ctx, res, t))
    say("c5 ALS 20 sweeps worst rel err %.3e" % worst)
    say("c5 budget: GPU refinement")
    loss = torch.empty(wl.K, dtype=torch.float64, device="cuda")
    ctx.refine(steps, loss)
    L = to_np(loss)
    G = [to_np(ctx.get_grad(n)) for n in range(3)]
    facs = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
    say("c5 budget: oracle refinement")
    for k in models:
        r = res[k]
        U = [u.copy() for u in r.U]
        U[-1] = U[-1] * r.lam[None, :]
        Tk = oracle.reduce_tensor(T, 0, int(wl.left_out[k]))
        Ur = oracle.gd_refine(Tk, U, steps)
        Up = r.padded(Ur)
        for n in range(3):
            fro, mx = errors(facs[n][:, cols(wl, k)], Up[n])
            say("c5 model %d mode %d after %d steps: normwise %.3e, elementwise %.3e"
                % (k, n, steps, fro, mx))
            assert max(fro, mx) <= TOL, (k, n, fro, mx)
        f, g = oracle.loss_and_grad(Tk, Ur)
        normT2 = float(np.sum(Tk ** 2))
        assert abs(L[k] - f) <= TOL * normT2, (k, L[k], f)
        gp = r.padded(g)
        for n in range(3):
            # near a stationary point the gradient is a difference of two
            # large terms: its error is measured against the size of the
            # MTTKRP it cancels
            scale = np.sqrt(normT2) * np.prod([np.linalg.norm(Ur[m]) for m in range(3) if m != n])
            e = np.linalg.norm(G[n][:, cols(wl, k)] - gp[n]) / max(scale, np.linalg.norm(gp[n]))
            say("c5 model %d mode %d gradient error %.3e (of the MTTKRP scale)" % (k, n, e))
            assert e <= TOL, (k, n, e)
