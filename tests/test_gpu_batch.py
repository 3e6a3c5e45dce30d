"""Batches of uneven models in one launch (ranks 1..10, several inits per
rank, all leave-one-out samples), as in the multi-model workflow: every
model's trajectory must match its own independent ALS run."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import make_ctx, rel, say, to_np, cols

pytestmark = pytest.mark.gpu


def _tol(r):
    """1e-11 when the last normal matrix has condition number <= 1e4;
    otherwise a conditioning-scaled bound (forward error ~ kappa * eps)."""
    kappa = float(np.linalg.cond(r.H_last))
    return (1e-11 if kappa <= 1e4 else 50.0 * kappa * 2.2e-16), kappa


def test_uneven_batch_small():
    wl = synth.config3(dims=(12, 10, 9), rank_max=10, inits_per_rank=2)
    say("uneven batch", wl.K, wl.C)
    sweeps = 3
    ctx = make_ctx(wl)
    ctx.sweep(sweeps)
    facs = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
    err = to_np(ctx.get_status()[0])
    rng = np.random.default_rng(1)
    models = sorted(set(rng.choice(wl.K, 40, replace=False).tolist() + [0, wl.K - 1]))
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, sweeps, models=models)
    for k in models:
        r = res[k]
        c = cols(wl, k)
        tol, kappa = _tol(r)
        Up = r.padded()
        for n in range(3):
            e = rel(facs[n][:, c], Up[n])
            assert e <= tol, (k, int(wl.ranks[k]), n, e, kappa)
        assert abs(err[k] - r.e_hist[-1]) <= max(tol, 1e-11) * r.normT2


def test_config3_full_size_sampled_models():
    """300x250x200 rank-8 noise-free tensor; ranks 1..10 x 5 inits x 300
    samples = 15,000 models (C = 82,500) in one fused launch per mode;
    stratified sample of models checked after 2 sweeps."""
    wl = synth.config3()
    say("c3 full", wl.K, wl.C)
    sweeps = 2
    ctx = make_ctx(wl)
    ctx.sweep(sweeps)
    facs = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
    err = to_np(ctx.get_status()[0])
    models = []
    per_parent = 300
    for parent in (0, 7, 22, 35, 49):        # ranks 1, 2, 5, 8, 10
        for p in (0, 149, 299):
            models.append(parent * per_parent + p)
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, sweeps, models=models)
    for k in models:
        r = res[k]
        tol, kappa = _tol(r)
        Up = r.padded()
        for n in range(3):
            e = rel(facs[n][:, cols(wl, k)], Up[n])
            assert e <= tol, (k, int(wl.ranks[k]), n, e, kappa)
        assert abs(err[k] - r.e_hist[-1]) <= max(tol, 1e-11) * r.normT2
