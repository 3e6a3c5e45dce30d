"""Split-precision path: the fused MTTKRP as three bfloat16 MFMA products
with float32 accumulation flushed to float64 (everything after it in
float64), against the float64 oracle.  The gate is 1e-5 relative per model;
each test prints the largest error it saw."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import make_ctx, oracle_model_mttkrp, rel, say, to_np, cols

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.mark.parametrize("seed,dims,ranks,lo", [
    (61, (37, 29, 23), [3, 5, 1, 7], [-1, 0, 36, 11]),
    (62, (13, 11, 9, 7), [2, 3, 12], [-1, 12, 6]),
    (63, (70, 45, 33), [12, 12, 8], [3, -1, 69]),
])
def test_split_mttkrp_within_gate(seed, dims, ranks, lo):
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.01)
    say("split mttkrp", seed)
    ctx = make_ctx(wl, precision=jk.JKC_SPLIT_BF16X3)
    worst = 0.0
    for n in range(len(dims)):
        M = to_np(ctx.mttkrp(n))
        for k in range(wl.K):
            e = rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
            worst = max(worst, e)
            assert e <= TOL, (n, k, e)
    say("split mttkrp worst rel err", worst)
    assert worst > 0.0   # it really is a reduced-precision path


def test_split_every_tiling():
    wl = synth.random_problem(64, (67, 31, 26), [5, 9, 2], [-1, 66, 3], noise=0.01)
    ctx = make_ctx(wl, precision=jk.JKC_SPLIT_BF16X3)
    refs = {(n, k): oracle_model_mttkrp(wl, k, n) for n in range(3) for k in range(wl.K)}
    for v in range(ctx.num_tilings()):
        for n in range(3):
            ctx.set_tiling(n, v, 4)
            M = to_np(ctx.mttkrp(n))
            for k in range(wl.K):
                assert rel(M[:, cols(wl, k)], refs[(n, k)]) <= TOL, (v, n, k)


def test_split_one_sweep_against_oracle():
    """One full sweep in split precision from the same init as the oracle:
    factors, lambda and fit.  Errors are stated."""
    wl = synth.random_problem(65, (40, 30, 20), [4, 4, 4], [-1, 0, 39], noise=0.01, true_rank=4)
    res = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 1, record_factors=[1])
    ctx = make_ctx(wl, precision=jk.JKC_SPLIT_BF16X3)
    ctx.sweep(1)
    fit = to_np(ctx.get_status()[1])
    worst = 0.0
    for k, r in res.items():
        Up = r.padded(r.U_hist[1])
        for n in range(3):
            e = rel(to_np(ctx.get_factors(n)[0])[:, cols(wl, k)], Up[n])
            worst = max(worst, e)
            assert e <= TOL, (k, n, e)
        assert abs(fit[k] - r.fit_hist[0]) <= TOL
    say("split one-sweep worst factor rel err", worst)


def test_config4_full_size_sampled_models():
    """The split-precision workload at full size: 200x120x100x80 float64
    tensor of rank 12 with 1 % noise, 200 leave-one-out models of rank 12
    (C = 2400); sampled models' MTTKRP in every mode."""
    wl = synth.config4()
    say("c4 full split mttkrp")
    ctx = make_ctx(wl, precision=jk.JKC_SPLIT_BF16X3)
    worst = 0.0
    for n in range(4):
        M = to_np(ctx.mttkrp(n))
        for k in (0, 199):
            e = rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
            worst = max(worst, e)
            assert e <= TOL, (n, k, e, ctx.describe(n))
    say("c4 worst rel err", worst)
