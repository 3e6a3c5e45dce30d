"""Parity of the fused float64 MTTKRP (Alg. 3, MTTKRP step) with the oracle's
per-submodel MTTKRP on the explicitly reduced tensor (Sec. 4.1, Case I and
Case II).  Each model's block of the fused result must match its own
MTTKRP to 1e-12 relative (float64 sums in a different order)."""
import numpy as np
import pytest

import synth
from gpu_util import make_ctx, oracle_model_mttkrp, rel, say, to_np, cols

pytestmark = pytest.mark.gpu

TOL = 1e-12

SPECS = [
    # (seed, dims, ranks, left_out, sampled_mode)
    (1, (37, 29, 23), [3, 5, 1, 7], [-1, 0, 36, 11], 0),
    (2, (70, 45, 33), [5, 3, 7, 1, 16, 2], [-1, 69, 0, 5, 30, 68], 0),
    (3, (150, 20, 17), [4] * 9, list(range(9)), 0),
    (4, (13, 11, 9, 7), [2, 3, 4], [-1, 12, 6], 0),
    (5, (21, 40, 19), [3, 2, 32], [5, -1, 39], 1),
    (6, (9, 8, 70), [6, 6], [69, 0], 2),
    (7, (33, 65), [3, 4, 2], [-1, 3, 32], 0),
]


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_fused_mttkrp_matches_per_model(spec):
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, sampled_mode=nh)
    say("mttkrp", seed, dims, ranks, lo, nh)
    ctx = make_ctx(wl)
    worst = 0.0
    for n in range(len(dims)):
        M = to_np(ctx.mttkrp(n))
        for k in range(wl.K):
            ref = oracle_model_mttkrp(wl, k, n)
            e = rel(M[:, cols(wl, k)], ref)
            worst = max(worst, e)
            assert e <= TOL, (n, k, e, ctx.describe(n))
    say("worst rel err", worst)


def test_every_tiling_matches():
    wl = synth.random_problem(11, (67, 31, 26), [5, 9, 2], [-1, 66, 3], noise=0.1)
    ctx = make_ctx(wl)
    refs = {(n, k): oracle_model_mttkrp(wl, k, n) for n in range(3) for k in range(wl.K)}
    for v in range(ctx.num_tilings()):
        for splits in (1, 3, 8):
            for n in range(3):
                say("tiling", v, splits, n)
                ctx.set_tiling(n, v, splits)
                M = to_np(ctx.mttkrp(n))
                for k in range(wl.K):
                    e = rel(M[:, cols(wl, k)], refs[(n, k)])
                    assert e <= TOL, (v, splits, n, k, e, ctx.describe(n))


def test_float32_tensor_is_read_exactly():
    wl = synth.random_problem(12, (40, 30, 20), [4, 4], [-1, 7], noise=0.05, dtype=np.float32)
    say("f32 tensor")
    ctx = make_ctx(wl)
    for n in range(3):
        M = to_np(ctx.mttkrp(n))
        for k in range(wl.K):
            assert rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n)) <= TOL


def test_in_place_tensor():
    wl = synth.random_problem(13, (30, 20, 10), [3, 3], [-1, 29], noise=0.05)
    say("copy_tensor=0")
    ctx = make_ctx(wl, copy_tensor=False)
    for n in range(3):
        M = to_np(ctx.mttkrp(n))
        for k in range(wl.K):
            assert rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n)) <= TOL


def test_mttkrp_bitwise_repeatable():
    wl = synth.random_problem(14, (90, 60, 40), [5] * 12, list(range(12)), noise=0.1)
    ctx = make_ctx(wl)
    for n in range(3):
        a = to_np(ctx.mttkrp(n))
        b = to_np(ctx.mttkrp(n))
        assert np.array_equal(a, b)


def test_config2_full_size_sampled_models():
    """The benchmark workload (100x200x200, 100 leave-one-out models of rank
    5) in its default launch configuration; sampled models checked."""
    wl = synth.config2()
    say("c2 full mttkrp")
    ctx = make_ctx(wl)
    for n in range(3):
        M = to_np(ctx.mttkrp(n))
        for k in (0, 37, 99):
            e = rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
            assert e <= TOL, (n, k, e, ctx.describe(n))


def test_case_I_row_is_zero_and_full_model_row_is_not():
    wl = synth.random_problem(15, (12, 10, 8), [2, 2], [-1, 4], noise=0.1)
    ctx = make_ctx(wl)
    M = to_np(ctx.mttkrp(0))
    assert np.all(M[4, 2:4] == 0.0)
    assert np.all(M[4, 0:2] != 0.0)
