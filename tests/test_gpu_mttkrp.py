"""Parity of the fused float64 MTTKRP (Alg. 3, MTTKRP step) with the oracle's
per-submodel MTTKRP on the explicitly reduced tensor (Sec. 4.1, Case I and
Case II).  Each model's block of the fused result must match its own
MTTKRP to 1e-12 relative (float64 sums in a different order)."""
import numpy as np
import pytest

import synth
import paper_2112_03985_amd as jk
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


@pytest.mark.parametrize("dims,dtype,split_list", [
    ((67, 31, 26), np.float64, (1, 3, 8)),
    ((19, 13, 11, 7), np.float32, (1, 5)),   # three other modes, float32 storage
])
def test_every_tiling_matches(dims, dtype, split_list):
    wl = synth.random_problem(11, dims, [5, 9, 2], [-1, dims[0] - 1, 3], noise=0.1, dtype=dtype)
    ctx = make_ctx(wl)
    N = len(dims)
    refs = {(n, k): oracle_model_mttkrp(wl, k, n) for n in range(N) for k in range(wl.K)}
    for v in range(ctx.num_tilings()):
        for splits in split_list:
            for n in range(N):
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


def test_tensor_past_2_gib_uses_64_bit_addressing():
    """A float64 tensor of 2^31 bytes or more (1024 x 1024 x 264, 2.2 GB)
    cannot use the buffer-load tilings (32-bit byte offsets): the default
    choice avoids them, the MTTKRP still matches the oracle, and forcing a
    buffer-load tiling is refused."""
    wl = synth.random_problem(15, (1024, 1024, 264), [2, 3], [-1, 5], noise=0.1)
    say("2 GiB tensor")
    ctx = make_ctx(wl, copy_tensor=False)
    for n in (0, 2):
        assert not ctx.describe(n).endswith("-buffer"), ctx.describe(n)
        M = to_np(ctx.mttkrp(n))
        for k in range(wl.K):
            e = rel(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
            assert e <= TOL, (n, k, e, ctx.describe(n))
    refused = 0
    for v in range(ctx.num_tilings()):
        try:
            ctx.set_tiling(0, v, 1)
        except jk.JkcError as e:
            assert "2^31 bytes" in str(e) or "narrow tiling" in str(e)
            refused += 1
        else:
            assert not ctx.describe(0).endswith("-buffer")
    assert refused > 0
