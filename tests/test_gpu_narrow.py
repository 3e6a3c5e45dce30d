"""The narrow vector-ALU MTTKRP (problems of at most 16 columns: the plain
per-submodel ALS of Alg. 2): chosen by default where it applies, per model
against the oracle at 1e-12 in every mode (3- and 4-way, every sampled
mode, float32 tensors, delete-d, K chunks of whole fibers), agreement with a
matrix-core tiling, a plain one-model ALS trajectory on the benchmark
tensor against the oracle at 1e-11, and refusal where it does not apply."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import errors, make_ctx, oracle_model_mttkrp, rel, say, to_np, cols

pytestmark = pytest.mark.gpu

TOL = 1e-12

SPECS = [
    # seed, dims, ranks, left_out, sampled mode
    (101, (37, 29, 23), [3, 5, 1], [-1, 0, 36], 0),
    (102, (13, 11, 9, 7), [2, 3], [-1, 12], 0),
    (103, (70, 45, 33), [6, 8, 2], [3, -1, 69], 0),
    (104, (21, 40, 17), [4, 6], [39, 5], 1),
    (105, (16, 9, 30, 5), [5, 5, 5], [29, 0, -1], 2),
    (106, (130, 12, 10), [2, 3], [-1, 100], 0),       # three lane slots
    (107, (200, 15, 11), [5], [17], 0),               # four lane slots, 8 columns
]


def _narrow_index(ctx):
    for v in range(ctx.num_tilings() - 1, -1, -1):
        try:
            ctx.set_tiling(0, v, 1)
        except jk.JkcError:
            continue
        if "valu-narrow" in ctx.describe(0):
            return v
    raise AssertionError("no narrow tiling")


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_narrow_mttkrp_matches_oracle_every_mode(spec):
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, sampled_mode=nh)
    say("narrow mttkrp", seed, dims)
    ctx = make_ctx(wl)
    for n in range(len(dims)):
        assert "valu-narrow" in ctx.describe(n), ctx.describe(n)
    v = _narrow_index(ctx)
    for splits in (1, 3, 64):
        for n in range(len(dims)):
            ctx.set_tiling(n, v, splits)
            M = to_np(ctx.mttkrp(n))
            for k in range(wl.K):
                fro, mx = errors(M[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
                assert max(fro, mx) <= TOL, (splits, n, k, fro, mx)


def test_narrow_finish_repeats_bitwise():
    """The kernels' own split-K finish leaves its arrival counters zeroed:
    repeated launches give the same bits, with ragged row tiles (31 and 22
    rows) and chunk counts that do not divide the fibers."""
    wl = synth.random_problem(111, (45, 31, 22), [4, 3], [7, -1], noise=0.1)
    say("narrow finish repeats")
    ctx = make_ctx(wl)
    v = _narrow_index(ctx)
    for splits in (5, 17):
        for n in range(3):
            ctx.set_tiling(n, v, splits)
            first = to_np(ctx.mttkrp(n))
            for _ in range(3):
                assert np.array_equal(to_np(ctx.mttkrp(n)), first), (splits, n)
            for k in range(wl.K):
                fro, mx = errors(first[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n))
                assert max(fro, mx) <= TOL, (splits, n, k, fro, mx)


def test_narrow_float32_delete_d_and_agreement_with_matrix_cores():
    wl = synth.random_problem(108, (33, 20, 19), [3, 4, 2], [[-1, -1], [0, 32], [5, 6]], noise=0.1,
                              dtype=np.float32)
    say("narrow f32 delete-2")
    a = make_ctx(wl)
    b = make_ctx(wl)
    for n in range(3):
        b.set_tiling(n, 0, 2)          # a matrix-core tiling
        Ma, Mb = to_np(a.mttkrp(n)), to_np(b.mttkrp(n))
        assert rel(Ma, Mb) <= TOL, n
        for k in range(wl.K):
            assert rel(Ma[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n)) <= TOL, (n, k)


def test_plain_one_model_als_on_the_benchmark_tensor():
    """Plain per-submodel ALS as the benchmark runs it: slice p removed
    explicitly (Alg. 2), a one-model context of rank 5 on the reduced
    99x200x200 tensor, every mode through the narrow MTTKRP (no shared
    contraction); 10 sweeps against the oracle's submodel fit per iteration."""
    import torch
    wl = synth.config2()
    p = 17
    k = 17
    red = np.delete(np.asarray(wl.T), p, axis=0)
    dims = list(red.shape)
    c = slice(5 * k, 5 * k + 5)
    init = [np.ascontiguousarray(np.delete(wl.init[0][:, c], p, axis=0)),
            np.ascontiguousarray(wl.init[1][:, c]), np.ascontiguousarray(wl.init[2][:, c])]
    Tg = jk.to_device_tensor(red)
    ctx = jk.JkCals(Tg, dims, 0, [5], [-1], [torch.from_numpy(u).cuda() for u in init])
    ctx.set_mttkrp_tree(False)
    for n in range(3):
        assert "valu-narrow" in ctx.describe(n)
    sweeps = 10
    say("plain one-model ALS, config-2 tensor, model", k)
    res = oracle.jk_als(red, 0, np.array([5]), np.array([-1]), init, sweeps,
                        record_factors=range(1, sweeps + 1))[0]
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        U = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
        for n in range(3):
            fro, mx = errors(U[n], res.U_hist[t][n])
            assert max(fro, mx) <= 1e-11, (t, n, fro, mx)
        err = to_np(ctx.get_status()[0])[0]
        assert abs(err - res.e_hist[t - 1]) <= 1e-11 * res.normT2


def test_narrow_refused_where_it_does_not_apply():
    wl = synth.random_problem(109, (12, 10, 8), [9, 9], [-1, 3])       # 18 columns
    ctx = make_ctx(wl)
    last = ctx.num_tilings() - 1
    with pytest.raises(jk.JkcError) as e:
        ctx.set_tiling(0, last, 1)
    assert "narrow tiling" in str(e.value)
    wl2 = synth.random_problem(110, (300, 6, 5), [3], [-1])             # 300 rows in mode 0
    ctx2 = make_ctx(wl2)
    assert "valu-narrow" not in ctx2.describe(1)
    with pytest.raises(jk.JkcError):
        ctx2.set_tiling(1, ctx2.num_tilings() - 1, 1)
