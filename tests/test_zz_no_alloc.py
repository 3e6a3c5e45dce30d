"""The allocation-free MTTKRP entry point (jk_cals_mttkrp_static) against
the context-based one (jk_cals_mttkrp) and the oracle: two calls in a row
on one GPU, the second on a smaller problem, so the shared fixed scratch is
reused with a different layout; every mode of both problems, including the
sampled mode (Case I rows) and a float32 tensor."""
import numpy as np
import pytest
import torch

import synth
import paper_2112_03985_amd as jk
from gpu_util import device_inputs, errors, make_ctx, oracle_model_mttkrp, say, to_np, cols

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _run(wl):
    T, init = device_inputs(wl)
    f32 = T.dtype == torch.float32
    ctx = jk.JkCals(T, wl.dims, wl.sampled_mode, wl.ranks, wl.left_out, init)
    # the no-allocation call gets its output buffer from the caller
    outs = [torch.empty((d, int(np.sum(wl.ranks))), dtype=torch.float64, device="cuda") for d in wl.dims]
    for n in range(len(wl.dims)):
        say("static mttkrp", wl.dims, "mode", n, "f32" if f32 else "f64")
        jk.jk_cals_mttkrp_static(T, wl.dims, wl.sampled_mode, wl.ranks, wl.left_out, init, n,
                                 out=outs[n])
        ref = to_np(ctx.mttkrp(n))
        got = to_np(outs[n])
        fro, mx = errors(got, ref)
        say("static vs context mode %d: normwise %.3e, elementwise %.3e" % (n, fro, mx))
        assert max(fro, mx) <= TOL, (n, fro, mx)
        for k in (0, wl.K - 1):
            e = max(errors(got[:, cols(wl, k)], oracle_model_mttkrp(wl, k, n)))
            assert e <= TOL, (n, k, e)
    torch.cuda.synchronize()


def test_static_mttkrp_two_calls_second_smaller():
    big = synth.random_problem(71, (96, 70, 50), [3, 5, 4, 2, 6, 3, 1, 5], [-1, 0, 95, 7, 40, 3, 12, 60],
                               noise=0.01)
    small = synth.random_problem(72, (21, 13, 9), [2, 3, 1], [-1, 20, 4], noise=0.01)
    _run(big)
    _run(small)


def test_static_mttkrp_float32_tensor_and_4way():
    wl = synth.random_problem(73, (17, 11, 9, 7), [2, 3, 2], [5, -1, 16], noise=0.01,
                              dtype=np.float32)
    _run(wl)
