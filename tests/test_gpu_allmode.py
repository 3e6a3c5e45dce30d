"""The one-pass all-mode MTTKRP of the loss gradient (jk_cals_set_allmode):
every mode's MTTKRP from a single read of the tensor.  Loss and gradient of
every model against the oracle (explicitly reduced tensors) at 1e-11, and
against the per-mode path of the same library (fused MTTKRP or shared
contraction) at 1e-12, on 3- and 4-way shapes with ragged row, fiber and
column tiles, every sampled mode, delete-d, float32 tensors, the largest
supported mode-0 size (256 rows), the 8-fiber step used when the 16-fiber
block does not fit in LDS, and gradient refinement."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import errors, make_ctx, rel, say, to_np, cols

pytestmark = pytest.mark.gpu

TOL = 1e-11

SPECS = [
    # seed, dims, ranks, left_out, sampled mode
    (81, (37, 29, 23), [3, 5, 1, 7], [-1, 0, 36, 11], 0),
    (82, (13, 11, 9, 7), [2, 3, 12], [-1, 12, 6], 0),
    (83, (70, 45, 33), [12, 12, 8, 9], [3, -1, 69, 0], 0),
    (84, (21, 40, 17), [4, 6], [39, 5], 1),
    (85, (16, 9, 30, 5), [5, 5, 5], [29, 0, -1], 2),
    (86, (24, 18, 10), [7, 2], [9, -1], 2),
]


def _lds_bytes(i0p, bk, I1, I2, N):
    """LDS of one block of the one-pass kernel: the staged tensor tile
    (double-buffered, row pitch 2 mod 32 doubles), the step's U_1 rows and
    per-column entries, U_0, and the mode-1 (and mode-2) accumulators of 32
    columns."""
    pitch = i0p + (2 if i0p % 32 == 0 else 18)
    i1p = -(-I1 // bk) * bk
    doubles = 2 * bk * pitch + 2 * bk * 32 + 4 * 32 + i0p * 32 + i1p * 32 + (I2 * 32 if N == 4 else 0)
    return 8 * doubles


def _reduced(wl, k, facs):
    c = cols(wl, k)
    U = [np.array(f[:, c], dtype=np.float64) for f in facs]
    p = wl.left_out[k]
    nh = wl.sampled_mode
    U[nh] = oracle.reduce_init(U[nh], p)
    Tk = oracle.reduce_tensor(np.asarray(wl.T, dtype=np.float64), nh, p)
    return Tk, U, oracle.left_out_rows(p)


def _allmode_ctx(wl):
    ctx = make_ctx(wl)
    ctx.set_allmode(True)
    return ctx


def _check_against_oracle(wl, ctx, models=None):
    import torch
    loss = torch.empty(wl.K, dtype=torch.float64, device="cuda")
    ctx.loss_grad(loss)
    L = to_np(loss)
    G = [to_np(ctx.get_grad(n)) for n in range(len(wl.dims))]
    worst = 0.0
    for k in (range(wl.K) if models is None else models):
        Tk, U, rows = _reduced(wl, k, wl.init)
        f, g = oracle.loss_and_grad(Tk, U)
        el = abs(L[k] - f) / max(1.0, 0.5 * np.sum(Tk ** 2))
        assert el <= TOL, (k, L[k], f)
        for n in range(len(wl.dims)):
            gn = g[n]
            if n == wl.sampled_mode and rows:
                full = np.zeros((wl.dims[n], gn.shape[1]))
                full[np.setdiff1d(np.arange(wl.dims[n]), rows)] = gn
                gn = full
            fro, mx = errors(G[n][:, cols(wl, k)], gn)
            worst = max(worst, fro, mx)
            assert max(fro, mx) <= TOL, (k, n, fro, mx)
    return worst


def _agree_with_per_mode_path(wl, refine_steps=4):
    import torch
    a, b = _allmode_ctx(wl), make_ctx(wl)
    b.set_allmode(False)
    la = torch.empty(wl.K, dtype=torch.float64, device="cuda")
    lb = torch.empty_like(la)
    a.loss_grad(la)
    b.loss_grad(lb)
    assert rel(to_np(la), to_np(lb)) <= 1e-12
    for n in range(len(wl.dims)):
        assert rel(to_np(a.get_grad(n)), to_np(b.get_grad(n))) <= 1e-12, n
    a.refine(refine_steps)
    b.refine(refine_steps)
    for n in range(len(wl.dims)):
        assert rel(to_np(a.get_factors(n)[0]), to_np(b.get_factors(n)[0])) <= 1e-11, n


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_allmode_loss_and_gradient_match_oracle(spec):
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.2, sampled_mode=nh)
    say("allmode grad", seed, dims)
    worst = _check_against_oracle(wl, _allmode_ctx(wl))
    say("allmode grad worst rel err", worst)


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_allmode_agrees_with_per_mode_path(spec):
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.2, sampled_mode=nh)
    say("allmode vs per-mode", seed)
    _agree_with_per_mode_path(wl)


def test_allmode_float32_tensor_and_delete_d():
    wl = synth.random_problem(87, (33, 20, 19), [3, 4, 2], [-1, 5, 32], noise=0.1,
                              dtype=np.float32)
    say("allmode f32")
    _check_against_oracle(wl, _allmode_ctx(wl))
    # delete-2: two zero rows per submodel in mode 0
    wl2 = synth.random_problem(88, (26, 15, 12, 4), [3, 2, 4], [[-1, -1], [0, 25], [7, 8]],
                               noise=0.1)
    say("allmode delete-2")
    _check_against_oracle(wl2, _allmode_ctx(wl2))


def test_allmode_largest_mode0_and_8_fiber_step():
    # 256 rows in mode 0: every 16-row tile of the mode-0 accumulators in use
    wl = synth.random_problem(89, (256, 21, 6), [3, 2], [-1, 255], noise=0.1)
    say("allmode 256 rows")
    _check_against_oracle(wl, _allmode_ctx(wl))
    # a 4-way block whose 16-fiber staging would not fit in LDS: 8 fibers per step
    wl8 = synth.random_problem(90, (200, 120, 100, 2), [2, 3], [-1, 17], noise=0.1)
    assert _lds_bytes(208, 16, 120, 100, 4) > 160 * 1024 >= _lds_bytes(208, 8, 120, 100, 4)
    say("allmode 8-fiber step")
    _check_against_oracle(wl8, _allmode_ctx(wl8))
    _agree_with_per_mode_path(wl8, refine_steps=1)


def test_allmode_default_follows_the_shared_contraction():
    """On where no shared contraction is held (4-way), off for 3-way float64
    problems that hold W; switching it on there changes only rounding."""
    wl3 = synth.random_problem(94, (12, 10, 8), [2, 3], [-1, 4], noise=0.1)
    wl4 = synth.random_problem(95, (12, 10, 8, 3), [2, 3], [-1, 4], noise=0.1)
    c3, c4 = make_ctx(wl3), make_ctx(wl4)
    assert c3.describe(3).startswith("tree")
    import torch
    la = torch.empty(wl4.K, dtype=torch.float64, device="cuda")
    lb = torch.empty_like(la)
    c4.loss_grad(la)
    ref = make_ctx(wl4)
    ref.set_allmode(True)
    ref.loss_grad(lb)
    assert np.array_equal(to_np(la), to_np(lb))   # the default is the one-pass kernel


def test_allmode_refused_where_not_available():
    wl = synth.random_problem(91, (257, 5, 4), [2], [-1])
    ctx = make_ctx(wl)
    with pytest.raises(jk.JkcError) as e:
        ctx.set_allmode(True)
    assert e.value.status == jk.JKC_EUNSUPPORTED
    ctx.set_allmode(False)
    wl2 = synth.random_problem(92, (6, 5), [2], [-1])
    with pytest.raises(jk.JkcError):
        make_ctx(wl2).set_allmode(True)
    wl3 = synth.random_problem(93, (6, 5, 4), [2], [-1])
    with pytest.raises(jk.JkcError):
        make_ctx(wl3, precision=jk.JKC_SPLIT_BF16X3).set_allmode(True)


def test_allmode_config5_full_size_sampled_models():
    """The refinement workload at full size (100x150x150 float32 tensor,
    100 leave-one-out models of rank 10): loss and gradient of sampled models
    against the oracle and the whole gradient against the per-mode path."""
    wl = synth.config5()
    say("allmode c5 full size")
    _check_against_oracle(wl, _allmode_ctx(wl), models=[0, 49, 99])
    _agree_with_per_mode_path(wl, refine_steps=2)
