"""The shared partial contraction of 3-way float64 sweeps (W = T x_2 U_2 at
mode 0, the MTTKRPs of modes 0 and 1 read from W): per-iteration parity with
the oracle's independent per-submodel ALS at 1e-11 for every sampled mode,
delete-d and shapes spanning several tiles with ragged tails; agreement with
the fused MTTKRP path (rounding only); bitwise repeatability; refusal where
W is not held."""
import numpy as np
import pytest

import oracle
import synth
import paper_2112_03985_amd as jk
from gpu_util import make_ctx, rel, say, to_np, cols, variant_geometry

pytestmark = pytest.mark.gpu

SPECS = [
    # (seed, dims, ranks, left_out, sampled_mode)
    (61, (37, 45, 23), [3, 5, 2, 4], [-1, 0, 36, 17], 0),
    (62, (19, 26, 31), [4, 1, 6], [25, -1, 3], 1),
    (63, (14, 11, 29), [2, 3, 3, 5, 1], [28, 0, -1, 13, 7], 2),
    (64, (150, 70, 9), [5, 3, 7], [-1, 149, 64], 0),
    (65, (23, 17, 40), [3, 2], [[4, 9, 16], [0, 1, 2]], 0),     # delete-3
]


@pytest.mark.parametrize("spec", SPECS, ids=[str(s[0]) for s in SPECS])
def test_tree_sweeps_match_oracle(spec):
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, sampled_mode=nh)
    sweeps = 4
    say("tree sweep parity", seed, dims, nh)
    res = oracle.jk_als(np.asarray(wl.T), nh, wl.ranks, wl.left_out, wl.init, sweeps,
                        record_factors=range(1, sweeps + 1))
    ctx = make_ctx(wl)
    for t in range(1, sweeps + 1):
        ctx.sweep(1)
        err, fit = (to_np(x) for x in ctx.get_status()[:2])
        lam = to_np(ctx.get_factors(0)[1])
        facs = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
        for k, r in res.items():
            c = cols(wl, k)
            ref = r.padded(r.U_hist[t])
            for n in range(3):
                assert rel(facs[n][:, c], ref[n]) <= 1e-11, (t, k, n)
            assert rel(lam[c], r.lam_hist[t - 1]) <= 1e-11
            assert abs(err[k] - r.e_hist[t - 1]) <= 1e-11 * r.normT2, (t, k)
            assert abs(fit[k] - r.fit_hist[t - 1]) <= 1e-9


@pytest.mark.parametrize("spec", SPECS[:2] + SPECS[3:4], ids=["61", "62", "64"])
def test_tree_and_fused_paths_agree(spec):
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.05, sampled_mode=nh)
    say("tree vs fused", seed)
    a, b, c = make_ctx(wl), make_ctx(wl), make_ctx(wl)
    b.set_mttkrp_tree(False)
    for x in (a, b, c):
        x.sweep(6)
    for n in range(3):
        ua, la = (to_np(x) for x in a.get_factors(n))
        ub, lb = (to_np(x) for x in b.get_factors(n))
        uc = to_np(c.get_factors(n)[0])
        assert rel(ua, ub) <= 1e-12 and rel(la, lb) <= 1e-12, n
        assert np.array_equal(ua, uc), n              # bitwise repeatable
    ea, eb = to_np(a.get_status()[0]), to_np(b.get_status()[0])
    assert np.allclose(ea, eb, rtol=1e-11, atol=0)
    # switching back and forth between sweeps keeps the iteration consistent
    d = make_ctx(wl)
    for s in range(6):
        d.set_mttkrp_tree(s % 2 == 0)
        d.sweep(1)
    for n in range(3):
        assert rel(to_np(d.get_factors(n)[0]), to_np(a.get_factors(n)[0])) <= 1e-12


def test_tree_with_compaction_and_tolerance_fit():
    wl = synth.random_problem(66, (30, 25, 20), [3] * 8, [-1] + list(range(7)), noise=0.02,
                              true_rank=3)
    say("tree fit + compaction")
    a, b = make_ctx(wl), make_ctx(wl)
    b.set_compaction(False)
    ia, fa, sa = a.fit(300, 1e-9)
    ib, fb, sb = b.fit(300, 1e-9)
    assert np.array_equal(ia, ib) and np.array_equal(fa, fb) and np.array_equal(sa, sb)
    for n in range(3):
        assert np.array_equal(to_np(a.get_factors(n)[0]), to_np(b.get_factors(n)[0]))


def test_tree_refused_where_not_held():
    wl4 = synth.random_problem(67, (6, 5, 4, 3), [2, 2], [-1, 1])
    ctx = make_ctx(wl4)
    with pytest.raises(jk.JkcError):
        ctx.set_mttkrp_tree(True)
    ctx.set_mttkrp_tree(False)
    wl2 = synth.random_problem(68, (9, 8), [2, 2], [-1, 3])
    with pytest.raises(jk.JkcError):
        make_ctx(wl2).set_mttkrp_tree(True)
    wl3 = synth.random_problem(69, (9, 8, 7), [2, 2], [-1, 3])
    with pytest.raises(jk.JkcError):
        make_ctx(wl3, precision=jk.JKC_SPLIT_BF16X3).set_mttkrp_tree(True)
    make_ctx(wl3).set_mttkrp_tree(True)
    # a problem whose cap excludes W: fused MTTKRP on every mode, W refused
    import torch
    T, init = (jk.to_device_tensor(wl3.T),
               [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in wl3.init])
    ctx = jk.JkCals(T, wl3.dims, 0, wl3.ranks, wl3.left_out, init, tree_max_gib=-1)
    assert ctx.describe(3) == ""
    with pytest.raises(jk.JkcError):
        ctx.set_mttkrp_tree(True)
    ref = make_ctx(wl3)
    ref.set_mttkrp_tree(False)
    ctx.sweep(3)
    ref.sweep(3)
    for n in range(3):
        assert np.array_equal(to_np(ctx.get_factors(n)[0]), to_np(ref.get_factors(n)[0]))


def test_describe_names_the_shared_contraction():
    wl = synth.random_problem(70, (12, 10, 8), [2, 3], [-1, 4])
    ctx = make_ctx(wl)
    assert ctx.describe(3).startswith("tree f64 ")
    assert ctx.describe(4) == "" and ctx.describe(-1) == ""
    ctx.set_mttkrp_tree(False)
    assert ctx.describe(3) == ""
    ctx.set_mttkrp_tree(True)
    assert ctx.describe(3).startswith("tree f64 ")
    wl4 = synth.random_problem(71, (6, 5, 4, 3), [2], [-1])
    assert make_ctx(wl4).describe(4) == ""


@pytest.mark.parametrize("spec", SPECS[:3], ids=["61", "62", "63"])
def test_gradient_with_and_without_the_shared_contraction(spec):
    """The all-mode MTTKRP of the loss gradient through W agrees with the
    fused per-mode MTTKRPs (rounding only), for every sampled mode."""
    import torch
    seed, dims, ranks, lo, nh = spec
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, sampled_mode=nh)
    say("tree gradient", seed)
    a, b = make_ctx(wl), make_ctx(wl)
    for c in (a, b):
        c.set_allmode(False)   # the per-mode paths (the one-pass kernel has its own tests)
    b.set_mttkrp_tree(False)
    la = torch.empty(wl.K, dtype=torch.float64, device="cuda")
    lb = torch.empty_like(la)
    a.loss_grad(la)
    b.loss_grad(lb)
    assert np.allclose(to_np(la), to_np(lb), rtol=1e-12, atol=0)
    for n in range(3):
        ga, gb = to_np(a.get_grad(n)), to_np(b.get_grad(n))
        assert rel(ga, gb) <= 1e-12, n
    a.refine(5)
    b.refine(5)
    for n in range(3):
        assert rel(to_np(a.get_factors(n)[0]), to_np(b.get_factors(n)[0])) <= 1e-11, n


def test_tree_every_tiling_matches_oracle():
    """Every compiled tiling computes W when forced on the shared-contraction
    slot (mode N of jk_cals_set_tiling): one sweep matches the oracle's
    per-submodel ALS at 1e-11, on a shape of several tiles with ragged tails
    (W has 37 * 45 = 1665 rows, K = 23)."""
    seed, dims, ranks, lo, nh = SPECS[0]
    wl = synth.random_problem(seed, dims, ranks, lo, noise=0.1, sampled_mode=nh)
    res = oracle.jk_als(np.asarray(wl.T), nh, wl.ranks, wl.left_out, wl.init, 1,
                        record_factors=[1])
    probe = make_ctx(wl)
    checked = 0
    for v in range(probe.num_tilings()):
        ctx = make_ctx(wl)
        try:
            ctx.set_tiling(3, v, 1)
        except jk.JkcError:
            continue                      # the narrow tiling (at most 16 columns)
        desc = ctx.describe(3)
        assert desc.startswith("tree ") and (" v%d " % v) in desc, desc
        say("tree tiling", desc)
        ctx.sweep(1)
        facs = [to_np(ctx.get_factors(n)[0]) for n in range(3)]
        err = to_np(ctx.get_status()[0])
        for k, r in res.items():
            c = cols(wl, k)
            ref = r.padded(r.U_hist[1])
            for n in range(3):
                assert rel(facs[n][:, c], ref[n]) <= 1e-11, (desc, k, n)
            assert abs(err[k] - r.e_hist[0]) <= 1e-11 * r.normT2, (desc, k)
        checked += 1
    assert checked >= probe.num_tilings() - 1


def test_tree_tiling_refusals():
    wl = synth.random_problem(70, (12, 10, 9), [2, 3], [-1, 4])
    ctx = make_ctx(wl)
    v = 0                                 # a matrix-core tiling (not the narrow one)
    ctx.set_tiling(0, v, 1)
    assert variant_geometry(ctx.describe(0)) is not None
    with pytest.raises(jk.JkcError):
        ctx.set_tiling(3, v, 2)           # W takes one K chunk
    with pytest.raises(jk.JkcError):
        ctx.set_tiling(4, v, 1)           # past the shared-contraction slot
    with pytest.raises(jk.JkcError):
        ctx.set_tiling(3, ctx.num_tilings(), 1)
    ctx.set_tiling(3, v, 1)
    wl4 = synth.random_problem(71, (6, 5, 4, 3), [2, 2], [-1, 1])
    with pytest.raises(jk.JkcError):
        make_ctx(wl4).set_tiling(4, v, 1)  # no W for four-way tensors
