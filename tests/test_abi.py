"""The C ABI without a GPU: the library loads, exports every function the
header declares, the header is valid C, and argument validation rejects bad
input before any device work (all calls here stop at validation)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import paper_2112_03985_amd as jk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(jk.LIB_PATH):
        pytest.fail("libjkcals.so is not built; run python -m paper_2112_03985_amd.build")
    return jk.lib()


def test_exports_every_header_function(L):
    names = jk.header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_header_is_valid_c(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    src = tmp_path / "t.c"
    src.write_text('#include "jk_cals.h"\nint main(void){jkc_problem p; (void)p; return JKC_OK;}\n')
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-c", str(src), "-o", str(tmp_path / "t.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _size(**kw):
    args = dict(dims=[4, 5, 6], sampled_mode=0, ranks=[2, 3], left_out=[-1, 3])
    args.update(kw)
    return jk.jk_cals_workspace_size(**args)


def test_workspace_size_valid_problem():
    s = _size()
    assert s > 4 * 5 * 6 * 8
    assert s % 256 == 0
    assert _size(ranks=[32] * 20, left_out=[-1] * 20) > s


def test_workspace_holds_the_shared_contraction_within_its_cap():
    # 3-way float64: W = [I_0 I_1] x ldc doubles (ldc = 16 here), 256-aligned;
    # an item of no bytes still takes one 256-byte slot
    w = 4 * 5 * 16 * 8
    w_aligned = (w + 255) // 256 * 256
    assert _size() - _size(tree_max_gib=-1) == w_aligned - 256
    assert _size(tree_max_gib=1) == _size()
    # not held for 4-way or split-precision problems
    assert _size(dims=[4, 5, 6, 3]) == _size(dims=[4, 5, 6, 3], tree_max_gib=-1)
    assert _size(precision=1) == _size(precision=1, tree_max_gib=-1)
    # a cap below W's size drops it: 2048 x 2048 x ldc 16 doubles = 512 MiB
    big = dict(dims=[2048, 2048, 2])
    assert _size(**big) - _size(tree_max_gib=-1, **big) == 2048 * 2048 * 16 * 8 - 256
    assert _size(tree_max_gib=64, **big) == _size(**big)


@pytest.mark.parametrize("kw,msg", [
    (dict(dims=[4]), "order"),
    (dict(dims=[2, 2, 2, 2, 2]), "order"),
    (dict(dims=[4, 0, 6]), "dims"),
    (dict(sampled_mode=3), "sampled_mode"),
    (dict(sampled_mode=-1), "sampled_mode"),
    (dict(ranks=[0, 3]), "rank"),
    (dict(ranks=[33, 3]), "rank"),
    (dict(left_out=[-2, 3]), "left_out"),
    (dict(left_out=[-1, 4]), "left_out"),
    (dict(dims=[1, 5, 6], left_out=[-1, 0]), "only sample"),
    (dict(precision=3), "precision"),
    (dict(tensor_dtype=5), "tensor_dtype"),
    (dict(precision=1, copy_tensor=0), "copy_tensor"),
    (dict(copy_tensor=3), "copy_tensor"),
    (dict(dims=[2 ** 15, 2 ** 15, 4], precision=1), "split precision needs"),
])
def test_invalid_problems_rejected(kw, msg):
    with pytest.raises(jk.JkcError) as e:
        _size(**kw)
    assert e.value.status == jk.JKC_EINVAL
    assert msg in str(e.value)


def test_null_arguments_rejected(L):
    assert L.jk_cals_workspace_size(None, None) == jk.JKC_EINVAL
    prob, keep = jk.make_problem([4, 5, 6], 0, [2], [-1])
    size = ctypes.c_size_t(0)
    assert L.jk_cals_workspace_size(ctypes.byref(prob), None) == jk.JKC_EINVAL
    assert L.jk_cals_workspace_size(ctypes.byref(prob), ctypes.byref(size)) == jk.JKC_OK
    assert jk.jk_cals_last_error() == ""
    ctx = ctypes.c_void_p(0)
    ptrs = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    # NULL tensor, NULL init, NULL/misaligned/too-small workspace: all
    # rejected before anything touches the device
    assert L.jk_cals_init(ctypes.byref(prob), None, ptrs, ctypes.c_void_p(0x100000), size, ctypes.byref(ctx)) == jk.JKC_EINVAL
    assert "tensor" in jk.jk_cals_last_error()
    assert L.jk_cals_init(ctypes.byref(prob), ctypes.c_void_p(0x1000), None, ctypes.c_void_p(0x100000), size, ctypes.byref(ctx)) == jk.JKC_EINVAL
    bad = (ctypes.c_void_p * 3)(0x1000, None, 0x1000)
    assert L.jk_cals_init(ctypes.byref(prob), ctypes.c_void_p(0x1000), bad, ctypes.c_void_p(0x100000), size, ctypes.byref(ctx)) == jk.JKC_EINVAL
    assert L.jk_cals_init(ctypes.byref(prob), ctypes.c_void_p(0x1000), ptrs, None, size, ctypes.byref(ctx)) == jk.JKC_EINVAL
    assert L.jk_cals_init(ctypes.byref(prob), ctypes.c_void_p(0x1000), ptrs, ctypes.c_void_p(0x100001), size, ctypes.byref(ctx)) == jk.JKC_EINVAL
    assert "aligned" in jk.jk_cals_last_error()
    assert L.jk_cals_init(ctypes.byref(prob), ctypes.c_void_p(0x1000), ptrs, ctypes.c_void_p(0x100000), ctypes.c_size_t(size.value - 1), ctypes.byref(ctx)) == jk.JKC_ENOMEM
    assert L.jk_cals_init(ctypes.byref(prob), ctypes.c_void_p(0x1000), ptrs, ctypes.c_void_p(0x100000), size, None) == jk.JKC_EINVAL
    assert ctx.value is None


def test_delete_d_validation(L):
    def status(lo, dims=(6, 5, 4), ranks=None):
        lo = np.asarray(lo)
        ranks = ranks or [2] * len(lo)
        prob, keep = jk.make_problem(list(dims), 0, ranks, lo)
        size = ctypes.c_size_t(0)
        return L.jk_cals_workspace_size(ctypes.byref(prob), ctypes.byref(size)), size.value
    ok, size2 = status([[-1, -1], [0, 1], [2, 5]])
    assert ok == jk.JKC_OK and size2 > 0
    assert status([[0, 0], [1, 2]])[0] == jk.JKC_EINVAL          # repeated sample
    assert status([[-1, 3], [1, 2]])[0] == jk.JKC_EINVAL         # -1 mixed with a sample
    assert status([[0, 6], [1, 2]])[0] == jk.JKC_EINVAL          # out of range
    assert status([list(range(6))])[0] == jk.JKC_EINVAL          # leaves nothing
    assert status([[0, 1, 2, 3, 4]])[0] == jk.JKC_OK             # d = I - 1


def test_null_context_rejected(L):
    assert L.jk_cals_mttkrp(None, 0, ctypes.c_void_p(0x1000)) == jk.JKC_EINVAL
    assert L.jk_cals_sweep(None, 1, None) == jk.JKC_EINVAL
    assert L.jk_cals_fit(None, 1, 0.0, None, None, None) == jk.JKC_EINVAL
    assert L.jk_cals_get_factors(None, 0, ctypes.c_void_p(0x1000), None) == jk.JKC_EINVAL
    assert L.jk_cals_set_factors(None, 0, ctypes.c_void_p(0x1000), None) == jk.JKC_EINVAL
    assert L.jk_cals_get_status(None, None, None, None, None) == jk.JKC_EINVAL
    assert L.jk_cals_loss_grad(None, None) == jk.JKC_EINVAL
    assert L.jk_cals_get_grad(None, 0, None, ctypes.c_void_p(0x1000)) == jk.JKC_EINVAL
    assert L.jk_cals_refine(None, 1, None) == jk.JKC_EINVAL
    assert L.jk_cals_tune(None, 1) == jk.JKC_EINVAL
    assert L.jk_cals_set_tiling(None, 0, 0, 1) == jk.JKC_EINVAL
    assert L.jk_cals_set_update_kernel(None, 0) == jk.JKC_EINVAL
    assert L.jk_cals_set_sweep_graph(None, 1) == jk.JKC_EINVAL
    assert L.jk_cals_set_compaction(None, 1) == jk.JKC_EINVAL
    assert L.jk_cals_set_mttkrp_tree(None, 1) == jk.JKC_EINVAL
    assert L.jk_cals_profile(None, 1) == jk.JKC_EINVAL
    assert L.jk_cals_profile_read(None, None, None) == jk.JKC_EINVAL
    stds = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    assert L.jk_cals_jackknife_std(None, 0, 1, 1, stds, None, None) == jk.JKC_EINVAL
    assert L.jk_cals_num_tilings(None) == 0
    assert L.jk_cals_describe(None, 0) == b""
    L.jk_cals_destroy(None)


def test_remove_slice_validation(L):
    prob, keep = jk.make_problem([4, 5, 6], 1, [1], [-1])
    t, o = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert L.jk_cals_remove_slice(ctypes.byref(prob), t, 5, o) == jk.JKC_EINVAL
    assert L.jk_cals_remove_slice(ctypes.byref(prob), t, -1, o) == jk.JKC_EINVAL
    assert L.jk_cals_remove_slice(ctypes.byref(prob), None, 0, o) == jk.JKC_EINVAL
    assert L.jk_cals_remove_slice(None, t, 0, o) == jk.JKC_EINVAL
    prob1, keep1 = jk.make_problem([4, 1, 6], 1, [1], [-1])
    assert L.jk_cals_remove_slice(ctypes.byref(prob1), t, 0, o) == jk.JKC_EINVAL


def test_static_mttkrp_validates_before_any_device_work(L):
    """jk_cals_mttkrp_static checks everything on the host first: a problem
    whose padded factors and output plane exceed the fixed scratch, a split
    precision, a NULL factor and a bad mode are refused (no pointer here is
    a real device address; none is touched)."""
    fake = ctypes.c_void_p(1 << 20)
    ptrs = (ctypes.c_void_p * 3)(1 << 20, 1 << 20, 1 << 20)
    # 5000 x 4000 x 2, C = 1024: one mode-0 output plane is 41 MB and the
    # padded mode-1 factor 33 MB, together above the 64 MiB scratch
    prob, keep = jk.make_problem([5000, 4000, 2], 0, [32] * 32, [-1] * 32)
    assert L.jk_cals_mttkrp_static(ctypes.byref(prob), fake, ptrs, 0, fake) == jk.JKC_EINVAL
    assert "scratch" in jk.jk_cals_last_error()
    prob, keep = jk.make_problem([4, 5, 6], 0, [2, 3], [-1, 3], precision=jk.JKC_SPLIT_BF16X3)
    assert L.jk_cals_mttkrp_static(ctypes.byref(prob), fake, ptrs, 0, fake) == jk.JKC_EUNSUPPORTED
    prob, keep = jk.make_problem([4, 5, 6], 0, [2, 3], [-1, 3])
    assert L.jk_cals_mttkrp_static(ctypes.byref(prob), fake, ptrs, 3, fake) == jk.JKC_EINVAL
    nulls = (ctypes.c_void_p * 3)(1 << 20, None, 1 << 20)
    assert L.jk_cals_mttkrp_static(ctypes.byref(prob), fake, nulls, 0, fake) == jk.JKC_EINVAL
    assert "factors[1]" in jk.jk_cals_last_error()
    assert L.jk_cals_mttkrp_static(ctypes.byref(prob), fake, ptrs, 0, None) == jk.JKC_EINVAL
