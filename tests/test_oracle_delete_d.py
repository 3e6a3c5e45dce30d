"""Pins of the oracle's delete-d jackknife (Sec. 4.1, closing remark: d zero
rows padded and kept zero instead of one; Sec. 4.2: flop ratio I/(I-d)):
explicit slice deletion, the Case I / Case II identities with d rows, the
leave-one-out special case, the flop-ratio bound, and exact recovery."""
import numpy as np

import oracle
import synth


def _rng(seed):
    return np.random.default_rng(9100 + seed)


def test_reduce_tensor_deletes_exactly_the_listed_slices():
    rng = _rng(1)
    T = rng.standard_normal((7, 5, 4))
    P = (1, 4, 6)
    keep = [i for i in range(7) if i not in P]
    ref = np.stack([T[i] for i in keep], axis=0)
    assert np.array_equal(oracle.reduce_tensor(T, 0, P), ref)
    T2 = rng.standard_normal((3, 8, 2))
    assert np.array_equal(oracle.reduce_tensor(T2, 1, [7, 0]), T2[:, 1:7, :])
    assert np.array_equal(oracle.reduce_tensor(T2, 1, [-1, -1]), T2)


def test_case_I_and_II_with_d_zero_rows():
    """Padding d rows with zeros in the sampled mode's factor makes the
    MTTKRP of the full tensor equal the submodel's MTTKRP on the reduced
    tensor: for n != n-hat exactly that (Case II), for n = n-hat on the
    kept rows, the d padded rows being discarded (Case I)."""
    rng = _rng(2)
    dims, R, nh, P = (9, 6, 5), 3, 0, [2, 3, 7]
    T = rng.standard_normal(dims)
    U = [rng.standard_normal((I, R)) for I in dims]
    Ured = list(U)
    Ured[nh] = np.delete(U[nh], P, axis=0)
    Upad = list(U)
    Upad[nh] = U[nh].copy()
    Upad[nh][P] = 0.0
    Tred = np.delete(T, P, axis=nh)
    keep = [i for i in range(dims[nh]) if i not in P]
    for n in range(3):
        full = oracle.mttkrp(T, Upad, n)
        red = oracle.mttkrp(Tred, Ured, n)
        if n == nh:
            assert np.allclose(full[keep], red, rtol=1e-13, atol=1e-13)
        else:
            assert np.allclose(full, red, rtol=1e-13, atol=1e-13)


def test_one_row_lists_equal_leave_one_out():
    wl = synth.random_problem(3, (8, 7, 6), [2, 2, 3], [-1, 3, 7], noise=0.1)
    a = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 3)
    b = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, [[-1], [3], [7]], wl.init, 3)
    for k in range(3):
        for ua, ub in zip(a[k].U, b[k].U):
            assert np.array_equal(ua, ub)
        assert a[k].fit_hist == b[k].fit_hist


def test_padded_reinserts_zero_rows_at_the_left_out_samples():
    wl = synth.random_problem(4, (8, 5, 4), [2], [[1, 6]], noise=0.1)
    r = oracle.jk_als(np.asarray(wl.T), 0, wl.ranks, wl.left_out, wl.init, 2)[0]
    full = r.padded()[0]
    assert full.shape == (8, 2)
    assert np.all(full[[1, 6]] == 0.0)
    assert np.array_equal(np.delete(full, [1, 6], axis=0), r.U[0])


def test_flop_ratio_is_at_most_two():
    """Sec. 4.2: JK-CALS's fused MTTKRP costs I/(I-d) times the flops of
    the separate submodel MTTKRPs, which is at most 2 for d <= I/2."""
    dims, R = (100, 200, 200), 5
    for d in (1, 2, 4, 5, 10, 25, 50):
        ratio = oracle.flops_jk_cals(dims, 0, R, d) / oracle.flops_jk_als(dims, 0, R, d)
        assert abs(ratio - 100 / (100 - d)) < 1e-12
        assert ratio <= 2.0
    assert oracle.flop_ratio(100, 50) == 2.0


def test_delete_d_recovers_a_noise_free_model():
    rng = _rng(5)
    dims, R = (12, 9, 8), 2
    A = [rng.standard_normal((I, R)) for I in dims]
    T = np.einsum("ir,jr,kr->ijk", *A)
    init = [a + 0.05 * rng.standard_normal(a.shape) for a in A]
    res = oracle.jk_als(T, 0, [R], [[0, 5, 11]], init, 60)[0]
    assert res.fit_hist[-1] > 1 - 1e-9
    assert abs(res.normT2 - np.sum(np.delete(T, [0, 5, 11], axis=0) ** 2)) < 1e-10 * res.normT2


def test_delete_d_table_groups():
    ranks, lo = synth.delete_d_table(10, 3, 4, include_full=True)
    assert lo.shape == (4, 3)
    assert list(lo[0]) == [-1, -1, -1]
    assert [list(r) for r in lo[1:]] == [[0, 1, 2], [3, 4, 5], [6, 7, 8]]
    assert list(ranks) == [4] * 4
