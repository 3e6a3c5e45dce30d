"""Pins of the oracle's jackknife loop (Alg. 2), the CP loss gradient and the
flop counts of Sec. 4.2.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import cp
from synth import dense_from_factors, random_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.Generator(np.random.PCG64(4242 + s))


def test_reduce_tensor_and_init():
    T = np.arange(2 * 3 * 4, dtype=float).reshape(2, 3, 4)
    np.testing.assert_array_equal(oracle.reduce_tensor(T, 1, 1), T[:, [0, 2], :])
    assert oracle.reduce_tensor(T, 0, -1) is not None
    np.testing.assert_array_equal(oracle.reduce_tensor(T, 0, -1), T)
    U = np.arange(12.0).reshape(4, 3)
    np.testing.assert_array_equal(oracle.reduce_init(U, 2), U[[0, 1, 3]])


def test_full_model_equals_plain_als():
    wl = random_problem(1, (6, 7, 8), ranks=[3, 2], left_out=[-1, 4], noise=0.1)
    res = oracle.jk_als(wl.T, 0, wl.ranks, wl.left_out, wl.init, 5)
    ref = oracle.cp_als(wl.T, [u[:, :3] for u in wl.init], 5)
    for a, b in zip(res[0].U, ref.U):
        np.testing.assert_array_equal(a, b)


def test_submodel_fits_its_reduced_tensor_exactly():
    """On noise-free low-rank data each leave-one-out submodel recovers its
    own reduced tensor, and its padded factors reproduce T off slice p
    (explicit residual, not the fast formula)."""
    rng = _rng(2)
    shape = (7, 8, 9)
    A = [rng.standard_normal((s, 2)) for s in shape]
    T = np.asarray(dense_from_factors(A))
    K = 3
    ranks = np.full(K, 2, np.int32)
    lo = np.array([0, 3, 6], np.int32)
    init = [np.concatenate([a + 0.3 * rng.standard_normal(a.shape)] * K, axis=1) for a in A]
    res = oracle.jk_als(T, 0, ranks, lo, init, 300)
    for k, r in res.items():
        p = int(lo[k])
        Tk = oracle.reduce_tensor(T, 0, p)
        fit = 1 - np.sqrt(cp.residual_explicit(Tk, r.U, r.lam) / np.sum(Tk ** 2))
        assert fit >= 1 - 1e-10
        Up = r.padded()
        assert np.all(Up[0][p] == 0.0)
        R = cp.reconstruct(Up, r.lam)
        assert np.all(R[p] == 0.0)
        keep = [i for i in range(shape[0]) if i != p]
        np.testing.assert_allclose(R[keep], T[keep], atol=1e-9 * np.abs(T).max())


@pytest.mark.parametrize("nhat", [0, 1, 2])
def test_submodel_matches_zero_row_full_tensor_iteration(nhat):
    """Two ALS sweeps of a submodel (reduced tensor) equal two sweeps driven
    by the full tensor with the zero-padded factor and the left-out output
    row zeroed, i.e. the Case I / Case II route of Alg. 3."""
    wl = random_problem(3, (5, 6, 7), ranks=[2], left_out=[3], noise=0.2, sampled_mode=nhat)
    p = 3
    r = oracle.jk_als(wl.T, nhat, wl.ranks, wl.left_out, wl.init, 2)[0]
    U = [u.copy() for u in wl.init]
    U[nhat][p] = 0.0
    T = np.asarray(wl.T)
    G = [cp.gram(u) for u in U]
    for _ in range(2):
        for n in range(3):
            M = cp.mttkrp(T, U, n)
            if n == nhat:
                M[p] = 0.0
            Un, _ = cp.solve_normal(M, cp.hadamard_of_grams(G, n))
            U[n], lam = cp.normalise_columns(Un)
            G[n] = cp.gram(U[n])
    for a, b in zip(r.padded(), U):
        np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-13)


def test_flop_counts_golden_pin11():
    with open(os.path.join(GOLDEN, "flops_sec4_2.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        a = oracle.flops_jk_als(c["dims"], c["sampled_mode"], c["R"], c["d"])
        b = oracle.flops_jk_cals(c["dims"], c["sampled_mode"], c["R"], c["d"])
        assert a == pytest.approx(c["jk_als_flops"], rel=1e-15)
        assert b == pytest.approx(c["jk_cals_flops"], rel=1e-15)
        assert b / a == pytest.approx(c["ratio"], rel=1e-15)
        assert oracle.flop_ratio(c["dims"][c["sampled_mode"]], c["d"]) == pytest.approx(c["ratio"])
        assert b / a <= 2.0


def test_gradient_matches_central_differences_pin12():
    """f is quadratic in every single entry, so a central difference at
    h = 1e-3 is exact up to rounding."""
    rng = _rng(4)
    T = rng.standard_normal((4, 5, 3))
    U = [rng.standard_normal((s, 2)) for s in T.shape]
    g = oracle.grad(T, U)
    fd = oracle.fd_grad(T, U, h=1e-3)
    f = oracle.loss_and_grad(T, U)[0]
    for (n, i, r), v in fd.items():
        assert abs(v - g[n][i, r]) <= 1e-9 * max(1.0, f)


def test_gradient_vanishes_after_exact_update_pin12():
    rng = _rng(5)
    T = rng.standard_normal((5, 6, 7))
    U = [rng.standard_normal((s, 3)) for s in T.shape]
    G = [cp.gram(u) for u in U]
    U[1], _ = cp.solve_normal(cp.mttkrp(T, U, 1), cp.hadamard_of_grams(G, 1))
    _, g = oracle.loss_and_grad(T, U)
    assert np.linalg.norm(g[1]) <= 1e-11 * np.linalg.norm(cp.mttkrp(T, U, 1))
    assert np.linalg.norm(g[0]) > 1e-3


def test_gradient_descent_decreases_loss():
    rng = _rng(6)
    T = rng.standard_normal((5, 6, 7))
    U = [rng.standard_normal((s, 2)) for s in T.shape]
    f0 = oracle.loss_and_grad(T, U)[0]
    U1 = oracle.gd_refine(T, U, 20)
    assert oracle.loss_and_grad(T, U1)[0] < f0
