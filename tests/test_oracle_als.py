"""Pins of the oracle's CP-ALS (Alg. 1) against mathematics: exact block
least squares, the error identity, monotone descent, exact recovery, fixed
points, R = 1 and N = 2 special cases, Gram symmetry, the pseudoinverse
fallback.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import cp
from synth import dense_from_factors


def _rng(s):
    return np.random.Generator(np.random.PCG64(777 + s))


def _lowrank(shape, R, seed, noise=0.0):
    rng = _rng(seed)
    A = [rng.standard_normal((s, R)) for s in shape]
    T = dense_from_factors(A)
    if noise:
        E = rng.standard_normal(shape)
        T = T + noise * np.linalg.norm(T) / np.linalg.norm(E) * E
    return np.asarray(T), A


def test_update_is_least_squares_pin3():
    """U_n = M_n H_n^{-1} solves min ||T_(n) - U KRP^T||_F (Sec. 3.2)."""
    rng = _rng(1)
    T = rng.standard_normal((6, 7, 8))
    U = [rng.standard_normal((s, 3)) for s in T.shape]
    G = [cp.gram(u) for u in U]
    for n in range(3):
        M = cp.mttkrp(T, U, n)
        H = cp.hadamard_of_grams(G, n)
        Un, fb = cp.solve_normal(M, H)
        assert not fb
        K = cp.krp_excluding(U, n)
        X, *_ = np.linalg.lstsq(K, cp.unfold(T, n).T, rcond=None)
        np.testing.assert_allclose(Un, X.T, rtol=1e-10, atol=1e-12)
        # normal-equation residual is at rounding level
        assert np.linalg.norm(Un @ H - M) <= 1e-12 * np.linalg.norm(M) * np.linalg.cond(H)


@pytest.mark.parametrize("shape,R", [((5, 6, 7), 2), ((3, 4, 5, 6), 3), ((6, 5), 2)])
def test_error_formula_matches_explicit_residual_pin4(shape, R):
    T, _ = _lowrank(shape, 3, seed=2, noise=0.3)
    init = [_rng(3).standard_normal((s, R)) for s in shape]
    for sweeps in (1, 2, 5):
        res = oracle.cp_als(T, init, sweeps)
        explicit = cp.residual_explicit(T, res.U, res.lam)
        assert abs(res.e_hist[-1] - explicit) <= 1e-11 * res.normT2
        fit = 1.0 - np.sqrt(explicit) / np.sqrt(res.normT2)
        assert abs(res.fit_hist[-1] - fit) <= 1e-7


def test_printed_sign_reading_is_rejected_z1():
    """The printed minus sign before the Hadamard-of-Gram term does not give
    the residual; the plus reading does (error step of Alg. 1)."""
    T, _ = _lowrank((5, 6, 7), 3, seed=4, noise=0.2)
    init = [_rng(5).standard_normal((s, 3)) for s in T.shape]
    res = oracle.cp_als(T, init, 4)
    explicit = cp.residual_explicit(T, res.U, res.lam)
    lam, G = res.lam, cp.gram(res.U[-1])
    quad = lam @ ((res.H_last * G) @ lam)
    inner = np.sum(lam[None, :] * res.U[-1] * res.M_last)
    printed = res.normT2 - quad - 2.0 * inner
    assert abs(printed - explicit) > 0.1 * res.normT2
    assert abs(res.normT2 + quad - 2.0 * inner - explicit) <= 1e-11 * res.normT2


def test_monotone_descent_pin6():
    T, _ = _lowrank((6, 7, 8), 4, seed=6, noise=0.1)
    init = [_rng(7).standard_normal((s, 3)) for s in T.shape]
    res = oracle.cp_als(T, init, 40)
    e = np.array(res.e_hist)
    assert np.all(e[1:] <= e[:-1] + 1e-12 * res.normT2)


def test_monotone_within_sweep_pin6():
    """Every single mode update is an exact block minimiser, so the explicit
    residual never increases from one update to the next."""
    T, _ = _lowrank((5, 6, 7), 3, seed=8, noise=0.2)
    U = [_rng(9).standard_normal((s, 3)) for s in T.shape]
    prev = cp.residual_explicit(T, U)
    for _ in range(5):
        for n in range(3):
            G = [cp.gram(u) for u in U]
            Un, _ = cp.solve_normal(cp.mttkrp(T, U, n), cp.hadamard_of_grams(G, n))
            U[n] = Un
            cur = cp.residual_explicit(T, U)
            assert cur <= prev * (1 + 1e-12) + 1e-20
            prev = cur


def test_exact_recovery_noise_free_pin7():
    T, _ = _lowrank((8, 9, 10), 3, seed=10)
    init = [_rng(11).standard_normal((s, 3)) for s in T.shape]
    res = oracle.cp_als(T, init, 400)
    explicit = cp.residual_explicit(T, res.U, res.lam)
    fit = 1.0 - np.sqrt(explicit / res.normT2)
    assert fit >= 1.0 - 1e-10


def test_fixed_point_at_truth_pin8():
    T, A = _lowrank((6, 7, 8), 3, seed=12)
    res = oracle.cp_als(T, A, 3)
    for n in range(2):
        ref = A[n] / np.linalg.norm(A[n], axis=0)
        np.testing.assert_allclose(res.U[n], ref, rtol=1e-11, atol=1e-12)
    explicit = cp.residual_explicit(T, res.U, res.lam)
    assert explicit <= 1e-22 * res.normT2
    assert res.fit_hist[-1] >= 1.0 - 1e-7


def test_rank_one_is_power_iteration_pin9():
    """R = 1: each update is T contracted with the other vectors, normalised
    (higher-order power iteration)."""
    rng = _rng(13)
    T = rng.standard_normal((5, 6, 7))
    init = [rng.standard_normal((s, 1)) for s in T.shape]
    res = oracle.cp_als(T, init, 25)
    x, y, z = (u[:, 0].copy() for u in init)
    for _ in range(25):
        x = np.einsum("ijk,j,k->i", T, y, z); x /= np.linalg.norm(x)
        y = np.einsum("ijk,i,k->j", T, x, z); y /= np.linalg.norm(y)
        zz = np.einsum("ijk,i,j->k", T, x, y); lam = np.linalg.norm(zz); z = zz / lam
    np.testing.assert_allclose(res.U[0][:, 0], x, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(res.U[1][:, 0], y, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(res.U[2][:, 0], z, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(res.lam[0], lam, rtol=1e-12)


def test_matrix_case_reaches_eckart_young_pin9():
    """N = 2: converged ALS gives the best rank-R approximation, whose error
    is the tail of the singular values."""
    rng = _rng(14)
    Q1, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    Q2, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    s = np.array([10, 8, 6, 1.0, 0.5, 0.4, 0.3, 0.2, 0.1, 0.05])
    T = (Q1[:, :10] * s) @ Q2.T
    init = [rng.standard_normal((12, 3)), rng.standard_normal((10, 3))]
    res = oracle.cp_als(T, init, 300)
    target = 1.0 - np.sqrt(np.sum(s[3:] ** 2)) / np.linalg.norm(s)
    assert abs(res.fit_hist[-1] - target) <= 1e-9
    explicit = cp.residual_explicit(T, res.U, res.lam)
    assert abs(explicit - np.sum(s[3:] ** 2)) <= 1e-10 * np.sum(s ** 2)


def test_gram_exactly_symmetric_pin10():
    rng = _rng(15)
    for rows, R in ((1000, 7), (333, 12), (50, 32)):
        G = cp.gram(rng.standard_normal((rows, R)))
        assert np.array_equal(G, G.T)


def test_pinv_fallback_on_singular_H():
    """Duplicated columns make H singular: the update falls back to the
    eigen pseudoinverse and agrees with the minimum-norm least-squares
    solution."""
    rng = _rng(16)
    T = rng.standard_normal((5, 6, 7))
    U = [rng.standard_normal((s, 3)) for s in T.shape]
    for n in (1, 2):
        U[n][:, 2] = U[n][:, 1]
    G = [cp.gram(u) for u in U]
    M = cp.mttkrp(T, U, 0)
    H = cp.hadamard_of_grams(G, 0)
    Un, fb = cp.solve_normal(M, H)
    assert fb
    ref = M @ np.linalg.pinv(H, rcond=1e-12)
    np.testing.assert_allclose(Un, ref, rtol=1e-8, atol=1e-10)


def test_normalisation_keeps_model():
    rng = _rng(17)
    U = rng.standard_normal((9, 4))
    U[:, 2] = 0.0
    V, lam = cp.normalise_columns(U)
    np.testing.assert_allclose(V * lam[None, :], U, rtol=1e-15, atol=0)
    assert lam[2] == 0.0 and np.all(V[:, 2] == 0.0)
    np.testing.assert_allclose(np.linalg.norm(V[:, [0, 1, 3]], axis=0), 1.0, rtol=1e-15)


def test_tolerance_stops_early():
    T, _ = _lowrank((6, 7, 8), 2, seed=18, noise=0.05)
    init = [_rng(19).standard_normal((s, 2)) for s in T.shape]
    res = oracle.cp_als(T, init, 1000, tol=1e-6)
    assert res.converged and res.iters < 1000
    assert abs(res.fit_hist[-1] - res.fit_hist[-2]) < 1e-6
