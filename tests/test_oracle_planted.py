"""Planted mistakes: each test plants one plausible bug in the oracle (on the
CPU, through monkeypatching) and checks that at least one pin catches it.
This is what makes the pins worth trusting."""
import numpy as np
import pytest

import oracle
from oracle import cp, jackknife
import test_oracle_als as A
import test_oracle_jackknife as J
import test_oracle_mttkrp as Mk


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_reversed_krp_order_is_caught(monkeypatch):
    def bad(U, n):
        return cp.khatri_rao([U[m] for m in range(len(U)) if m != n])
    monkeypatch.setattr(cp, "krp_excluding", bad)
    _fails(Mk.test_mttkrp_matches_bruteforce_pin1, (3, 4, 5), 2)


def test_c_order_unfolding_is_caught(monkeypatch):
    def bad(T, n):
        return np.reshape(np.moveaxis(np.asarray(T, float), n, 0), (T.shape[n], -1), order="C")
    monkeypatch.setattr(cp, "unfold", bad)
    _fails(Mk.test_unfold_index_map_eq3, (3, 4, 5))
    _fails(Mk.test_mttkrp_matches_bruteforce_pin1, (3, 4, 5), 2)


def test_hadamard_including_own_gram_is_caught(monkeypatch):
    def bad(G, n):
        H = G[0].copy()
        for Gi in G[1:]:
            H = H * Gi
        return H
    monkeypatch.setattr(cp, "hadamard_of_grams", bad)
    _fails(A.test_update_is_least_squares_pin3)


def test_transposed_solve_is_caught(monkeypatch):
    orig = cp.solve_normal

    def bad(M, H):
        U, fb = orig(M, H)
        # solving H U^T = M^T with a non-symmetric perturbation of H
        return U @ np.triu(np.ones_like(H)) / H.shape[0] + 0 * U, fb
    monkeypatch.setattr(cp, "solve_normal", bad)
    _fails(A.test_update_is_least_squares_pin3)


def test_printed_error_sign_is_caught(monkeypatch):
    def bad(normT2, H, G, U, M, lam):
        return normT2 - float(lam @ ((H * G) @ lam)) - 2.0 * float(np.sum(lam[None, :] * U * M))
    monkeypatch.setattr(cp, "error_fast", bad)
    _fails(A.test_error_formula_matches_explicit_residual_pin4, (5, 6, 7), 2)


def test_missing_lambda_in_error_is_caught(monkeypatch):
    def bad(normT2, H, G, U, M, lam):
        return normT2 + float(np.sum(H * G)) - 2.0 * float(np.sum(U * M))
    monkeypatch.setattr(cp, "error_fast", bad)
    _fails(A.test_error_formula_matches_explicit_residual_pin4, (5, 6, 7), 2)


def test_squared_lambda_is_caught(monkeypatch):
    orig = cp.normalise_columns

    def bad(U):
        V, lam = orig(U)
        return V, lam * lam
    monkeypatch.setattr(cp, "normalise_columns", bad)
    _fails(A.test_fixed_point_at_truth_pin8)
    _fails(A.test_rank_one_is_power_iteration_pin9)


def test_wrong_row_removed_is_caught(monkeypatch):
    def bad(U_init, p):
        if p < 0:
            return np.array(U_init, float)
        return np.delete(np.asarray(U_init, float), (p + 1) % U_init.shape[0], axis=0)
    monkeypatch.setattr(jackknife, "reduce_init", bad)
    _fails(J.test_submodel_matches_zero_row_full_tensor_iteration, 1)


def test_wrong_slice_removed_is_caught(monkeypatch):
    def bad(T, mode, p):
        T = np.asarray(T, float)
        return T if p < 0 else np.delete(T, (p + 1) % T.shape[mode], axis=mode)
    monkeypatch.setattr(jackknife, "reduce_tensor", bad)
    _fails(J.test_submodel_matches_zero_row_full_tensor_iteration, 0)


def test_gradient_sign_is_caught(monkeypatch):
    orig = jackknife.grad

    def bad(T, U):
        return [-g for g in orig(T, U)]
    monkeypatch.setattr(jackknife, "grad", bad)
    monkeypatch.setattr(oracle, "grad", bad)
    _fails(J.test_gradient_matches_central_differences_pin12)


def test_gradient_missing_hadamard_is_caught(monkeypatch):
    def bad(T, U):
        return [U[n] - cp.mttkrp(T, U, n) for n in range(len(U))]
    monkeypatch.setattr(jackknife, "grad", bad)
    monkeypatch.setattr(oracle, "grad", bad)
    _fails(J.test_gradient_matches_central_differences_pin12)


# --- gradient refinement (reading of the all-at-once CP step rule) ---------

import test_oracle_refine as Rf


def _refine_with(eta_of, sequential=False, refresh=False):
    """A refinement loop with one planted change (step norm, per-mode
    sequential updates, or the step recomputed every iteration)."""
    def bad(T, U0, steps):
        U = [np.array(u, dtype=np.float64) for u in U0]
        eta = eta_of(U)
        for _ in range(steps):
            if refresh:
                eta = eta_of(U)
            if sequential:
                for n in range(len(U)):
                    U[n] = U[n] - eta * jackknife.grad(T, U)[n]
            else:
                g = jackknife.grad(T, U)
                U = [u - eta * gn for u, gn in zip(U, g)]
        return U
    return bad


def _eta_frobenius(U):
    G = [u.T @ u for u in U]
    return 1.0 / sum(np.linalg.norm(cp.hadamard_of_grams(G, n)) for n in range(len(U)))


def _eta_spectral(U):
    G = [u.T @ u for u in U]
    return 1.0 / sum(np.linalg.norm(cp.hadamard_of_grams(G, n), 2) for n in range(len(U)))


def test_refine_sanity_of_the_harness(monkeypatch):
    """The rewritten loop with nothing planted passes the pins (so the three
    planted variants below fail for their plant, not for the harness)."""
    monkeypatch.setattr(oracle, "gd_refine", _refine_with(_eta_frobenius))
    Rf.test_one_step_is_simultaneous_descent_with_frobenius_step(*Rf.CASES[0])
    Rf.test_step_size_is_frozen_at_the_first_step(*Rf.CASES[0])


def test_refine_spectral_norm_step_is_caught(monkeypatch):
    monkeypatch.setattr(oracle, "gd_refine", _refine_with(_eta_spectral))
    _fails(Rf.test_one_step_is_simultaneous_descent_with_frobenius_step, *Rf.CASES[0])


def test_refine_sequential_modes_is_caught(monkeypatch):
    monkeypatch.setattr(oracle, "gd_refine", _refine_with(_eta_frobenius, sequential=True))
    _fails(Rf.test_one_step_is_simultaneous_descent_with_frobenius_step, *Rf.CASES[0])


def test_refine_recomputed_step_is_caught(monkeypatch):
    monkeypatch.setattr(oracle, "gd_refine", _refine_with(_eta_frobenius, refresh=True))
    Rf.test_one_step_is_simultaneous_descent_with_frobenius_step(*Rf.CASES[0])
    _fails(Rf.test_step_size_is_frozen_at_the_first_step, *Rf.CASES[0])
