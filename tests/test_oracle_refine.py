"""Pins of the oracle's gradient-refinement rule (a reading: the paper cites
gradient-based all-at-once CP in Sec. 2 but states no rule).  The rule read
here: every factor of one model moves at once by the step
eta = 1 / sum_n ||H_n||_F, H_n = (KRP excluding n)^T (KRP excluding n),
with eta taken from the factors before the first step and kept fixed.

Nothing below calls the oracle's loss, gradient, Khatri-Rao or Gram code:
the loss is the dense reconstruction written out with einsum, the gradient
is its central difference (exact up to rounding, because the loss is
quadratic in every single entry), and H_n is formed from an explicitly
built Khatri-Rao matrix.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle


def _rng(s):
    return np.random.Generator(np.random.PCG64(7100 + s))


def _reconstruct(U):
    """Dense [[U_1, ..., U_N]] from the defining sum over rank-one terms."""
    R = U[0].shape[1]
    X = np.zeros(tuple(u.shape[0] for u in U))
    for r in range(R):
        t = U[0][:, r]
        for u in U[1:]:
            t = np.multiply.outer(t, u[:, r])
        X += t
    return X


def _loss(T, U):
    D = T - _reconstruct(U)
    return 0.5 * float(np.sum(D * D))


def _fd_gradient(T, U, h=1e-3):
    """Central differences of the written-out loss for every entry."""
    U = [np.array(u, dtype=np.float64) for u in U]
    g = [np.zeros_like(u) for u in U]
    for n, u in enumerate(U):
        for i, r in itertools.product(range(u.shape[0]), range(u.shape[1])):
            keep = u[i, r]
            u[i, r] = keep + h
            fp = _loss(T, U)
            u[i, r] = keep - h
            fm = _loss(T, U)
            u[i, r] = keep
            g[n][i, r] = (fp - fm) / (2.0 * h)
    return g


def _explicit_krp(mats):
    """Rows indexed by every combination of the listed matrices' rows (any
    fixed order: only Z^T Z is used), column r the product of column r."""
    R = mats[0].shape[1]
    rows = []
    for idx in itertools.product(*[range(m.shape[0]) for m in mats]):
        row = np.ones(R)
        for m, i in zip(mats, idx):
            row = row * m[i]
        rows.append(row)
    return np.array(rows)


def _step(U):
    """eta = 1 / sum_n ||Z_n^T Z_n||_F with Z_n the Khatri-Rao product of
    every factor but U_n."""
    s = 0.0
    for n in range(len(U)):
        Z = _explicit_krp([U[m] for m in range(len(U)) if m != n])
        s += np.linalg.norm(Z.T @ Z, "fro")
    return 1.0 / s


def _problem(seed, dims, R):
    rng = _rng(seed)
    T = rng.standard_normal(dims)
    U = [0.7 * rng.standard_normal((d, R)) for d in dims]
    return T, U


CASES = [(0, (4, 3, 5), 2), (1, (3, 4, 2, 3), 2), (2, (5, 4, 3), 3)]


@pytest.mark.parametrize("seed,dims,R", CASES)
def test_one_step_is_simultaneous_descent_with_frobenius_step(seed, dims, R):
    T, U = _problem(seed, dims, R)
    eta = _step(U)
    g = _fd_gradient(T, U)
    want = [u - eta * gn for u, gn in zip(U, g)]
    got = oracle.gd_refine(T, U, 1)
    scale = max(np.linalg.norm(u) for u in U)
    for a, b in zip(got, want):
        assert np.linalg.norm(a - b) <= 1e-9 * scale


@pytest.mark.parametrize("seed,dims,R", CASES)
def test_step_size_is_frozen_at_the_first_step(seed, dims, R):
    """Three steps: every step uses eta from the starting factors."""
    T, U = _problem(seed, dims, R)
    eta0 = _step(U)
    want = [np.array(u) for u in U]
    for _ in range(3):
        g = _fd_gradient(T, want)
        want = [u - eta0 * gn for u, gn in zip(want, g)]
    got = oracle.gd_refine(T, U, 3)
    # the pin is only sharp if eta would have changed along the way
    assert abs(_step(want) - eta0) > 1e-6 * eta0
    scale = max(np.linalg.norm(u) for u in U)
    for a, b in zip(got, want):
        assert np.linalg.norm(a - b) <= 1e-9 * scale


def test_zero_steps_return_the_input():
    T, U = _problem(3, (3, 4, 5), 2)
    got = oracle.gd_refine(T, U, 0)
    for a, b in zip(got, U):
        np.testing.assert_array_equal(a, b)


def test_fixed_point_at_an_exact_decomposition():
    """At factors that reproduce T exactly the gradient is zero, so the
    refinement leaves them in place."""
    rng = _rng(4)
    U = [rng.standard_normal((d, 2)) for d in (4, 5, 3)]
    T = _reconstruct(U)
    got = oracle.gd_refine(T, U, 5)
    for a, b in zip(got, U):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
