"""Pins of the oracle's unfolding, Khatri-Rao product and MTTKRP against the
definitions (Sec. 3.1, Eq. (1), Eq. (3)) and the Case I / Case II identities
of Sec. 4.1.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import cp
from synth import dense_from_factors


def _rng(s):
    return np.random.Generator(np.random.PCG64(1234 + s))


SHAPES = [(3, 4, 5), (2, 3, 4, 5), (4, 3), (1, 3, 2)]


@pytest.mark.parametrize("shape", SHAPES)
def test_unfold_index_map_eq3(shape):
    """Element (i_1..i_N) sits at row i_n, column j of Eq. (3)."""
    T = _rng(0).standard_normal(shape)
    for n in range(len(shape)):
        Tn = cp.unfold(T, n)
        for idx in itertools.product(*[range(s) for s in shape]):
            j, stride = 0, 1
            for k in range(len(shape)):
                if k == n:
                    continue
                j += idx[k] * stride
                stride *= shape[k]
            assert Tn[idx[n], j] == T[idx]


def test_khatri_rao_columnwise_kronecker():
    A = _rng(1).standard_normal((3, 2))
    B = _rng(2).standard_normal((4, 2))
    C = _rng(3).standard_normal((2, 2))
    K = cp.khatri_rao([A, B, C])
    for r in range(2):
        np.testing.assert_array_equal(K[:, r], np.kron(np.kron(A[:, r], B[:, r]), C[:, r]))


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 4, 5), (5, 2)])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_mttkrp_matches_bruteforce_pin1(shape, R):
    rng = _rng(10 + R)
    T = rng.standard_normal(shape)
    U = [rng.standard_normal((s, R)) for s in shape]
    for n in range(len(shape)):
        M = cp.mttkrp(T, U, n)
        B = cp.mttkrp_bruteforce(T, U, n)
        assert np.linalg.norm(M - B) <= 1e-14 * max(np.linalg.norm(B), 1.0)


def test_krp_gram_identity_pin2():
    rng = _rng(20)
    U = [rng.standard_normal((s, 3)) for s in (3, 4, 5, 2)]
    for n in range(4):
        K = cp.krp_excluding(U, n)
        G = [u.T @ u for u in U]
        H = cp.hadamard_of_grams(G, n)
        np.testing.assert_allclose(K.T @ K, H, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape,nhat", [((5, 4, 3), 0), ((4, 5, 3), 1), ((3, 4, 5, 2), 2)])
def test_case_I_and_II_pin5(shape, nhat):
    """Sec. 4.1: the MTTKRP of the reduced tensor equals the MTTKRP of the
    full tensor with a zero row inserted at p in the sampled mode's factor
    (Case II, n != n-hat) and with row p discarded (Case I, n = n-hat)."""
    rng = _rng(30)
    T = rng.standard_normal(shape)
    R = 2
    for p in range(shape[nhat]):
        Tr = oracle.reduce_tensor(T, nhat, p)
        Ur = [rng.standard_normal((s, R)) for s in Tr.shape]
        Upad = [u.copy() for u in Ur]
        Upad[nhat] = np.insert(Ur[nhat], p, 0.0, axis=0)
        for n in range(len(shape)):
            Mr = cp.mttkrp_bruteforce(Tr, Ur, n)
            Mf = cp.mttkrp(T, Upad, n)
            if n == nhat:
                Mf = np.delete(Mf, p, axis=0)
            assert np.linalg.norm(Mf - Mr) <= 1e-14 * max(np.linalg.norm(Mr), 1.0)


def test_case_II_slice_term_pin14():
    """With row p restored in the sampled factor, the full MTTKRP exceeds the
    reduced one by exactly the contribution of slice p (sum over the slice
    only), computed here by brute force on that slice."""
    rng = _rng(40)
    shape, nhat, p, R = (4, 3, 5), 0, 2, 2
    T = rng.standard_normal(shape)
    U = [rng.standard_normal((s, R)) for s in shape]
    Uz = [u.copy() for u in U]
    Uz[nhat][p, :] = 0.0
    S = np.zeros_like(T)
    S[p] = T[p]
    for n in (1, 2):
        lhs = cp.mttkrp(T, U, n) - cp.mttkrp(T, Uz, n)
        rhs = cp.mttkrp_bruteforce(S, U, n)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)


def test_mttkrp_rank_one_closed_form():
    """For T = a o b o c the mode-1 MTTKRP with factors (.., u, v) is
    a * (b.u) * (c.v)."""
    rng = _rng(50)
    a, b, c = rng.standard_normal(4), rng.standard_normal(5), rng.standard_normal(6)
    T = dense_from_factors([a[:, None], b[:, None], c[:, None]])
    u, v, w = rng.standard_normal((5, 1)), rng.standard_normal((6, 1)), rng.standard_normal((4, 1))
    M0 = cp.mttkrp(T, [w, u, v], 0)
    np.testing.assert_allclose(M0[:, 0], a * (b @ u[:, 0]) * (c @ v[:, 0]), rtol=1e-13)
    M2 = cp.mttkrp(T, [w, u, v], 2)
    np.testing.assert_allclose(M2[:, 0], c * (a @ w[:, 0]) * (b @ u[:, 0]), rtol=1e-13)
