"""Pins of the jackknife post-processing oracle (Alg. 2, permutation and scale
adjustment and the standard deviation step) against facts that do not come
from the oracle: planted permutations and signs, exhaustive search over all
permutations, closed-form cosines, the classical jackknife identity for a
sample mean, and the two-submodel closed form."""
import itertools

import numpy as np

import oracle


def _rng(seed):
    return np.random.default_rng(9000 + seed)


def test_congruence_closed_form_angles():
    # unit vectors at known angles in every mode: cos products by hand
    th = [0.3, 1.1, 2.0]
    U = [np.array([[1.0], [0.0]]), np.array([[1.0], [0.0]]), np.array([[2.0], [0.0]])]
    V = [np.array([[np.cos(t)], [np.sin(t)]]) for t in th]
    phi = oracle.congruence(U, V, [0, 1, 2])
    assert abs(phi[0, 0] - np.cos(0.3) * np.cos(1.1) * np.cos(2.0)) < 1e-15
    phi12 = oracle.congruence(U, V, [1, 2])
    assert abs(phi12[0, 0] - np.cos(1.1) * np.cos(2.0)) < 1e-15


def test_match_recovers_planted_permutation_and_signs():
    rng = _rng(1)
    dims, R = (9, 12, 8, 7), 6
    V = [rng.standard_normal((I, R)) for I in dims]
    perm = rng.permutation(R)            # reference component s sits at column perm[s]
    U = [np.empty_like(v) for v in V]
    flips = {}
    for n, v in enumerate(V):
        sg = rng.choice([-1.0, 1.0], size=R)
        sc = rng.uniform(0.5, 3.0, size=R)
        U[n][:, perm] = v * (sg * sc) + 1e-3 * rng.standard_normal(v.shape)
        flips[n] = sg
    for nh in range(4):
        got, signs = oracle.match_components(U, V, nh)
        assert np.array_equal(got, perm)
        assert set(signs) == set(range(4)) - {nh}
        for n, s in signs.items():
            assert np.array_equal(s, flips[n])


def test_match_equals_exhaustive_search():
    rng = _rng(2)
    for trial in range(20):
        R = 3 + trial % 3
        dims = (6, 5, 7)
        U = [rng.standard_normal((I, R)) for I in dims]
        V = [rng.standard_normal((I, R)) for I in dims]
        perm, _ = oracle.match_components(U, V, 0)
        phi = np.abs(oracle.congruence(U, V, [1, 2]))
        best = max(itertools.permutations(range(R)),
                   key=lambda p: sum(phi[p[s], s] for s in range(R)))
        assert abs(sum(phi[perm[s], s] for s in range(R)) -
                   sum(phi[best[s], s] for s in range(R))) < 1e-14


def test_std_zero_for_copies_of_the_reference():
    rng = _rng(3)
    dims, R = (11, 9, 8), 4
    V = [rng.standard_normal((I, R)) for I in dims]
    subs = []
    for k in range(5):
        perm = rng.permutation(R)
        U = []
        for n, v in enumerate(V):
            u = np.empty_like(v)
            u[:, perm] = v * rng.choice([-1.0, 1.0], size=R) * rng.uniform(0.2, 5.0, size=R)
            U.append(u)
        U[0] = rng.standard_normal(U[0].shape)   # the sampled mode is free
        subs.append(U)
    S = oracle.jackknife_std(subs, V, 0)
    assert set(S) == {1, 2}
    for n in (1, 2):
        assert S[n].shape == (dims[n], R)
        assert np.max(S[n]) < 1e-14


def test_std_of_leave_one_out_means_is_the_classical_standard_error():
    """For the leave-one-out means of a sample x_1..x_n, the jackknife
    standard deviation equals the sample standard deviation / sqrt(n)."""
    rng = _rng(4)
    n = 9
    x = rng.uniform(-0.5, 0.5, size=n)
    ref = [np.ones((3, 1)), np.array([[0.1], [0.99]]), np.array([[1.0], [0.0]])]
    subs = []
    for k in range(n):
        m = (x.sum() - x[k]) / (n - 1)
        subs.append([rng.uniform(0.5, 1.0, size=(3, 1)),
                     np.array([[m], [np.sqrt(1.0 - m * m)]]),   # unit norm, positive second entry
                     np.array([[1.0], [0.0]])])
    S = oracle.jackknife_std(subs, ref, 0)
    assert abs(S[1][0, 0] - np.std(x, ddof=1) / np.sqrt(n)) < 1e-14
    assert S[2][0, 0] == 0.0


def test_two_submodels_closed_form():
    rng = _rng(5)
    dims, R = (5, 6, 4), 3
    V = [rng.standard_normal((I, R)) for I in dims]
    A = [v + 0.05 * rng.standard_normal(v.shape) for v in V]
    B = [v + 0.05 * rng.standard_normal(v.shape) for v in V]
    S = oracle.jackknife_std([A, B], V, 0)
    for n in (1, 2):
        a = A[n] / np.linalg.norm(A[n], axis=0)
        b = B[n] / np.linalg.norm(B[n], axis=0)
        a = a * np.sign(np.sum(a * V[n], axis=0))
        b = b * np.sign(np.sum(b * V[n], axis=0))
        assert np.max(np.abs(S[n] - np.abs(a - b) / 2)) < 1e-15


def test_single_submodel_has_zero_deviation():
    rng = _rng(6)
    V = [rng.standard_normal((I, 2)) for I in (4, 5, 6)]
    S = oracle.jackknife_std([[v + 0.1 for v in V]], V, 1)
    assert set(S) == {0, 2} and all(np.max(s) == 0.0 for s in S.values())
