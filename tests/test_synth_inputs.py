"""The seeded workload generators: shapes, reproducibility, noise level,
model tables, and an oracle run of the small configuration."""
import numpy as np

import oracle
import synth


def test_config1_shapes_and_table():
    wl = synth.config1()
    assert wl.dims == (20, 30, 40) and wl.T.flags.f_contiguous
    assert wl.K == 21 and wl.C == 63
    assert wl.left_out[0] == -1 and list(wl.left_out[1:]) == list(range(20))
    assert [u.shape for u in wl.init] == [(20, 63), (30, 63), (40, 63)]
    # one shared parent: every model's block is the same
    for u in wl.init:
        np.testing.assert_array_equal(u[:, :3], u[:, 60:63])


def test_generators_are_reproducible():
    a, b = synth.config1(), synth.config1()
    np.testing.assert_array_equal(a.T, b.T)
    for x, y in zip(a.init, b.init):
        np.testing.assert_array_equal(x, y)


def test_noise_level_is_relative_frobenius():
    rng = np.random.Generator(np.random.PCG64(5))
    T0 = np.asfortranarray(rng.standard_normal((4, 5, 6)))
    T = synth.add_noise(T0, rng, 0.02)
    assert abs(np.linalg.norm(T - T0) / np.linalg.norm(T0) - 0.02) < 1e-12


def test_config2_structure_small():
    wl = synth.config2(dims=(10, 40, 40))
    assert wl.K == 10 and wl.C == 50
    A = wl.truth
    assert np.all(A[0] >= 0) and np.all(A[0] <= 1)
    assert np.all(A[1] > 0) and np.all(A[2] > 0)


def test_config3_table_small():
    wl = synth.config3(dims=(6, 5, 4), rank_max=3, inits_per_rank=2)
    assert wl.K == 6 * 3 * 2
    assert wl.C == 6 * 2 * (1 + 2 + 3)
    assert wl.init[0].shape == (6, wl.C)


def test_config1_oracle_fits_well():
    wl = synth.config1()
    res = oracle.jk_als(wl.T, 0, wl.ranks, wl.left_out, wl.init, 50, models=[0, 1, 20])
    for r in res.values():
        assert r.fit_hist[-1] > 0.98
