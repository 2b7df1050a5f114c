"""Pins of the synthetic workload generator (input side, shared by both paths)."""
import numpy as np
import pytest

from workloads import (tiny, small_fp64, medium_fp64, batch_instance, full_nnz, basis,
                       pair_uniform, WaveletSpec, make_matrix)


def test_index_model_counts():
    for G in range(1, 6):
        lev, kx, ky = basis(G)
        assert lev.size == 4 ** G
        # level j occupies [4^j, 4^(j+1)) (index 0, the scaling function, is level 0)
        for j in range(G):
            assert np.all(lev[4 ** j:4 ** (j + 1)] == j)
        assert np.all(kx < (1 << lev)) and np.all(ky < (1 << lev))


@pytest.mark.parametrize("G,a,expect", [(3, 1.5, 3556), (4, 1.5, 32488), (6, 1.5, 1254448)])
def test_exact_pattern_counts(G, a, expect):
    """Full symmetric nnz of the a * 2^-min(j,j') cut-off rule (exact integer distances)."""
    m = tiny(G, a).matrix() if G < 6 else small_fp64().matrix()
    assert full_nnz(m) == expect


def test_small_config_lower_count():
    m = small_fp64().matrix()
    assert m["n"] == 4096 and m["colptr"][-1] == 629272


def test_csc_shape_and_dominance():
    m = tiny(4, 1.7).matrix()
    n, cp, ri, v = m["n"], m["colptr"], m["rowind"], m["values"]
    A = np.zeros((n, n))
    for j in range(n):
        rows = ri[cp[j]:cp[j + 1]]
        assert rows[0] == j and np.all(np.diff(rows) > 0)
        A[rows, j] = v[cp[j]:cp[j + 1]]
    A = A + np.tril(A, -1).T
    off = np.abs(A).sum(1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) > off)           # strictly diagonally dominant => SPD
    assert np.linalg.eigvalsh(A).min() > 0


def test_dense_when_cutoff_covers_domain():
    """N = 16: every support pair is within 1.2 * 2^-min(j,j'), so the matrix is dense."""
    assert full_nnz(tiny(2, 1.2).matrix()) == 256


def test_determinism_and_pair_symmetry():
    a = tiny(4, 1.5, seed=3).matrix()
    b = tiny(4, 1.5, seed=3).matrix()
    assert np.array_equal(a["values"], b["values"]) and np.array_equal(a["rowind"], b["rowind"])
    i = np.array([3, 10, 77]); j = np.array([10, 3, 5])
    u1 = pair_uniform(9, i, j); u2 = pair_uniform(9, j, i)
    assert np.array_equal(u1, u2) and np.all(np.abs(u1) < 1)


def test_splitmix64_reference_values():
    """SplitMix64 from state 0 yields 0xE220A8397B1DCDAF (first output of the published generator)."""
    from workloads import splitmix64
    assert int(splitmix64(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_batch_instance_ranges():
    for i in range(16):
        w = batch_instance(i)
        assert w.spec.grid_exp in (5, 6, 7)
        assert 0.1 <= w.spec.ell <= 0.5 and 1.2 <= w.spec.a <= 2.0 and w.spec.s in (0.25, 0.5, 0.75)


def test_heat_spot_forcing_follows_the_circle():
    """The time-stepping forcing: n x len(times); at each time the largest
    coefficient among the finest wavelets sits next to the spot centre
    r (cos 2 pi t, sin 2 pi t), r = 1/2, on [0,1]^2 mapped to [-1,1]^2; the
    trajectory has period 1 and the coefficients carry the factor 2^-j."""
    from workloads import WaveletSpec, centers, heat_spot_forcing
    spec = WaveletSpec(5, 1.5, 0.375, "exp", 0.3, 1.5, 7)
    times = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    F = heat_spot_forcing(spec, times)
    c, level = centers(spec.grid_exp)
    assert F.shape == (4 ** spec.grid_exp, times.size)
    fine = level == spec.grid_exp - 1
    for i, t in enumerate(times):
        spot = np.array([0.5 * np.cos(2 * np.pi * t), 0.5 * np.sin(2 * np.pi * t)])
        best = np.argmax(np.where(fine, F[:, i], -np.inf))
        assert np.linalg.norm((2 * c[best] - 1) - spot) <= 2.0 ** -(spec.grid_exp - 1) * np.sqrt(2)
    np.testing.assert_allclose(F[:, 0], F[:, -1], rtol=1e-12, atol=0)
    # a coefficient is 2^-j times f at the support centre
    x = 2 * c - 1
    f0 = 100 * np.exp(-40 * (x[:, 0] - 0.5) ** 2 - 40 * x[:, 1] ** 2)
    np.testing.assert_allclose(F[:, 0], 2.0 ** -level * f0, rtol=1e-12)
