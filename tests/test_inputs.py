"""Seeded input generators: the counter generator follows its published definition, draws are
deterministic, and the Gaussian random field has the requested statistics (its values are
otherwise generator-defined, so parity on them is by construction)."""
import math

import numpy as np

import inputs


def test_splitmix64_published_sequence():
    # SplitMix64 started from state 0 yields 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F
    z = np.arange(1, 4, dtype=np.uint64) * inputs.GOLDEN
    out = inputs._mix64(z)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_determinism_and_ranges():
    a = inputs.uniform(3, 5, 1000, 0.0, 0.1)
    b = inputs.uniform(3, 5, 1000, 0.0, 0.1)
    assert np.array_equal(a, b) and a.min() >= 0.0 and a.max() < 0.1
    assert not np.array_equal(a, inputs.uniform(3, 6, 1000, 0.0, 0.1))
    # counters are addressable: an offset window equals the tail of a longer draw
    assert np.array_equal(inputs.uniform(3, 5, 10, offset=990), inputs.uniform(3, 5, 1000)[990:])
    k = inputs.randint(1, 2, 20000, 8, 128)
    assert k.min() == 8 and k.max() == 128
    z = inputs.normal(1, 1, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01


def test_grf_statistics():
    pts = np.array([[0.0, 0.0], [0.2, 0.0]])
    vals = np.array([inputs.grf_rff(pts, seed=s, stream=1, nfeat=512) for s in range(600)])
    var = vals.var(axis=0).mean()
    cov = np.mean(vals[:, 0] * vals[:, 1])
    assert abs(var - 0.5) < 0.08
    assert abs(cov - 0.5 * math.exp(-0.5)) < 0.08


def test_initial_guess_boundary_zero():
    U = inputs.initial_guess([18, 18], seed=1)
    m = inputs.boundary_mask([18, 18])
    assert np.all(U[m] == 0) and np.all(U[~m] > 0) and U.max() < 0.1
    assert m.sum() == 4 * 17


def test_cylinder_weights_and_sizes():
    p = inputs.quarter_cylinder(48, 3)
    assert p.shape == [51, 51, 51] and p.ndof == 132651
    assert p.weights.min() > 0.7 and p.weights.max() <= 1.0 + 1e-15
    # single quadratic span: along the angle (axis 1) the weights are 1, sqrt(2)/2, 1;
    # natural order is (i2, i1, i0) when reshaped
    p2 = inputs.quarter_cylinder(1, 2)
    w = p2.weights.reshape(3, 3, 3)
    for i0 in range(3):
        assert np.allclose(w[0, :, i0], [1.0, math.sqrt(0.5), 1.0], atol=1e-16)
    assert np.allclose(w[:, 0, :], 1.0)


def test_grf_grid_statistics():
    """Circulant-embedding field: variance 0.5 and correlation 0.5 exp(-1/2) at distance 0.2."""
    fs = np.array([inputs.grf_grid(32, seed=9, stream=s) for s in range(400)])
    assert abs(fs.var() - 0.5) < 0.05
    lag = round(0.2 * 32)                       # 0.2 / h cells
    c = np.mean(fs[:, :, :-lag] * fs[:, :, lag:])
    assert abs(c - 0.5 * np.exp(-0.5 * (lag / 32 / 0.2) ** 2)) < 0.05
    assert np.array_equal(inputs.grf_grid(32, 9, 3), inputs.grf_grid(32, 9, 3))
