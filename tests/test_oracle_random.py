"""Pins of the oracle's random streams: Philox4x64-10 against numpy's library
implementation, own ln/sincos against libm, and the Gaussian transform by its
moments and a Kolmogorov-Smirnov test."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import fmath, philox, projection


@pytest.mark.parametrize("key,ctr", [((0, 0), (1, 0, 0, 0)), ((7, 9), (5, 3, 2, 1)),
                                     ((2**64 - 1, 0x10), (123456789, 2**40, 0, 7))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox bumps the counter before producing a block
    start = np.array(ctr, dtype=np.uint64)
    start[0] -= np.uint64(1)
    bg = np.random.Philox(counter=start, key=np.array(key, dtype=np.uint64))
    ref = bg.random_raw(12).reshape(3, 4)
    ctrs = np.array([ctr] * 3, dtype=np.uint64)
    ctrs[:, 0] += np.arange(3, dtype=np.uint64)
    out = philox.philox4x64(ctrs, np.array(key, dtype=np.uint64))
    assert np.array_equal(out, ref)


def test_philox_block_grid_layout():
    blk = philox.block_grid(5, 0x10, 3, 2)
    one = philox.philox4x64(np.array([2, 1, 0, 0], dtype=np.uint64),
                            np.array([5, 0x10], dtype=np.uint64))
    assert np.array_equal(blk[2, 1], one)


def _ulps(a, ref):
    return np.abs(a - ref) / np.spacing(np.maximum(np.abs(ref), 1e-300))


def test_ln_against_libm():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.random(100000), 2.0 ** -rng.uniform(0, 60, 100000),
                        rng.uniform(1, 1e6, 10000), [1.0, 0.5, 2.0 ** -52]])
    ref = np.array([math.log(v) for v in x])
    got = fmath.ln(x)
    assert _ulps(got, ref).max() <= 4
    assert got[-3] == 0.0


def test_sincos_against_libm():
    rng = np.random.default_rng(4)
    u = np.concatenate([rng.random(100000), [0.0, 0.125, 0.25, 0.5, 0.75, 1.0]])
    s, c = fmath.sincos_2pi(u)
    rs = np.array([math.sin(2 * math.pi * v) for v in u])
    rc = np.array([math.cos(2 * math.pi * v) for v in u])
    assert np.max(np.abs(s - rs)) < 2e-15 and np.max(np.abs(c - rc)) < 2e-15
    # exact quadrant points
    assert s[-6] == 0.0 and c[-6] == 1.0
    assert s[-4] == 1.0 and c[-4] == 0.0
    assert c[-3] == -1.0 and s[-2] == -1.0
    assert np.all(s * s + c * c - 1.0 < 1e-15)


def test_uniform_open_interval_exact():
    x = np.array([0, 2**64 - 1, 2**63, 4095, 4096], dtype=np.uint64)
    u = fmath.uniform52(x)
    assert u[0] == 2.0 ** -53 and u[1] == 1.0 - 2.0 ** -53
    assert u[2] == 0.5 + 2.0 ** -53 and u[3] == u[0] and u[4] == 3 * 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_box_muller_radius_identity():
    rng = np.random.default_rng(5)
    u0, u1 = rng.random(1000) + 1e-9, rng.random(1000)
    z0, z1 = fmath.box_muller(u0, u1)
    np.testing.assert_allclose(z0 * z0 + z1 * z1, -2.0 * np.log(u0), rtol=1e-13)


def test_normals_moments_and_ks():
    blk = philox.block_grid(11, 0x10, 50000, 8)
    z = fmath.normals_from_block(blk).ravel()          # 1.6M normals
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(stats.skew(z)) < 5 * math.sqrt(6.0 / n)
    assert abs(stats.kurtosis(z)) < 5 * math.sqrt(24.0 / n)
    assert stats.kstest(z[:200000], "norm").pvalue > 1e-4
    # independence of the two Box-Muller outputs and across columns
    zz = fmath.normals_from_block(blk).reshape(-1, 32)
    corr = np.corrcoef(zz.T)
    assert np.max(np.abs(corr - np.eye(32))) < 5 / math.sqrt(zz.shape[0])


def test_theta_scale_and_fp32():
    t = projection.theta(0, 4000, 64)
    assert t.dtype == np.float64 and t.shape == (4000, 64)
    assert np.array_equal(t.astype(np.float32).astype(np.float64), t)
    assert abs(t.std() - 64 ** -0.5) < 0.01 * 64 ** -0.5 * 5
    # column count not a multiple of 4 takes the leading columns of the blocks
    t6 = projection.gaussian_matrix(0, 0x10, 10, 6, 1.0)
    t8 = projection.gaussian_matrix(0, 0x10, 10, 8, 1.0)
    assert np.array_equal(t6, t8[:, :6])
