"""Pins for the oracle's random numbers: Philox4x32-10 against the published
known-answer vectors, the uniform mapping, Box-Muller special values and the
Marsaglia-Tsang gamma sampler against SciPy's gamma distribution."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert list(O.philox(ctr, key)) == out


def test_philox_counter_sensitivity():
    # every counter word and key word changes the output
    base = O.philox([1, 2, 3, 4], [5, 6])
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert not np.array_equal(O.philox(c, [5, 6]), base)
    for i in range(2):
        k = [5, 6]
        k[i] ^= 1
        assert not np.array_equal(O.philox([1, 2, 3, 4], k), base)


def test_uniform_range_and_binary32_exact():
    assert O.uniform(0) == 2.0 ** -24
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for r in [0, 255, 256, 12345678, 0x80000000, 0xFFFFFF00, 0xFFFFFFFF]:
        u = O.uniform(r)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in binary32


def test_box_muller_special_values():
    # u1 = exp(-1/2) gives radius 1; u2 = 1/8 gives angle pi/4
    z0, z1 = O.box_muller(np.exp(-0.5), 0.125)
    assert abs(z0 - np.sqrt(0.5)) < 1e-15 and abs(z1 - np.sqrt(0.5)) < 1e-15
    z0, z1 = O.box_muller(np.exp(-2.0), 0.5)  # radius 2, angle pi
    assert abs(z0 + 2.0) < 1e-15 and abs(z1) < 1e-15


def test_box_muller_gaussian_statistics():
    n = 40000
    z = np.empty(2 * n)
    key = [7, 0]
    for i in range(n):
        r = O.philox([i, 3, 0, 0], key)
        z[2 * i], z[2 * i + 1] = O.box_muller(O.uniform(r[0]), O.uniform(r[1]))
    assert abs(z.mean()) < 5 / np.sqrt(2 * n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / (2 * n))
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the pair is independent
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / np.sqrt(n)


@pytest.mark.parametrize("shape,scale", [(4.0, 0.25), (4.0, 3.0), (1.5, 1.0)])
def test_gamma_matches_scipy(shape, scale):
    n = 20000
    g = np.array([O.gamma(shape, scale, 11, i, 5, 16)[0] for i in range(n)])
    assert abs(g.mean() - shape * scale) < 5 * np.sqrt(shape) * scale / np.sqrt(n)
    assert stats.kstest(g, stats.gamma(shape, scale=scale).cdf).pvalue > 1e-3
