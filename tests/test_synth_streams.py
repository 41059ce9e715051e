"""The index streams of the access-pattern microbenchmarks (Section 4.1):
constant strides exactly, the keep-with-probability-1/k rule's geometric
gaps (mean k, variance k(k-1)) and the Gaussian gaps (mean m, deviation sd)
within sampling error."""
import numpy as np
import pytest

import synth


def test_constant_stride_exact():
    rng = np.random.default_rng(0)
    assert synth.index_stream("IS", 5, 7, rng).tolist() == [0, 7, 14, 21, 28]


@pytest.mark.parametrize("k", [1, 2, 8, 530])
def test_random_stride_law(k):
    n = 400_000
    ind = synth.index_stream("IR", n, k, np.random.default_rng(k))
    g = np.diff(ind)
    assert ind[0] >= 0 and np.all(g >= 1)                     # strictly increasing
    se = np.sqrt(k * (k - 1) / n) + 1e-12
    assert abs(g.mean() - k) <= 6 * se
    if k > 1:
        assert abs(g.var() / (k * (k - 1)) - 1) < 0.05
    else:
        assert np.all(g == 1)


def test_random_stride_matches_elementwise_rule():
    """The geometric gaps have the law of testing every element against 1/k:
    compare the fraction of gaps equal to 1, 2, 3 with (1-p)^(j-1) p."""
    k, n = 4, 400_000
    g = np.diff(synth.index_stream("IR", n, k, np.random.default_rng(5)))
    p = 1.0 / k
    for j in (1, 2, 3):
        assert abs((g == j).mean() - (1 - p) ** (j - 1) * p) < 0.005


@pytest.mark.parametrize("m,sd", [(4, 0.0), (16, 64.0), (1, 256.0)])
def test_gaussian_strides(m, sd):
    n = 200_000
    ind = synth.index_stream("GAUSS", n, m, np.random.default_rng(7), sd)
    assert ind.min() >= 0
    g = np.diff(ind)
    if sd == 0:
        assert np.all(g == m)
    else:
        assert abs(g.mean() - m) < 6 * sd / np.sqrt(n) + 0.01
        assert abs(g.std() / np.sqrt(sd * sd + 1 / 12) - 1) < 0.02
        assert (g < 0).mean() > 0.3 if sd > 8 * m else True     # backward jumps present
