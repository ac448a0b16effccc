"""Pins of the oracle's resolution-rescaling analysis (block-mean
aggregation and the Quantile Error Curve) against exact special cases."""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import coarsen


def test_block_mean_of_constants_ramps_and_partial_blocks():
    rows, cols, b, B = 26, 37, 12, 3          # partial blocks at both edges
    yy, xx = np.mgrid[0:rows, 0:cols]
    rad = np.stack([np.full(rows * cols, 2.5), (xx + 10 * yy).ravel().astype(np.float64),
                    np.where((xx // b + yy // b) % 2 == 0, 1.0, 3.0).ravel()], axis=1).astype(np.float32)
    m = coarsen.block_mean(rad, rows, cols, b)
    R, C = rows // b, cols // b
    assert m.shape == (R * C, B)
    np.testing.assert_array_equal(m[:, 0], 2.5)
    # a linear ramp averages to its value at the block centre
    cy = (np.arange(R) * b + (b - 1) / 2.0)[:, None]
    cx = (np.arange(C) * b + (b - 1) / 2.0)[None, :]
    np.testing.assert_allclose(m[:, 1], (cx + 10 * cy).ravel(), rtol=0, atol=1e-5)
    np.testing.assert_array_equal(m[:, 2], np.where((np.arange(C)[None, :] + np.arange(R)[:, None]) % 2 == 0, 1.0, 3.0).ravel())


def test_normal_and_mixture_quantiles():
    q = np.array(coarsen.QEC_LEVELS)
    np.testing.assert_allclose(coarsen.normal_quantile(q), stats.norm.ppf(q), rtol=0, atol=1e-13)
    # one component: its own quantiles
    for p in q:
        assert coarsen.mixture_quantile([800.0], [50.0], p) == pytest.approx(800 + 50 * stats.norm.ppf(p), abs=1e-8)
    # two mirror-image components: the median is the midpoint
    assert coarsen.mixture_quantile([600.0, 1400.0], [80.0, 80.0], 0.5) == pytest.approx(1000.0, abs=1e-8)
    # well-separated components: the 25 % quantile is the lower one's median
    assert coarsen.mixture_quantile([600.0, 1600.0], [10.0, 10.0], 0.25) == pytest.approx(600.0, abs=1e-6)


def test_qec_vanishes_when_fine_and_coarse_agree():
    """Every fine pixel N(900, 120) and the coarse posterior N(900, 120): the
    mixture QEC is zero; fine E[T] placed at the normal's quantile points
    make the empirical QEC small."""
    rows = cols = 24
    b = 12
    n = rows * cols
    fine = np.tile([900.0, 120.0], (n, 1))
    coarse = np.tile([900.0, 120.0], (4, 1))
    ok = np.ones(n, bool)
    _, valid, emp, mix = coarsen.qec(fine, ok, coarse, np.ones(4, bool), rows, cols, b)
    assert valid.all()
    np.testing.assert_allclose(mix, 0.0, atol=1e-7)
    # empirical: 144 values at the (i + 0.5)/144 quantiles of N(900, 120)
    et = 900 + 120 * stats.norm.ppf((np.arange(144) + 0.5) / 144)
    fine2 = fine.copy()
    for r in range(2):
        for c in range(2):
            idx = ((r * b + np.arange(b))[:, None] * cols + (c * b + np.arange(b))[None, :]).ravel()
            fine2[idx, 0] = np.random.default_rng(r * 2 + c).permutation(et)
    _, _, emp2, _ = coarsen.qec(fine2, ok, coarse, np.ones(4, bool), rows, cols, b)
    assert np.abs(emp2).max() < 12.0          # order-statistic spacing at the tails
    assert np.abs(emp2[:, 3]).max() < 1e-9    # the median is exact by symmetry


def test_qec_selection_and_signs():
    rows = cols = 12
    b = 12
    rng = np.random.default_rng(1)
    fine = np.stack([rng.uniform(600, 1200, 144), rng.uniform(20, 80, 144)], axis=1)
    ok = rng.uniform(size=144) < 0.5
    # a coarse posterior shifted up by 100 K gives a QEC >= 100 - (spread) ...
    coarse = np.array([[np.median(fine[ok, 0]) + 100.0, 1e-3]])
    n_used, valid, emp, mix = coarsen.qec(fine, ok, coarse, np.array([True]), rows, cols, b)
    assert n_used[0] == ok.sum() and valid[0]
    assert emp[0, 3] == pytest.approx(100.0, abs=1e-9)
    # too few selected fine pixels: not valid
    _, v2, e2, _ = coarsen.qec(fine, np.zeros(144, bool), coarse, np.array([True]), rows, cols, b)
    assert not v2[0] and np.all(np.isnan(e2))
