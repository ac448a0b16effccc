"""Spatial-resolution rescaling analysis (Keely et al., the resolution
rescaling of the methods section and its Results): test infrastructure, like
the rest of ``oracle/``.

  * ``block_mean``: coarse radiance as the mean of b x b fine pixels in
    radiance space (the paper aggregates 12 x 12); partial blocks at the
    right and bottom edges are dropped.  The mean of each block and band is
    formed in float64 and rounded once to float32.
  * ``qec``: the Quantile Error Curve QEC(q) = Q_coarse(q) - Q_fine(q) per
    coarse pixel, q in (0.05, 0.10, 0.25, 0.50, 0.75, 0.90, 0.95), where
    Q_coarse is the quantile of the coarse pixel's moment-matched Gaussian
    N(E[T], sigma[T]) and Q_fine the quantile of the fine retrievals inside
    its footprint: either their empirical distribution of E[T] (linear
    interpolation between order statistics) or their Gaussian-mixture
    reconstruction, the equal-weight mixture of the fine pixels' N(E[T],
    sigma[T]).
"""
from __future__ import annotations

import numpy as np
from scipy import optimize, special

QEC_LEVELS = (0.05, 0.10, 0.25, 0.50, 0.75, 0.90, 0.95)


def block_mean(rad, rows: int, cols: int, block: int):
    """[rows * cols, B] float32 (row-major pixels) -> [(rows // block) *
    (cols // block), B] float32."""
    rad = np.asarray(rad)
    B = rad.shape[1]
    R, C = rows // block, cols // block
    img = rad.reshape(rows, cols, B)[:R * block, :C * block].astype(np.float64)
    m = img.reshape(R, block, C, block, B).sum(axis=(1, 3)) / float(block * block)
    return m.reshape(R * C, B).astype(np.float32)


def normal_quantile(q):
    """Phi^{-1}(q) of the standard normal."""
    return np.sqrt(2.0) * special.erfinv(2.0 * np.asarray(q, np.float64) - 1.0)


def mixture_quantile(mu, sd, q: float) -> float:
    """x with (1/n) sum_i Phi((x - mu_i)/sd_i) = q (Brent's method)."""
    mu = np.asarray(mu, np.float64)
    sd = np.asarray(sd, np.float64)

    def F(x):
        return 0.5 * np.mean(special.erfc(-(x - mu) / (sd * np.sqrt(2.0)))) - q
    lo = float(np.min(mu - 12.0 * sd))
    hi = float(np.max(mu + 12.0 * sd))
    return optimize.brentq(F, lo, hi, xtol=1e-10, rtol=1e-15, maxiter=500)


def selection(status, f, moments, converged_mask: int, f_min: float):
    """Pixels that take part (fine pixels in a footprint's distribution, or a
    coarse pixel itself): converged, fire fraction at least f_min, finite
    E[T] and a positive finite sigma[T]."""
    st = np.asarray(status).astype(np.int64)
    m = np.asarray(moments, np.float64)
    return (((st & converged_mask) != 0) & (np.asarray(f) >= f_min) & np.isfinite(m[:, 0])
            & np.isfinite(m[:, 1]) & (m[:, 1] > 0))


def qec(fine_moments, fine_ok, coarse_moments, coarse_ok, rows: int, cols: int, block: int,
        levels=QEC_LEVELS, min_fine: int = 5):
    """Per coarse pixel: number of fine pixels used, validity, and the
    empirical and mixture QEC at the given levels ([n_coarse, n_levels],
    NaN where not valid).  A coarse pixel is valid when it is selected itself
    (coarse_ok) and at least min_fine of its fine pixels are."""
    fm = np.asarray(fine_moments, np.float64)
    cm = np.asarray(coarse_moments, np.float64)
    R, C = rows // block, cols // block
    levels = np.asarray(levels, np.float64)
    zq = normal_quantile(levels)
    n_used = np.zeros(R * C, np.int64)
    valid = np.zeros(R * C, bool)
    emp = np.full((R * C, len(levels)), np.nan)
    mix = np.full((R * C, len(levels)), np.nan)
    for r in range(R):
        for c in range(C):
            k = r * C + c
            idx = ((r * block + np.arange(block))[:, None] * cols + (c * block + np.arange(block))[None, :]).ravel()
            sel = idx[np.asarray(fine_ok)[idx]]
            n_used[k] = len(sel)
            if not (coarse_ok[k] and len(sel) >= min_fine):
                continue
            valid[k] = True
            gauss = cm[k, 0] + cm[k, 1] * zq
            et, sd = fm[sel, 0], fm[sel, 1]
            emp[k] = gauss - np.quantile(et, levels, method="linear")
            mix[k] = gauss - np.array([mixture_quantile(et, sd, q) for q in levels])
    return n_used, valid, emp, mix
