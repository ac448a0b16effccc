"""Pins of the oracle's fire-candidate index (Sec. 2.1, HFDI) against values
worked by hand, the Planck closed form for a thermal-only spectrum, and the
invariants of the ratio."""
import numpy as np

import oracle
import scenegen
from _helpers import noisy_spectra


def _tab(lsat=None):
    return oracle.band_tables(scenegen.make_atmosphere(0, 0, sat_level=lsat))


def test_bands_and_hand_values():
    tab = _tab()
    ia = oracle.nearest_band(tab.lam, 2430.0)
    ib = oracle.nearest_band(tab.lam, 2061.0)
    assert abs(tab.lam[ia] - 2430.0) <= 0.5 * (tab.lam[1] - tab.lam[0])
    assert abs(tab.lam[ib] - 2061.0) <= 0.5 * (tab.lam[1] - tab.lam[0])
    L = np.ones((4, tab.B), np.float32)
    L[0, ia], L[0, ib] = 3.0, 1.0       # (3 - 1) / (3 + 1) = 0.5
    L[1, ia], L[1, ib] = 1.0, 3.0       # -0.5
    L[2, ia], L[2, ib] = 9.0, 11.0      # -0.1 (float32 rounding decides)
    L[3, ia], L[3, ib] = 0.0, 0.0       # 0/0
    h = oracle.hfdi(tab, L)
    assert h[0] == np.float32(0.5) and h[1] == np.float32(-0.5)
    assert h[2] == np.float32(-2.0) / np.float32(20.0)
    assert np.isnan(h[3])
    idx, _ = oracle.hfdi_candidates(tab, L)
    want = [0] + ([2] if float(np.float32(-2.0) / np.float32(20.0)) >= -0.1 else [])
    assert list(idx) == want


def test_thermal_only_spectrum_is_the_planck_ratio():
    """A spectrum of pure emission f tau_up B(T) with a spectrally flat
    tau_up gives HFDI = (B(2430, T) - B(2061, T)) / (B(2430, T) + B(2061, T))
    at the band centres, independent of f."""
    tab = _tab()
    ia, ib = oracle.nearest_band(tab.lam, 2430.0), oracle.nearest_band(tab.lam, 2061.0)
    T = np.array([500.0, 800.0, 1200.0, 2000.0])
    L = np.zeros((len(T), tab.B), np.float32)
    for k, t in enumerate(T):
        L[k] = (0.01 * oracle.planck(tab.lam, t)).astype(np.float32)
    h = oracle.hfdi(tab, L)
    Ba, Bb = oracle.planck(tab.lam[ia], T), oracle.planck(tab.lam[ib], T)
    np.testing.assert_allclose(h, (Ba - Bb) / (Ba + Bb), rtol=1e-5, atol=1e-6)
    # hotter is whiter: the index falls with temperature beyond the Wien
    # peak crossing, and at 500 K the longer band dominates
    assert h[0] > 0.5


def test_invariants_and_reflected_sunlight():
    tab = _tab()
    X = scenegen.config0_states(256)
    L = noisy_spectra(tab, X, 1, 0, 0)
    h = oracle.hfdi(tab, L)
    # scale invariance (powers of two keep float32 exact) and antisymmetry
    np.testing.assert_array_equal(oracle.hfdi(tab, L * np.float32(4.0)), h)
    ia, ib = oracle.nearest_band(tab.lam, 2430.0), oracle.nearest_band(tab.lam, 2061.0)
    Ls = L.copy()
    Ls[:, [ia, ib]] = L[:, [ib, ia]]
    np.testing.assert_array_equal(oracle.hfdi(tab, Ls), -h)
    # reflected sunlight alone (f = 0): the 5778 K sun is dimmer at 2430 than
    # at 2061 nm (by ~0.58), so background pixels whose reflectance is
    # positive at both bands fall below the threshold (the linear reflectance
    # of the synthetic draws can reach zero at the long-wave end, where the
    # index of a near-zero radiance is noise)
    Xb = X.copy()
    Xb[:, 0] = 0.0
    hb = oracle.hfdi(tab, noisy_spectra(tab, Xb, 1, 0, 0))
    rho = lambda lam: Xb[:, 3] + Xb[:, 4] * (lam - oracle.LAMBDA_REF_NM)
    ok = (rho(2061.0) >= 0.02) & (rho(2430.0) >= 0.02)
    assert ok.sum() > 200
    assert np.all(hb[ok] < -0.1)
    # strong fires are candidates
    hot = (X[:, 0] > 0.01) & (X[:, 1] > 800)
    assert hot.sum() > 10 and np.all(h[hot] >= -0.1)


def test_saturated_bands_make_a_candidate():
    X = scenegen.config0_states(64)
    X[:, 0] = 0.0
    tab0 = _tab()
    L = noisy_spectra(tab0, X, 1, 0, 0)
    ia = oracle.nearest_band(tab0.lam, 2430.0)
    lsat = np.full(tab0.B, 1e6, np.float32)
    lsat[ia] = np.float32(np.median(L[:, ia]))
    tab = _tab(lsat)
    idx, h = oracle.hfdi_candidates(tab, L)
    sat = L[:, ia] >= lsat[ia]
    assert np.all(h < -0.1)
    np.testing.assert_array_equal(idx, np.nonzero(sat)[0])
