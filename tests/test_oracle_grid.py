"""Pins of the oracle's Gaussian-mixture thermal model on the temperature
grid (model 3; Sec. 2.2: a discrete sum over a grid spanning [350, 2200] K of
an eta-weighted flaming and smouldering Gaussian): limits that reduce it to a
single Planck radiance or to a plain average, Stefan-Boltzmann through the
forward model, the Jacobian against finite differences, and noise-free
recovery by the LM oracle."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import scenegen

SIGMA_SB = 5.670374419e-8
LO, HI, X0 = scenegen.default_prior(3)


def _thermal_only(lam):
    z = np.zeros_like(lam)
    return oracle.Tables(lam=lam, K=z.copy(), tau2=z.copy(), tup=np.ones_like(lam), ratm=z.copy(),
                         S=z.copy(), lsat=None)


def test_grid_nodes():
    T = oracle.grid_nodes(32)
    assert T[0] == 350.0 and T[-1] == 2200.0 and len(T) == 32
    np.testing.assert_allclose(np.diff(T), 1850.0 / 31, rtol=1e-13)


@pytest.mark.parametrize("q", [16, 32])
def test_narrow_components_on_nodes_are_single_planck_radiances(q):
    """A component much narrower than the node spacing, centred on a node,
    puts all its weight there: the thermal term is f tau_up (eta B(T_h) +
    (1 - eta) B(T_s)) exactly."""
    tab = oracle.band_tables(scenegen.make_atmosphere(0, 0))
    T = oracle.grid_nodes(q)
    ts, th = T[3], T[q - 4]
    for eta, f in [(0.3, 0.05), (0.8, 0.01)]:
        x = np.array([[f, eta, ts, 1.0, th, 1.0, 0.2, 1e-5]])
        bg = oracle.forward(tab, np.array([[0.0, eta, ts, 1.0, th, 1.0, 0.2, 1e-5]]), 3, q=q)[0]
        L = oracle.forward(tab, x, 3, q=q)[0]
        want = bg + f * tab.tup * (eta * oracle.planck(tab.lam, th) + (1 - eta) * oracle.planck(tab.lam, ts))
        np.testing.assert_allclose(L, want, rtol=1e-12)


def test_very_wide_components_average_the_grid():
    """sigma >> the grid span makes the weights uniform: the thermal term is
    the plain mean of B over the nodes."""
    lam = np.linspace(400.0, 2500.0, 50)
    tab = _thermal_only(lam)
    T = oracle.grid_nodes(32)
    L = oracle.forward(tab, np.array([[1.0, 0.5, 600.0, 1e9, 1500.0, 1e9, 0.0, 0.0]]), 3, q=32)[0]
    want = np.mean([oracle.planck(lam, t) for t in T], axis=0)
    np.testing.assert_allclose(L, want, rtol=1e-9)


@pytest.mark.parametrize("ms,ss,mh,sh,eta", [(600.0, 80.0, 1200.0, 150.0, 0.4), (800.0, 200.0, 1800.0, 60.0, 0.9)])
def test_stefan_boltzmann_through_the_forward_model(ms, ss, mh, sh, eta):
    """f = 1, tau_up = 1, no solar term: pi int L dlam = sigma sum_i p_i T_i^4
    with p the normalised Gaussian weights on the nodes."""
    u = np.linspace(math.log(5.0), math.log(1e9), 60001)
    lam = np.exp(u)
    tab = _thermal_only(lam)
    L = oracle.forward(tab, np.array([[1.0, eta, ms, ss, mh, sh, 0.0, 0.0]]), 3, q=32)[0]
    tot = math.pi * integrate.simpson(L * lam, x=u)
    T = oracle.grid_nodes(32)

    def e4(mu, sig):
        w = np.exp(-0.5 * ((T - mu) / sig) ** 2)
        return float((w * T ** 4).sum() / w.sum())
    assert tot == pytest.approx(SIGMA_SB * (eta * e4(mh, sh) + (1 - eta) * e4(ms, ss)), rel=1e-9)


def test_jacobian_finite_difference():
    atm = scenegen.make_atmosphere(0, 1, rho_atm=0.01, s_sph=0.1)
    tab = oracle.band_tables(atm)
    rng = np.random.default_rng(31)
    X = scenegen.draw_states_gauss_grid2(rng, 12)
    X[:, 0] = np.exp(rng.uniform(np.log(1e-3), np.log(0.2), 12))
    _, J = oracle.forward(tab, X, 3, jacobian=True)
    n = X.shape[1]
    for j in range(n):
        h = 1e-5 * np.maximum(np.abs(X[:, j]), 1e-3 if j < n - 1 else 1e-6)

        def cd(hh):
            Xp, Xm = X.copy(), X.copy()
            Xp[:, j] += hh
            Xm[:, j] -= hh
            return (oracle.forward(tab, Xp, 3) - oracle.forward(tab, Xm, 3)) / (2 * hh[:, None])
        fd = (4 * cd(h / 2) - cd(h)) / 3.0
        num = np.linalg.norm(J[:, :, j] - fd, axis=1)
        den = np.linalg.norm(J[:, :, j], axis=1)
        assert np.all(num <= 1e-6 * den + 1e-14), (j, (num / den).max())


def test_truth_is_a_fixed_point_of_the_lm_oracle():
    """Noise-free spectra, LM started at the truth: it stops there (the
    residual stays at the float32 floor of the spectra and the state does not
    move); the two-component mixture is degenerate enough that starts away
    from the truth can stop in flat valleys of equal cost, which the parity
    tests cover."""
    tab = oracle.band_tables(scenegen.make_atmosphere(5, 0))
    X = scenegen.config5_states(64, scene=2)
    X = X[X[:, 0] >= 1e-2][:16]
    lobs = oracle.forward(tab, X, 3).astype(np.float32)
    zt = oracle.x_to_z(X, LO, HI)
    r = oracle.retrieve(tab, lobs, 3, LO, HI, X0, z0=zt, opts=oracle.LMOptions(max_iter=300))
    et, _ = oracle.mixture_moments(X[:, 1], X[:, 4], X[:, 5], X[:, 2], X[:, 3])
    assert np.all(r.converged)
    assert np.all(r.rrr <= 1e-7), r.rrr
    # the float32 rounding of the spectra moves the minimum along the flat
    # directions of the mixture by up to ~0.6 K in E[T]
    np.testing.assert_allclose(r.moments[:, 0], et, atol=1.0)
    np.testing.assert_allclose(r.state[:, 0], X[:, 0], rtol=1e-3)
