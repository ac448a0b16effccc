"""Pins of the oracle's staged Adam (Sec. 2.5, eq. adam) against facts that do
not come from its own code: finite differences of the windowed loss
(eq. loss), the closed form of Adam's first step (bias correction makes
m_hat = g and v_hat = g^2 at t = 1), convergence to the known truth of a
noise-free one-variable problem, and the LM oracle's outputs at a shared
point."""
import dataclasses

import numpy as np
import pytest

import oracle
import scenegen
from _helpers import noisy_spectra

LO, HI, X0 = scenegen.default_prior(1)


@pytest.fixture(scope="module")
def scene():
    atm = scenegen.make_atmosphere(0, 0)
    return oracle.band_tables(atm)


@pytest.fixture(scope="module")
def pixels(scene):
    states = scenegen.config0_states(64)
    states = states[states[:, 0] > 3e-3][:6]
    return states, noisy_spectra(scene, states, 1, 0, 0)


def windowed_loss_fd(tab, lobs, z, windows, h=1e-6, model=1, lo=LO, hi=HI):
    """Central differences of sum_{b in window_j, unsaturated} (L_obs - L)^2
    in z_j, per pixel; windows: j -> (lo_nm, hi_nm)."""
    P, n = z.shape
    G = np.zeros((P, n))
    for j, (wl, wh) in windows.items():
        win = (tab.lam >= wl) & (tab.lam <= wh)
        for p in range(P):
            u = win if tab.lsat is None else win & (lobs[p] < tab.lsat)
            e = np.zeros(n)
            e[j] = h
            Lp = oracle.forward(tab, oracle.z_to_x(z[p] + e, lo, hi)[None], model)[0]
            Lm = oracle.forward(tab, oracle.z_to_x(z[p] - e, lo, hi)[None], model)[0]
            lp = ((lobs[p].astype(np.float64) - Lp) ** 2)[u].sum()
            lm = ((lobs[p].astype(np.float64) - Lm) ** 2)[u].sum()
            G[p, j] = (lp - lm) / (2 * h)
    return G


def z_of(res):
    return oracle.x_to_z(res.state, LO, HI)


@pytest.mark.parametrize("eps,saturate", [(1e-8, False), (0.3, False), (3.0, True)])
def test_first_step_is_the_closed_form_on_a_finite_difference_gradient(scene, pixels, eps, saturate):
    """t = 1: z_1 = z_0 - lr g / (|g| + eps) with g = dLoss/dz; with eps near
    |g| the step length measures |g| itself (the factor 2 of the squared
    residual, the dx/dz scaling and the window); saturated bands are left
    out; held variables stay put."""
    states, lobs = pixels
    if saturate:
        # about half of the pixels saturate in each band
        lsat = np.median(lobs, axis=0).astype(np.float32)
        scene = oracle.Tables(scene.lam, scene.K, scene.tau2, scene.tup, scene.ratm, scene.S, lsat)
    win = {0: (900.0, 2500.0), 1: (900.0, 1800.0), 2: (1500.0, 2500.0), 3: (350.0, 2500.0)}
    lr = 0.01
    stage = oracle.AdamStage(1, lr, (0, 1, 2, 3), win, clip=0.0)
    z0 = np.tile(oracle.x_to_z(X0, LO, HI), (len(states), 1))
    r = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, [stage], eps=eps)
    G = windowed_loss_fd(scene, lobs, z0, win)
    want = z0 - lr * G / (np.abs(G) + eps)
    want[:, 4] = z0[:, 4]
    # pixels brighter than the median in more than B - 6 bands have no solve
    ok = (r.status & oracle.ST_NODOF) == 0
    assert ok.sum() >= 4 and np.all(np.isnan(r.state[~ok]))
    got = z_of(r)[ok]
    np.testing.assert_allclose(got, np.clip(want[ok], -1, 1), rtol=0, atol=lr * 1e-5)
    np.testing.assert_allclose(got[:, 4], z0[ok, 4], rtol=0, atol=1e-14)
    assert np.all(r.iters[ok] == 1)


def test_two_component_stage_two_windows(scene):
    """The second stage of the two-component model: each component's
    variables see their own window, f and eta the union (first-step closed
    form on finite differences)."""
    lo, hi, x0 = scenegen.default_prior(2)
    states = scenegen.config2_states(4)
    states[:, 0] = 0.02
    lobs = noisy_spectra(scene, states, 2, 2, 0)
    stage = dataclasses.replace(oracle.paper_stages(2, lo, hi, x0)[1], steps=1, clip=0.0)
    assert stage.window[2] == oracle.OMEGA_SMOL and stage.window[4] == oracle.OMEGA_HOT
    eps, lr = 1.0, stage.lr
    r = oracle.adam_retrieve(scene, lobs, 2, lo, hi, x0, [stage], eps=eps)
    z0 = np.tile(oracle.x_to_z(x0, lo, hi), (len(states), 1))
    G = windowed_loss_fd(scene, lobs, z0, stage.window, model=2, lo=lo, hi=hi)
    want = np.clip(z0 - lr * G / (np.abs(G) + eps), -1, 1)
    np.testing.assert_allclose(oracle.x_to_z(r.state, lo, hi), want, rtol=0, atol=lr * 1e-5)


def test_global_norm_clip_scales_the_gradient_before_the_moments(scene, pixels):
    """With ||g|| above the clip c the step uses g c / ||g|| (norm over the
    free variables): with eps comparable to the clipped components the step
    length shows the scaling."""
    states, lobs = pixels
    win = {j: (350.0, 2500.0) for j in (0, 1, 3)}
    z0 = np.tile(oracle.x_to_z(X0, LO, HI), (len(states), 1))
    G = windowed_loss_fd(scene, lobs, z0, win)
    norm = np.sqrt((G ** 2).sum(1))
    c = 0.25 * norm.min()
    eps = 0.1 * c
    lr = 0.02
    r = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0,
                             [oracle.AdamStage(1, lr, (0, 1, 3), win, clip=c)], eps=eps)
    Gc = G * (c / norm)[:, None]
    want = z0 - lr * Gc / (np.abs(Gc) + eps)
    for j in (2, 4):
        want[:, j] = z0[:, j]
    np.testing.assert_allclose(z_of(r), np.clip(want, -1, 1), rtol=0, atol=lr * 1e-5)
    # a clip that never binds is no clip
    big = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0,
                               [oracle.AdamStage(7, lr, (0, 1, 3), win, clip=1e30)])
    none = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0,
                                [oracle.AdamStage(7, lr, (0, 1, 3), win, clip=0.0)])
    assert np.array_equal(big.state, none.state)


def test_each_stage_starts_a_fresh_optimiser(scene, pixels):
    """After any first stage, a one-step second stage moves by the t = 1
    closed form at the first stage's end point."""
    states, lobs = pixels
    win = {j: (350.0, 2500.0) for j in range(5)}
    first = oracle.AdamStage(6, 0.03, (0, 1, 2, 3, 4), win, clip=1.0)
    eps, lr = 0.5, 0.004
    b = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0,
                             [first, oracle.AdamStage(1, lr, (0, 1, 2, 3, 4), win, clip=0.0)], eps=eps)
    za = z_of(oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, [first], eps=eps))
    G = windowed_loss_fd(scene, lobs, za, win)
    want = np.clip(za - lr * G / (np.abs(G) + eps), -1, 1)
    np.testing.assert_allclose(z_of(b), want, rtol=0, atol=lr * 1e-5)
    assert np.all(b.iters == 7)


def test_stage_start_values_and_held_variables(scene, pixels):
    states, lobs = pixels
    win = {1: (350.0, 2500.0)}
    z0 = oracle.x_to_z(states, LO, HI) * 0.5
    st = [oracle.AdamStage(0, 0.1, (1,), win, zset={2: -1.0, 4: 0.25}),
          oracle.AdamStage(3, 0.01, (1,), win)]
    r = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, st, z0=z0)
    z = z_of(r)
    np.testing.assert_allclose(z[:, [0, 3]], z0[:, [0, 3]], rtol=0, atol=1e-14)
    np.testing.assert_allclose(z[:, 2], -1.0, atol=1e-14)
    np.testing.assert_allclose(z[:, 4], 0.25, atol=1e-14)
    assert np.all(np.abs(z[:, 1] - z0[:, 1]) <= 3 * 0.01 + 1e-12)
    assert np.all(r.iters == 3)


def test_each_variable_alone_converges_to_the_truth(scene):
    """Noise-free spectra, every other variable at its true value: Adam on the
    one free variable, with the learning rate cut tenfold twice (three
    stages), ends at the true value -- a wrong sign or scale in any Jacobian
    column would run to a bound or stall."""
    states = scenegen.config0_states(64)
    states = states[states[:, 0] > 3e-3][:6]
    lobs = noisy_spectra(scene, states, 1, 0, 0, snr=None)
    zt = oracle.x_to_z(states, LO, HI)
    zdef = oracle.x_to_z(X0, LO, HI)
    for j in range(5):
        z0 = zt.copy()
        z0[:, j] = zdef[j]
        st = [oracle.AdamStage(200, lr, (j,), {j: (350.0, 2500.0)}, 0.0) for lr in (0.02, 0.002, 0.0002)]
        r = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, st, z0=z0)
        err = np.abs(z_of(r)[:, j] - zt[:, j])
        assert err.max() < 1e-6, (j, err)


def test_outputs_at_a_given_point_match_the_lm_oracle(scene, pixels):
    """With no steps the result is the output of the given start point: the
    covariance, moments and relative residual are the same computation as the
    LM oracle's at its converged point."""
    states, lobs = pixels
    lm = oracle.retrieve(scene, lobs, 1, LO, HI, X0)
    zl = oracle.x_to_z(lm.state, LO, HI)
    r = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, [], z0=zl)
    np.testing.assert_allclose(r.state, lm.state, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r.cov, lm.cov, rtol=1e-9, atol=0)
    np.testing.assert_allclose(r.moments, lm.moments, rtol=1e-12)
    np.testing.assert_allclose(r.rrr, lm.rrr, rtol=1e-12)
    assert np.all((r.status & oracle.ST_COVSING) == (lm.status & oracle.ST_COVSING))


def test_paper_schedule_lowers_the_loss_and_flags_bad_pixels(scene):
    states = scenegen.config0_states(48)
    lobs = noisy_spectra(scene, states, 1, 0, 0)
    lobs[3, 10] = np.nan
    stages = oracle.paper_stages(1, LO, HI, X0)
    assert [s.steps for s in stages] == [30, 100]
    assert [s.lr for s in stages] == [0.03, 0.015]
    r = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, stages)
    start = oracle.adam_retrieve(scene, lobs, 1, LO, HI, X0, [])
    ok = np.isfinite(r.rrr)
    assert not ok[3] and r.status[3] & oracle.ST_NONFINITE and r.iters[3] == 0
    assert ok.sum() == 47
    assert np.all(r.rrr[ok] < start.rrr[ok])
    assert np.all(r.iters[ok] == 130)
    # saturation leaves too few bands: no solve
    tab = oracle.Tables(scene.lam, scene.K, scene.tau2, scene.tup, scene.ratm, scene.S,
                        np.full(scene.B, 1e-9, np.float32))
    nd = oracle.adam_retrieve(tab, lobs[:2], 1, LO, HI, X0, stages)
    assert np.all(nd.status & oracle.ST_NODOF) and np.all(np.isnan(nd.state))
