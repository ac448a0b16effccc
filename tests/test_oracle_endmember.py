"""Pins of the oracle's endmember surface (model 4; Sec. 2.2 and Sec. 2.4:
reflectance as a mixture of five library spectra with fractions on the unit
simplex, projected back onto it after each optimiser step, Sec. 2.5): the
projection against brute force over supports, the forward model against
the linear-reflectance model it reduces to, the Jacobian against finite
differences, noise-free recovery (fractions at zero included), the
Karush-Kuhn-Tucker conditions of the constrained LM solution and an
independent SQP solve of the same problem, and one Adam step by hand."""
import dataclasses
import itertools

import numpy as np
import pytest
from scipy import optimize

import oracle
import scenegen

LO, HI, X0 = scenegen.default_prior(4)
SF = oracle.SIMPLEX_FIRST
K = oracle.N_ENDMEMBERS


def _tables(rho_atm=0.02, s_sph=0.1, endm=None):
    atm = scenegen.make_atmosphere(0, 0, rho_atm=rho_atm, s_sph=s_sph)
    if endm is None:
        endm = scenegen.endmember_library(atm.hr_lambda_nm)
    return oracle.band_tables(atm, endm)


def _brute_projection(v):
    """Nearest point of the simplex: for every support S the minimiser of
    |x - v|^2 on {sum x = 1, x_i = 0 off S} is v_S - (sum v_S - 1)/|S|;
    among the feasible candidates take the nearest."""
    best, bd = None, np.inf
    n = len(v)
    for r in range(1, n + 1):
        for S in itertools.combinations(range(n), r):
            x = np.zeros(n)
            S = list(S)
            x[S] = v[S] - (v[S].sum() - 1.0) / len(S)
            if np.all(x >= -1e-15):
                d = np.sum((x - v) ** 2)
                if d < bd:
                    best, bd = np.maximum(x, 0.0), d
    return best


def test_projection_matches_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(300):
        v = rng.normal(0.2, 0.6, K)
        np.testing.assert_allclose(oracle.project_simplex(v), _brute_projection(v), atol=1e-14)
    x = rng.dirichlet(np.ones(K))
    np.testing.assert_allclose(oracle.project_simplex(x), x, atol=1e-16)   # a fixed point
    np.testing.assert_allclose(oracle.project_simplex(np.full(K, 7.0)), np.full(K, 0.2), atol=1e-15)
    e = oracle.project_simplex(np.array([3.0, -1.0, 0.5, 0.0, 2.0]))
    np.testing.assert_allclose(e, [1.0, 0.0, 0.0, 0.0, 0.0], atol=1e-15)


def test_linear_library_reduces_to_linear_reflectance():
    """With E_k = a_k + b_k (lambda - 1440 nm) the mixture is the linear
    reflectance rho0 = sum x_k a_k, rho1 = sum x_k b_k of model 1: radiance
    and the thermal Jacobian columns agree, and d/dx_k = a_k d/drho0 +
    b_k d/drho1."""
    atm = scenegen.make_atmosphere(0, 0, rho_atm=0.03, s_sph=0.15)
    a = np.array([0.05, 0.3, 0.2, 0.12, 0.04])
    b = np.array([1e-4, -5e-5, 2e-5, 8e-5, 0.0])
    tab = oracle.band_tables(atm)
    endm = a[:, None] + b[:, None] * (tab.lam[None, :] - oracle.LAMBDA_REF_NM)   # band level
    tab = dataclasses.replace(tab, endm=np.ascontiguousarray(endm))
    rng = np.random.default_rng(3)
    for _ in range(4):
        xs = rng.dirichlet(np.ones(K))
        th = [10 ** rng.uniform(-4, -1), rng.uniform(600, 1400), rng.uniform(50, 300)]
        x4 = np.array([th + list(xs)])
        x1 = np.array([th + [xs @ a, xs @ b]])
        L4, J4 = oracle.forward(tab, x4, 4, jacobian=True)
        L1, J1 = oracle.forward(tab, x1, 1, jacobian=True)
        np.testing.assert_allclose(L4, L1, rtol=1e-13)
        np.testing.assert_allclose(J4[0, :, :3], J1[0, :, :3], rtol=1e-12)
        want = J1[0, :, 3:4] * a[None, :] + J1[0, :, 4:5] * b[None, :]
        np.testing.assert_allclose(J4[0, :, SF:], want, rtol=1e-12, atol=1e-14)


def test_library_resampling_keeps_constants_and_is_the_atmosphere_srf():
    atm = scenegen.make_atmosphere(0, 0)
    H = atm.hr_lambda_nm.size
    const = np.array([0.1, 0.2, 0.3, 0.4, 0.5])[:, None] * np.ones((1, H))
    tab = oracle.band_tables(atm, const)
    np.testing.assert_allclose(tab.endm, const[:, :tab.B], rtol=1e-14)
    lib = scenegen.endmember_library(atm.hr_lambda_nm)
    W = oracle.srf_matrix(atm.wavelength_nm, atm.fwhm_nm, atm.hr_lambda_nm)
    np.testing.assert_allclose(oracle.band_tables(atm, lib).endm, lib @ W.T, rtol=1e-14)


def test_jacobian_against_central_differences():
    tab = _tables()
    x = np.array([[0.02, 950.0, 140.0, 0.3, 0.1, 0.25, 0.15, 0.2]])
    _, J = oracle.forward(tab, x, 4, jacobian=True)
    step = np.array([1e-6, 1e-3, 1e-3, 1e-6, 1e-6, 1e-6, 1e-6, 1e-6])
    for j in range(8):
        xp, xm = x.copy(), x.copy()
        xp[0, j] += step[j]
        xm[0, j] -= step[j]
        fd = (oracle.forward(tab, xp, 4) - oracle.forward(tab, xm, 4))[0] / (2 * step[j])
        np.testing.assert_allclose(J[0, :, j], fd, rtol=2e-6, atol=1e-9 * np.abs(fd).max())


def test_model4_needs_endmembers_and_unit_fraction_boxes():
    tab = _tables()
    bare = dataclasses.replace(tab, endm=None)
    with pytest.raises(ValueError):
        oracle.forward(bare, np.array([X0]), 4)
    L = oracle.forward(tab, np.array([X0]), 4).astype(np.float32)
    hi = HI.copy()
    hi[SF] = 0.9
    with pytest.raises(ValueError):
        oracle.retrieve(tab, L, 4, LO, hi, X0)


def _truth(n, seed):
    X = scenegen.draw_states_endmember1(scenegen.rng_for(40, seed, scenegen.STREAM_PARAMS), n)
    X[: n // 2, 3] = 0.0                     # half the pixels with one or two
    X[: n // 4, 6] = 0.0                     # fractions exactly at zero
    X[:, SF:] /= X[:, SF:].sum(axis=1, keepdims=True)
    return X


def test_noise_free_recovery_including_zero_fractions():
    tab = _tables()
    X = _truth(48, 0)
    L = oracle.forward(tab, X, 4).astype(np.float32)
    r = oracle.retrieve(tab, L, 4, LO, HI, X0, opts=oracle.LMOptions(max_iter=200))
    assert np.all(r.converged)
    np.testing.assert_allclose(r.state[:, SF:].sum(axis=1), 1.0, atol=1e-14)
    assert np.all(r.state[:, SF:] >= 0.0)
    np.testing.assert_allclose(r.state[:, SF:], X[:, SF:], atol=2e-5)
    np.testing.assert_allclose(r.state[:, 1], X[:, 1], rtol=1e-4)
    np.testing.assert_allclose(r.state[:, 0], X[:, 0], rtol=1e-3)
    # fractions that are zero in truth stay within float32 rounding of zero
    assert np.all(r.state[:24, 3] <= 1e-6) and np.all(r.state[:12, 6] <= 1e-6)


def _noisy(n, seed):
    tab = _tables()
    X = _truth(n, seed)
    L = oracle.forward(tab, X, 4)
    e = scenegen.noise_normals(40, seed, n, tab.B)
    return tab, X, (L * (1.0 + e / 300.0)).astype(np.float32)


def _loss_grad_z(tab, lobs, z, scale=False):
    """F(z) = sum (L_obs - L)^2 over all bands and dF/dz, from the forward
    model and its Jacobian (finite-difference pinned above); with ``scale``
    also 2 sqrt(F) |dL/dz_j|, the size a gradient component takes when the
    residual is not orthogonal to that column."""
    x = oracle.z_to_x(z, LO, HI)
    L, J = oracle.forward(tab, x[None, :], 4, jacobian=True)
    r = lobs.astype(np.float64) - L[0]
    Jz = J[0] * 0.5 * (HI - LO)
    F, g = float(r @ r), -2.0 * (Jz.T @ r)
    if scale:
        return F, g, 2.0 * np.sqrt(F) * np.linalg.norm(Jz, axis=0)
    return F, g


def test_constrained_solution_satisfies_kkt():
    """At the LM solution: interior box variables have zero gradient, the
    positive fractions share one gradient value lambda, and a fraction at
    zero has gradient >= lambda (moving weight onto it cannot help); zero
    means small against each component's natural scale 2 sqrt(F) |dL/dz_j|."""
    tab, X, lobs = _noisy(12, 1)
    r = oracle.retrieve(tab, lobs, 4, LO, HI, X0, opts=oracle.LMOptions(max_iter=300, ftol=1e-13, ftol_undetected=1e-13, xtol=1e-12))
    checked = 0
    tol = 1e-6
    for p in range(len(X)):
        if not r.converged[p]:
            continue
        z = oracle.x_to_z(r.state[p], LO, HI)
        F, g, sc = _loss_grad_z(tab, lobs[p], z, scale=True)
        pos = r.state[p, SF:] > 0
        lam = g[SF:][pos].mean()
        gs, ss = g[SF:] - lam, sc[SF:]
        assert np.all(np.abs(gs[pos]) <= tol * ss[pos]), (p, gs, ss)
        assert np.all(gs[~pos] >= -tol * ss[~pos]), (p, gs, ss)
        for j in range(SF):
            if -1.0 < z[j] < 1.0:
                assert abs(g[j]) <= tol * sc[j], (p, j, g[j], sc[j])
        checked += 1
    assert checked >= 8


def test_sqp_from_the_lm_solution_finds_nothing_better():
    """An independent solver (scipy SLSQP with the simplex as an equality
    constraint and the box as bounds) started at the LM solution cannot
    lower the loss by more than rounding, and started at the prior start
    reaches no lower loss than LM."""
    tab, X, lobs = _noisy(6, 2)
    r = oracle.retrieve(tab, lobs, 4, LO, HI, X0, opts=oracle.LMOptions(max_iter=300))
    cons = {"type": "eq", "fun": lambda z: 0.5 * (z[SF:] + 1.0).sum() - 1.0,
            "jac": lambda z: np.r_[np.zeros(SF), np.full(K, 0.5)]}
    for p in range(len(X)):
        z_lm = oracle.x_to_z(r.state[p], LO, HI)
        F_lm, _ = _loss_grad_z(tab, lobs[p], z_lm)

        def fun(z):
            return _loss_grad_z(tab, lobs[p], np.clip(z, -1, 1))

        for start, slack in [(z_lm, 1e-7), (oracle.x_to_z(X0, LO, HI), 1e-4)]:
            res = optimize.minimize(fun, start, jac=True, method="SLSQP", bounds=[(-1, 1)] * 8,
                                    constraints=[cons], options={"maxiter": 500, "ftol": 1e-16})
            zs = np.clip(res.x, -1, 1)
            zs[SF:] = 2.0 * oracle.project_simplex(0.5 * (zs[SF:] + 1.0)) - 1.0
            F_sqp, _ = _loss_grad_z(tab, lobs[p], zs)
            assert F_lm <= F_sqp * (1.0 + slack), (p, F_lm, F_sqp)


def test_one_adam_step_by_hand():
    """One Adam step (t = 1: m_hat = g, v_hat = g^2) with no clip from the
    prior start: z_1 = clip(z_0 - lr g / (|g| + eps)) on the free variables,
    then the fractions projected onto the simplex."""
    tab, X, lobs = _noisy(3, 3)
    stage = dataclasses.replace(oracle.paper_stages(4, LO, HI, X0)[0], steps=1, clip=0.0, zset=None)
    r = oracle.adam_retrieve(tab, lobs, 4, LO, HI, X0, [stage])
    z0 = oracle.x_to_z(X0, LO, HI)
    for p in range(3):
        _, g = _loss_grad_z(tab, lobs[p], z0)      # stage 1's window covers every band
        z1 = z0.copy()
        for j in stage.free:
            z1[j] = np.clip(z0[j] - stage.lr * g[j] / (abs(g[j]) + oracle.ADAM_EPS), -1, 1)
        z1[SF:] = 2.0 * oracle.project_simplex(0.5 * (z1[SF:] + 1.0)) - 1.0
        np.testing.assert_allclose(oracle.x_to_z(r.state[p], LO, HI), z1, atol=1e-12)
        np.testing.assert_allclose(r.state[p, SF:].sum(), 1.0, atol=1e-14)


def test_paper_stages_for_the_endmember_surface():
    s1, s2 = oracle.paper_stages(4, LO, HI, X0)
    assert (s1.steps, s1.lr, s2.steps, s2.lr) == (30, 0.03, 100, 0.015)
    assert set(s1.free) == {0, 1, 3, 4, 5, 6, 7} and s1.zset == {2: -1.0}
    assert set(s2.free) == {0, 1, 2}
    assert all(s1.window[j] == oracle.OMEGA_1 for j in s1.free)
    assert all(s2.window[j] == oracle.OMEGA_2 for j in s2.free)
