"""Pins of the oracle's full forward model (model 5; Sec. 2.2: the
eta-weighted smouldering and flaming Gaussians on the [350, 2200] K grid
over the five-endmember simplex surface of Sec. 2.4, the state the paper's
two Adam stages act on, Sec. 2.5): the reduction to the linear-surface
Gaussian-mixture model for a linear library, the Jacobian against finite
differences, the truth as a fixed point of the constrained LM on noise-free
spectra, the Karush-Kuhn-Tucker conditions of noisy solutions, one Adam
step by hand, and the stages' free sets against the paper's x_1 and x_2."""
import dataclasses

import numpy as np

import oracle
import scenegen

MODEL = 5
LO, HI, X0 = scenegen.default_prior(MODEL)
SF = oracle.simplex_first(MODEL)
K = oracle.N_ENDMEMBERS


def _tables(rho_atm=0.02, s_sph=0.1):
    atm = scenegen.make_atmosphere(7, 0, rho_atm=rho_atm, s_sph=s_sph)
    return oracle.band_tables(atm, scenegen.endmember_library(atm.hr_lambda_nm))


def _states(n, seed, f_lo=1e-2):
    X = scenegen.draw_states_full(scenegen.rng_for(7, seed, scenegen.STREAM_PARAMS), n)
    X[:, 0] = np.exp(np.random.default_rng(seed).uniform(np.log(f_lo), np.log(0.1), n))
    return X


def test_layout():
    assert oracle.n_state(MODEL) == 11 and SF == 6
    assert np.all(LO[SF:] == 0.0) and np.all(HI[SF:] == 1.0)
    np.testing.assert_allclose(X0[SF:].sum(), 1.0)


def test_linear_library_reduces_to_the_gaussian_mixture_model():
    """E_k = a_k + b_k (lambda - 1440 nm): model 5 equals model 3 with
    rho0 = sum x_k a_k, rho1 = sum x_k b_k, radiance and thermal columns,
    and d/dx_k = a_k d/drho0 + b_k d/drho1."""
    atm = scenegen.make_atmosphere(7, 0, rho_atm=0.03, s_sph=0.15)
    a = np.array([0.05, 0.3, 0.2, 0.12, 0.04])
    b = np.array([1e-4, -5e-5, 2e-5, 8e-5, 0.0])
    tab = oracle.band_tables(atm)
    tab = dataclasses.replace(tab, endm=np.ascontiguousarray(a[:, None] + b[:, None] * (tab.lam[None, :] - oracle.LAMBDA_REF_NM)))
    X = _states(6, 1)
    for q in (16, 32):
        L5, J5 = oracle.forward(tab, X, MODEL, q=q, jacobian=True)
        X3 = np.concatenate([X[:, :6], (X[:, SF:] @ a)[:, None], (X[:, SF:] @ b)[:, None]], axis=1)
        L3, J3 = oracle.forward(tab, X3, 3, q=q, jacobian=True)
        np.testing.assert_allclose(L5, L3, rtol=1e-13)
        np.testing.assert_allclose(J5[:, :, :6], J3[:, :, :6], rtol=1e-11, atol=1e-13 * np.abs(J3).max())
        want = J3[:, :, 6:7] * a[None, None, :] + J3[:, :, 7:8] * b[None, None, :]
        np.testing.assert_allclose(J5[:, :, SF:], want, rtol=1e-12, atol=1e-14)


def test_jacobian_against_central_differences():
    tab = _tables()
    x = np.array([[0.03, 0.4, 600.0, 90.0, 1250.0, 140.0, 0.3, 0.1, 0.25, 0.15, 0.2]])
    _, J = oracle.forward(tab, x, MODEL, jacobian=True)
    step = np.array([1e-6, 1e-6, 1e-3, 1e-3, 1e-3, 1e-3] + [1e-6] * 5)
    for j in range(11):
        xp, xm = x.copy(), x.copy()
        xp[0, j] += step[j]
        xm[0, j] -= step[j]
        fd = (oracle.forward(tab, xp, MODEL) - oracle.forward(tab, xm, MODEL))[0] / (2 * step[j])
        np.testing.assert_allclose(J[0, :, j], fd, rtol=2e-6, atol=1e-9 * np.abs(fd).max())


def test_truth_is_a_fixed_point_on_noise_free_spectra():
    """Started at the truth (z0), the constrained LM stays there and reports
    convergence: the truth is a stationary point of the masked loss with the
    simplex constraint, fractions at zero included."""
    tab = _tables()
    X = _states(24, 2)
    X[:8, SF + 1] = 0.0
    X[:, SF:] /= X[:, SF:].sum(axis=1, keepdims=True)
    L = oracle.forward(tab, X, MODEL)
    z0 = oracle.x_to_z(X, LO, HI)
    r = oracle.retrieve(tab, L.astype(np.float32), MODEL, LO, HI, X0, z0=z0, opts=oracle.LMOptions(max_iter=100))
    assert np.all(r.converged)
    assert np.all(r.rrr <= 1e-6)
    np.testing.assert_allclose(r.state[:, SF:], X[:, SF:], atol=1e-5)
    np.testing.assert_allclose(r.state[:, SF:].sum(axis=1), 1.0, atol=1e-14)
    et, _ = oracle.mixture_moments(X[:, 1], X[:, 4], X[:, 5], X[:, 2], X[:, 3])
    np.testing.assert_allclose(r.moments[:, 0], et, atol=0.5)


def test_noisy_solutions_satisfy_kkt():
    tab = _tables()
    X = _states(16, 3)
    L = oracle.forward(tab, X, MODEL)
    e = scenegen.noise_normals(7, 3, len(X), tab.B)
    lobs = (L * (1.0 + e / 300.0)).astype(np.float32)
    r = oracle.retrieve(tab, lobs, MODEL, LO, HI, X0, opts=oracle.LMOptions(max_iter=400, ftol=1e-13, ftol_undetected=1e-13, xtol=1e-12))
    checked = 0
    for p in range(len(X)):
        if not r.converged[p]:
            continue
        z = oracle.x_to_z(r.state[p], LO, HI)
        Lm, J = oracle.forward(tab, r.state[p][None, :], MODEL, jacobian=True)
        res = lobs[p].astype(np.float64) - Lm[0]
        Jz = J[0] * 0.5 * (HI - LO)
        F, g = float(res @ res), -2.0 * (Jz.T @ res)
        sc = 2.0 * np.sqrt(F) * np.linalg.norm(Jz, axis=0)
        pos = r.state[p, SF:] > 0
        lam = g[SF:][pos].mean()
        gs = g[SF:] - lam
        assert np.all(np.abs(gs[pos]) <= 1e-5 * sc[SF:][pos]), (p, gs)
        assert np.all(gs[~pos] >= -1e-5 * sc[SF:][~pos]), (p, gs)
        for j in range(SF):
            if -1.0 < z[j] < 1.0 and sc[j] > 0:
                assert abs(g[j]) <= 1e-5 * sc[j], (p, j, g[j], sc[j])
        checked += 1
    assert checked >= 6


def test_one_adam_step_by_hand():
    """Stage 1 starts with eta at 1 and the flaming spread at its lower bound
    (z_start), takes one t = 1 step lr g/(|g| + eps) on the free variables
    and projects the fractions onto the simplex."""
    tab = _tables()
    X = _states(3, 4)
    L = oracle.forward(tab, X, MODEL)
    lobs = L.astype(np.float32)
    st = dataclasses.replace(oracle.paper_stages(MODEL, LO, HI, X0)[0], steps=1, clip=0.0)
    r = oracle.adam_retrieve(tab, lobs, MODEL, LO, HI, X0, [st])
    z0 = oracle.x_to_z(X0, LO, HI)
    for j, v in st.zset.items():
        z0[j] = v
    for p in range(3):
        Lm, J = oracle.forward(tab, oracle.z_to_x(z0, LO, HI)[None, :], MODEL, jacobian=True)
        res = lobs[p].astype(np.float64) - Lm[0]
        g = -2.0 * (J[0].T @ res) * 0.5 * (HI - LO)       # stage 1 covers every band
        z1 = z0.copy()
        for j in st.free:
            z1[j] = np.clip(z0[j] - st.lr * g[j] / (abs(g[j]) + oracle.ADAM_EPS), -1, 1)
        z1[SF:] = 2.0 * oracle.project_simplex(0.5 * (z1[SF:] + 1.0)) - 1.0
        np.testing.assert_allclose(oracle.x_to_z(r.state[p], LO, HI), z1, atol=1e-12)


def test_stages_free_the_papers_state_vectors():
    s1, s2 = oracle.paper_stages(MODEL, LO, HI, X0)
    # x_1 = {x_surf, alpha_1, T_1}: f, the flaming mean (eta held at 1, its
    # spread at the lower bound) and the five fractions
    assert set(s1.free) == {0, 4} | set(range(SF, SF + K))
    assert s1.zset == {1: 1.0, 5: -1.0}
    # x_2 = {mu_hot, sig_hot, mu_smol, sig_smol, eta, alpha}, surface held
    assert set(s2.free) == {0, 1, 2, 3, 4, 5}
    assert s2.window[4] == s2.window[5] == oracle.OMEGA_HOT
    assert s2.window[2] == s2.window[3] == oracle.OMEGA_SMOL
    assert (s1.steps, s1.lr, s2.steps, s2.lr) == (30, 0.03, 100, 0.015)
