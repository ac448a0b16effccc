"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs (all device work goes through the C ABI).

Tolerances:
  FP64 kernels vs oracle  -- same arithmetic, different summation order and
                             exp/log implementations: forward 1e-11 norm-wise,
                             retrieved T within 1e-3 K, f within 1e-8.
  FP32-bulk vs oracle     -- the gate of _helpers.assert_parity: every
                             pixel both converge on ends at a fit as good as
                             the oracle's (loss at the GPU state, evaluated by
                             the oracle); at the same minimum, temperature
                             within 0.5 K and fire fraction within 1e-4 where
                             the data determine them, relative radiance
                             residual within 1e-5, posterior s.d. within 2 %.
"""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import CONVERGED, assert_parity, noisy_spectra

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def world(dev):
    atm = scenegen.make_atmosphere(0, 0)
    tab = oracle.band_tables(atm)
    scene = ff.Scene(atm)
    lo, hi, x0 = scenegen.default_prior(1)
    return atm, tab, scene, ff.Prior(1, lo, hi, x0)


@pytest.fixture(scope="module")
def cfg0(world, dev):
    """Config-0 style workload (1,000 px of the seeded 4,096) + oracle result."""
    atm, tab, scene, prior = world
    X = scenegen.config0_states(4096)[:1000]
    lobs = noisy_spectra(tab, X, 1, 0, 0)
    ref = oracle.retrieve(tab, lobs, 1, prior.lo, prior.hi, prior.x0)
    return X, lobs, ref


def _run(scene, lobs, prior, dev, **opt):
    out = ff.retrieve(scene, torch.from_numpy(np.ascontiguousarray(lobs)).to(dev), prior,
                      options=ff.default_options(**opt), state_f64=True)
    torch.cuda.synchronize()
    return out.numpy()


# --------------------------------------------------------------------------
def test_scene_tables(world):
    atm, tab, scene, _ = world
    T = scene.band_tables()
    np.testing.assert_allclose(T[:, 0], tab.lam, rtol=0, atol=0)
    for c, ref in [(1, tab.K), (2, tab.tau2), (3, tab.tup), (4, tab.ratm), (5, tab.S)]:
        np.testing.assert_allclose(T[:, c], ref, rtol=1e-13, atol=1e-300)
    assert np.all(np.isinf(T[:, 6]))


def test_scene_tables_with_atmosphere_terms(dev):
    atm = scenegen.make_atmosphere(0, 3, rho_atm=0.02, s_sph=0.15, cos_sza=0.7,
                                   sat_level=np.full(284, 5.0, np.float32))
    tab = oracle.band_tables(atm)
    T = ff.Scene(atm).band_tables()
    for c, ref in [(1, tab.K), (2, tab.tau2), (3, tab.tup), (4, tab.ratm), (5, tab.S)]:
        np.testing.assert_allclose(T[:, c], ref, rtol=1e-13)
    np.testing.assert_array_equal(T[:, 6], 5.0)


@pytest.mark.parametrize("model", [1, 2])
def test_forward_fp64(world, dev, model):
    atm, tab, scene, _ = world
    rng = np.random.default_rng(5 + model)
    X = (scenegen.draw_states_lognormal1 if model == 1 else scenegen.draw_states_lognormal2)(rng, 48)
    Lr, Jr = oracle.forward(tab, X, model, jacobian=True)
    L, J = ff.forward(scene, torch.tensor(X, device=dev), model, jacobian=True)
    L, J = L.cpu().numpy(), J.cpu().numpy()
    assert np.all(np.linalg.norm(L - Lr, axis=1) <= 1e-11 * np.linalg.norm(Lr, axis=1))
    for j in range(X.shape[1]):
        assert np.all(np.linalg.norm(J[:, :, j] - Jr[:, :, j], axis=1) <= 1e-11 * np.linalg.norm(Jr[:, :, j], axis=1) + 1e-300)


@pytest.mark.parametrize("model", [1, 2])
def test_forward_fp32(world, dev, model):
    atm, tab, scene, _ = world
    rng = np.random.default_rng(9 + model)
    X = (scenegen.draw_states_lognormal1 if model == 1 else scenegen.draw_states_lognormal2)(rng, 48)
    Lr, Jr = oracle.forward(tab, X, model, jacobian=True)
    L, J = ff.forward(scene, torch.tensor(X, dtype=torch.float32, device=dev), model, jacobian=True)
    L, J = L.cpu().double().numpy(), J.cpu().double().numpy()
    assert np.all(np.linalg.norm(L - Lr, axis=1) <= 2e-6 * np.linalg.norm(Lr, axis=1))
    for j in range(X.shape[1]):
        assert np.all(np.linalg.norm(J[:, :, j] - Jr[:, :, j], axis=1) <= 3e-6 * np.linalg.norm(Jr[:, :, j], axis=1))


@pytest.mark.parametrize("q", [16, 24])
def test_forward_lower_quadrature_order(world, dev, q):
    """Lower Gauss-Hermite orders on the FP32 path stay within 2e-5 of the
    32-node FP64 oracle for the workload's temperature ranges."""
    atm, tab, scene, _ = world
    X = scenegen.draw_states_lognormal1(np.random.default_rng(3), 64)
    Lr = oracle.forward(tab, X, 1)
    L = ff.forward(scene, torch.tensor(X, dtype=torch.float32, device=dev), 1, n_quad=q).cpu().double().numpy()
    rel = np.linalg.norm(L - Lr, axis=1) / np.linalg.norm(Lr, axis=1)
    assert rel.max() <= (2e-5 if q == 24 else 2e-4), rel.max()


@pytest.mark.parametrize("lpp", [1, 2, 8])
def test_retrieve_fp64_parity(world, dev, cfg0, lpp):
    X, lobs, ref = cfg0
    atm, tab, scene, prior = world
    r = _run(scene, lobs, prior, dev, precision=ff.PRECISION_FP64, lanes_per_pixel=lpp)
    conv = (r["status"].astype(np.int64) & CONVERGED) != 0
    assert (conv == ref.converged).mean() >= 0.995
    both = conv & ref.converged
    np.testing.assert_allclose(r["state_f64"][both, 1], ref.state[both, 1], atol=1e-3)
    np.testing.assert_allclose(r["state_f64"][both, 0], ref.state[both, 0], atol=1e-8)
    np.testing.assert_allclose(r["rrr"][both], ref.rrr[both], atol=1e-8, rtol=1e-6)
    np.testing.assert_array_equal(r["iters"][both] > 0, ref.iters[both] > 0)
    # moments to the state tolerance; covariance (sigma^2 A^-1: amplifies the
    # 1e-6 relative state differences by the condition number) on its
    # diagonal and correlations where the fire is well determined
    np.testing.assert_allclose(r["moments"][both], ref.moments[both], rtol=0, atol=1e-3)
    fin = both & (ref.state[:, 0] >= 1e-3) & ((ref.status & oracle.ST_COVSING) == 0)
    fin &= ((r["status"] & ff.ST_COV_SINGULAR) == 0)
    cg, cr = oracle.unpack_cov(r["cov"][fin], 5), oracle.unpack_cov(ref.cov[fin], 5)
    dg, dr = np.diagonal(cg, axis1=1, axis2=2), np.diagonal(cr, axis1=1, axis2=2)
    print("cov diag rel diff max", np.abs(dg / dr - 1).max())
    np.testing.assert_allclose(dg, dr, rtol=1e-3)
    corr_g = cg / np.sqrt(dg[:, :, None] * dg[:, None, :])
    corr_r = cr / np.sqrt(dr[:, :, None] * dr[:, None, :])
    np.testing.assert_allclose(corr_g, corr_r, atol=1e-4)


@pytest.mark.parametrize("acc,lpp", [(ff.ACCUMULATE_FP32, 1), (ff.ACCUMULATE_FP64, 1), (ff.ACCUMULATE_FP32, 2),
                                     (ff.ACCUMULATE_FP32, 4), (ff.ACCUMULATE_FP32, 16), (ff.ACCUMULATE_FP64, 64)])
def test_retrieve_fp32_parity(world, dev, cfg0, acc, lpp):
    X, lobs, ref = cfg0
    atm, tab, scene, prior = world
    r = _run(scene, lobs, prior, dev, accumulate=acc, lanes_per_pixel=lpp)
    rep = assert_parity(r, ref, tab=tab, lobs=lobs, min_t=700, label=f"acc {acc} lanes/pixel {lpp}")
    assert rep["both"] >= 0.95 * len(X)
    assert rep["same_frac"] >= 0.999


@pytest.mark.parametrize("lpp", [1, 4])
def test_schedules_and_block_sizes_are_bitwise_identical(world, dev, cfg0, lpp):
    X, lobs, ref = cfg0
    atm, tab, scene, prior = world
    base = _run(scene, lobs, prior, dev, lanes_per_pixel=lpp)
    for kw in [dict(schedule=ff.SCHEDULE_STATIC), dict(block_size=64), dict(block_size=128, blocks_per_cu=1)]:
        r = _run(scene, lobs, prior, dev, lanes_per_pixel=lpp, **kw)
        for k in ("state", "cov", "moments", "rrr", "iters", "status"):
            np.testing.assert_array_equal(r[k], base[k], err_msg=f"{kw} {k}")


def test_noise_free_recovery_fp32(world, dev):
    atm, tab, scene, prior = world
    X = scenegen.config0_states(512, scene=7)
    X = X[X[:, 0] >= 1e-3][:200]
    lobs = noisy_spectra(tab, X, 1, 0, 7, snr=None)
    r = _run(scene, lobs, prior, dev)
    conv = (r["status"] & CONVERGED) != 0
    assert conv.mean() >= 0.97
    assert np.all(r["rrr"][conv] <= 1e-5)
    assert np.abs(r["moments"][conv, 0] - X[conv, 1]).max() <= 0.5
    assert np.abs(r["state"][conv, 0] - X[conv, 0]).max() <= 1e-4


@pytest.mark.parametrize("lpp", [1, 16])
def test_edge_cases(world, dev, cfg0, lpp):
    X, lobs, ref = cfg0
    atm, tab, scene, prior = world
    # empty batch
    r = _run(scene, lobs[:0], prior, dev, lanes_per_pixel=lpp)
    assert r["state"].shape == (0, 5)
    with pytest.raises(ff.FirefitError):
        _run(scene, lobs[:4], prior, dev, lanes_per_pixel=3)
    # one pixel and a ragged count equal the corresponding rows of the full run
    full = _run(scene, lobs[:130], prior, dev, lanes_per_pixel=lpp)
    one = _run(scene, lobs[17:18], prior, dev, lanes_per_pixel=lpp)
    for k in ("state", "rrr", "iters", "status"):
        np.testing.assert_array_equal(one[k][0], full[k][17])
    rag = _run(scene, lobs[:65], prior, dev, lanes_per_pixel=lpp)
    np.testing.assert_array_equal(rag["state"], full["state"][:65])
    # non-finite input
    bad = lobs[:3].copy()
    bad[1, 100] = np.nan
    bad[2, 0] = np.inf
    r = _run(scene, bad, prior, dev, lanes_per_pixel=lpp)
    assert r["status"][1] == ff.ST_NONFINITE_INPUT and r["status"][2] == ff.ST_NONFINITE_INPUT
    assert np.isnan(r["state"][1:]).all() and np.isnan(r["rrr"][1:]).all() and (r["iters"][1:] == 0).all()
    np.testing.assert_array_equal(r["state"][0], full["state"][0])
    # no iterations allowed: the default start is returned with MAX_ITER
    # (z is held in FP64 on both paths; the FP32 path's state is then
    # rounded to float)
    for prec, tol in ((ff.PRECISION_FP64, 1e-14), (ff.PRECISION_FP32, 1e-14)):
        r = _run(scene, lobs[:8], prior, dev, max_iter=0, precision=prec, lanes_per_pixel=lpp)
        assert np.all((r["status"] & ff.ST_MAX_ITER) != 0) and np.all(r["iters"] == 0)
        np.testing.assert_allclose(r["state_f64"], np.tile(prior.x0, (8, 1)), rtol=tol, atol=1e-12)


def test_saturated_bands(dev):
    """Bands at or above the saturation level are masked (eq. loss); a pixel
    with every band saturated has no degrees of freedom."""
    atm = scenegen.make_atmosphere(0, 0)
    tab = oracle.band_tables(atm)
    X = scenegen.config0_states(64, scene=2)
    X = X[X[:, 0] > 1e-2][:16]
    lobs = noisy_spectra(tab, X, 1, 0, 2)
    sat = np.full(tab.B, np.float32(np.percentile(lobs, 90)), np.float32)
    atm.sat_level = sat
    tab = oracle.band_tables(atm)
    scene = ff.Scene(atm)
    lo, hi, x0 = scenegen.default_prior(1)
    prior = ff.Prior(1, lo, hi, x0)
    lobs[0, :] = sat[0] * 2
    ref = oracle.retrieve(tab, lobs, 1, lo, hi, x0)
    r = _run(scene, lobs, prior, dev, precision=ff.PRECISION_FP64)
    assert r["status"][0] == ff.ST_NO_DOF and ref.status[0] == oracle.ST_NODOF
    both = ((r["status"] & CONVERGED) != 0) & ref.converged
    np.testing.assert_allclose(r["state_f64"][both, 1], ref.state[both, 1], atol=1e-3)
    np.testing.assert_allclose(r["rrr"][both], ref.rrr[both], rtol=1e-6)


def test_batch_equals_single_scene_runs(dev):
    """A ragged multi-scene launch gives bitwise the per-scene results."""
    lo, hi, x0 = scenegen.default_prior(1)
    prior = ff.Prior(1, lo, hi, x0)
    scenes, rads, singles = [], [], []
    for s, P in enumerate([70, 1, 333]):
        atm = scenegen.make_atmosphere(4, s)
        tab = oracle.band_tables(atm)
        X = scenegen.config0_states(P, scene=10 + s)
        lobs = noisy_spectra(tab, X, 1, 4, s)
        sc = ff.Scene(atm)
        scenes.append(sc)
        rads.append(torch.from_numpy(lobs).to(dev))
        singles.append(_run(sc, lobs, prior, dev))
    outs = ff.retrieve_batch(scenes, rads, prior)
    torch.cuda.synchronize()
    for o, s1 in zip(outs, singles):
        o = o.numpy()
        for k in ("state", "cov", "rrr", "iters", "status"):
            np.testing.assert_array_equal(o[k], s1[k])


def test_batch_beyond_one_launch_equals_single_scene_runs(dev):
    """More scenes than one launch takes (16): the batch is split into
    launches of at most 16 scenes, each scene's outputs bitwise those of its
    own run; scenes of one and zero pixels included."""
    lo, hi, x0 = scenegen.default_prior(1)
    prior = ff.Prior(1, lo, hi, x0)
    sizes = [37, 1, 0, 90, 5, 64, 65, 3, 120, 17, 2, 33, 8, 71, 1, 44, 29, 12, 6, 50]
    scenes, rads, singles = [], [], []
    for s, P in enumerate(sizes):
        atm = scenegen.make_atmosphere(7, s % 5)
        tab = oracle.band_tables(atm)
        X = scenegen.config0_states(max(P, 1), scene=40 + s)[:P]
        lobs = noisy_spectra(tab, X, 1, 7, s) if P else np.zeros((0, tab.B), np.float32)
        sc = ff.Scene(atm)
        scenes.append(sc)
        rads.append(torch.from_numpy(np.ascontiguousarray(lobs)).to(dev))
        singles.append(_run(sc, lobs, prior, dev))
    outs = ff.retrieve_batch(scenes, rads, prior)
    torch.cuda.synchronize()
    assert len(outs) == len(sizes)
    for o, s1, P in zip(outs, singles, sizes):
        o = o.numpy()
        assert o["state"].shape[0] == P
        for k in ("state", "cov", "rrr", "iters", "status"):
            np.testing.assert_array_equal(o[k], s1[k])


@pytest.mark.parametrize("lpp", [1, 4])
def test_warm_start_and_fallback(world, dev, cfg0, lpp):
    """A per-pixel start z0: pixels that converge from it keep that result;
    pixels that do not are solved again from x0 and take that result when it
    converged or fits better (USED_FALLBACK), iterations summing both runs."""
    X, lobs, ref = cfg0
    atm, tab, scene, prior = world
    P = 200
    lo, hi = prior.lo, prior.hi
    z_true = np.clip(oracle.x_to_z(X[:P], lo, hi), -1, 1)
    z0 = z_true.copy()
    z0[1::2] = np.array([0.9, -0.95, 0.95, 0.9, 0.9])   # a poor start for odd pixels
    z0 = z0.astype(np.float32).astype(np.float64)          # the start the device receives
    opts = dict(max_iter=12)
    ref_warm = oracle.retrieve(tab, lobs[:P], 1, lo, hi, prior.x0, z0=z0, opts=oracle.LMOptions(max_iter=12))
    ref_cold = oracle.retrieve(tab, lobs[:P], 1, lo, hi, prior.x0, opts=oracle.LMOptions(max_iter=12))
    out = ff.retrieve(scene, torch.from_numpy(lobs[:P]).to(dev), prior,
                      z0=torch.tensor(z0, dtype=torch.float32, device=dev),
                      options=ff.default_options(precision=ff.PRECISION_FP64, lanes_per_pixel=lpp, **opts),
                      state_f64=True)
    torch.cuda.synchronize()
    r = out.numpy()
    st = r["status"].astype(np.int64)
    assert np.all(st & ff.ST_WARM_START)
    warm_ok = ref_warm.converged
    # the fallback is used exactly where the warm start failed and the
    # default-start run converged or fits better
    expect_fb = ~warm_ok & (ref_cold.converged | (ref_cold.rrr < ref_warm.rrr))
    agree = ((st & ff.ST_USED_FALLBACK) != 0) == expect_fb
    assert agree.mean() >= 0.98
    sel = agree & expect_fb
    np.testing.assert_allclose(r["state_f64"][sel, 1], ref_cold.state[sel, 1], atol=1e-3)
    np.testing.assert_array_equal(r["iters"][sel], ref_warm.iters[sel] + 1 + ref_cold.iters[sel])
    keep = agree & warm_ok
    np.testing.assert_allclose(r["state_f64"][keep, 1], ref_warm.state[keep, 1], atol=1e-3)
    # good starts need far fewer iterations than the plain default-start solve
    good = (np.arange(P) % 2 == 0) & ((st & ff.ST_USED_FALLBACK) == 0)
    assert r["iters"][good].mean() < 0.5 * ref.iters[:P][good].mean()


def test_two_component_model_parity(dev):
    """Eight-parameter smouldering + flaming mixture with fires of
    1e-3 <= f <= 0.05: FP64 follows the oracle (converged sets agree on
    >= 97 %; E[T] within 1e-2 K and f within 1e-7 on >= 90 % of the pixels
    both converge on -- the rest part along the mixture's flat valleys --
    and every pixel passes the loss checks); FP32 under the parity gate,
    with the flat-direction shortfall bounded (see the stress-set test)."""
    atm = scenegen.make_atmosphere(2, 0)
    tab = oracle.band_tables(atm)
    X = scenegen.config2_states(256)
    X[:, 0] = np.exp(np.random.default_rng(4).uniform(np.log(1e-3), np.log(0.05), len(X)))
    lobs = noisy_spectra(tab, X, 2, 2, 0)
    lo, hi, x0 = scenegen.default_prior(2)
    prior = ff.Prior(2, lo, hi, x0)
    scene = ff.Scene(atm)
    ref = oracle.retrieve(tab, lobs, 2, lo, hi, x0, opts=oracle.LMOptions(max_iter=200))
    r = _run(scene, lobs, prior, dev, precision=ff.PRECISION_FP64, max_iter=200)
    conv = (r["status"].astype(np.int64) & CONVERGED) != 0
    assert (conv == ref.converged).mean() >= 0.97
    both = conv & ref.converged
    close = (np.abs(r["moments"][:, 0] - ref.moments[:, 0]) <= 1e-2) & \
            (np.abs(r["state_f64"][:, 0] - ref.state[:, 0]) <= 1e-7)
    print("FP64: both", both.sum(), "close", (close & both).sum())
    assert (close & both).sum() >= 0.9 * both.sum()
    assert_parity(r, ref, model=2, tab=tab, lobs=lobs, min_same=0.97, min_t=0, label="n=8 FP64")
    for acc in (ff.ACCUMULATE_FP32, ff.ACCUMULATE_FP64):
        r32 = _run(scene, lobs, prior, dev, accumulate=acc, max_iter=200)
        rep = assert_parity(r32, ref, model=2, tab=tab, lobs=lobs, min_same=0.9, min_t=0,
                            label=f"n=8 acc {acc}", flat_worse_frac=0.02)
        assert rep["both"] >= 150


def test_stress_set_as_specified(dev):
    """The precision stress set as drawn: two-component (smouldering +
    flaming lognormal, eight variables) states with 1e-5 <= f <= 1e-3, a
    seeded 2,048-pixel subsample of the 262,144 pixels, through FP32 bulk,
    FP32 with FP64 accumulation and all-FP64 against the oracle on the same
    radiance, at most 200 iterations on both sides (the eight-variable
    mixture walks its flat valleys longer than the one-component model).
    At these fractions nothing but the fit is determined: the oracle's
    posterior s.d. of E[T] exceeds 2e4 K and of f exceeds 1e-3 on every
    pixel (the area-temperature degeneracy), so no pixel qualifies for a
    value comparison and the gate is the loss check, in distribution along
    the flat directions.  FP64 follows the oracle's trajectory: E[T] within
    1e-2 K, f within 1e-7 and the residual within 1e-8 on >= 90 % of the
    pixels both converge on (the rest part along flat valleys after up to
    200 iterations, where the summation order's rounding is enough to take
    another path); every pixel passes the loss checks."""
    atm = scenegen.make_atmosphere(2, 0)
    tab = oracle.band_tables(atm)
    Xall = scenegen.config2_states(262144)
    idx = scenegen.subsample(2, 0, len(Xall), 2048)
    X = Xall[idx]
    assert X[:, 0].min() >= 1e-5 and X[:, 0].max() <= 1e-3
    lobs = noisy_spectra(tab, X, 2, 2, 0)
    lo, hi, x0 = scenegen.default_prior(2)
    prior = ff.Prior(2, lo, hi, x0)
    scene = ff.Scene(atm)
    ref = oracle.retrieve(tab, lobs, 2, lo, hi, x0, opts=oracle.LMOptions(max_iter=200))
    print("oracle converged", ref.converged.mean(), "mean iterations", ref.iters.mean())
    r64 = _run(scene, lobs, prior, dev, precision=ff.PRECISION_FP64, max_iter=200)
    conv = (r64["status"].astype(np.int64) & CONVERGED) != 0
    assert (conv == ref.converged).mean() >= 0.98
    both = conv & ref.converged
    close = (np.abs(r64["moments"][:, 0] - ref.moments[:, 0]) <= 1e-2) & \
            (np.abs(r64["state_f64"][:, 0] - ref.state[:, 0]) <= 1e-7) & (np.abs(r64["rrr"] - ref.rrr) <= 1e-8)
    print("FP64: both", both.sum(), "close", (close & both).sum())
    assert (close & both).sum() >= 0.9 * both.sum()
    assert_parity(r64, ref, model=2, tab=tab, lobs=lobs, min_same=0.99, min_t=0, label="stress set FP64")
    for acc in (ff.ACCUMULATE_FP32, ff.ACCUMULATE_FP64):
        r32 = _run(scene, lobs, prior, dev, accumulate=acc, lanes_per_pixel=4, max_iter=200)
        # along the flat directions the FP32 thermal term's rounding (~1e-3
        # chi^2 units of F) steers the solve: it ends worse than the oracle
        # somewhat more often than better (measured at 1e-3 / 0.1 / 1 chi^2:
        # 229 / 30 / 6 worse against 185 / 17 / 1 better of 1,567); bounded
        rep = assert_parity(r32, ref, model=2, tab=tab, lobs=lobs, min_same=0.9, min_t=0,
                            label=f"stress set FP32 acc {acc}", flat_worse_frac=0.01)
        c32 = (r32["status"].astype(np.int64) & CONVERGED) != 0
        assert c32.mean() >= ref.converged.mean() - 0.02
        assert rep["both"] >= 0.5 * len(X)
        # errors per output on the pixels both converge on
        b = rep["both_mask"]
        for name, g, o in (("E[T]", r32["moments"][:, 0], ref.moments[:, 0]),
                           ("sigma[T]", r32["moments"][:, 1], ref.moments[:, 1]),
                           ("f", r32["state"][:, 0], ref.state[:, 0]), ("rrr", r32["rrr"], ref.rrr)):
            e = np.abs(g - o)[b]
            print(f"  {name}: median {np.median(e):.3g} p99 {np.percentile(e, 99):.3g} max {e.max():.3g}")


@pytest.mark.parametrize("lpp", [1, 4])
def test_start_rows_without_a_start(world, dev, cfg0, lpp):
    """A start row whose first entry is NaN carries no start: those pixels
    are solved bitwise as without z0 (no fallback, no FF_ST_WARM_START); the
    others as a warm-started retrieval of those rows alone."""
    X, lobs, ref = cfg0
    atm, tab, scene, prior = world
    P = 300
    z = np.clip(oracle.x_to_z(X[:P], prior.lo, prior.hi), -1, 1).astype(np.float32)
    none = np.arange(P) % 3 == 0
    z[none] = np.nan
    opts = ff.default_options(lanes_per_pixel=lpp)
    mixed = ff.retrieve(scene, torch.from_numpy(lobs[:P]).to(dev), prior,
                        z0=torch.from_numpy(z).to(dev), options=opts).numpy()
    plain = _run(scene, lobs[:P][none], prior, dev, lanes_per_pixel=lpp)
    warm = ff.retrieve(scene, torch.from_numpy(np.ascontiguousarray(lobs[:P][~none])).to(dev), prior,
                       z0=torch.from_numpy(np.ascontiguousarray(z[~none])).to(dev), options=opts).numpy()
    torch.cuda.synchronize()
    for k in ("state", "cov", "moments", "rrr", "iters", "status"):
        np.testing.assert_array_equal(mixed[k][none], plain[k], err_msg=k)
        np.testing.assert_array_equal(mixed[k][~none], warm[k], err_msg=k)
    assert np.all((mixed["status"][none] & ff.ST_WARM_START) == 0)
    assert np.all((mixed["status"][~none] & ff.ST_WARM_START) != 0)
