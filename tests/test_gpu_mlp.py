"""GPU parity and gain of the learned warm start (network kernels through the
C ABI against the FP64 oracle in oracle/mlp.py).

Tolerances:
  generator    -- states and targets are FP64 draws stored as float32
                  (relative 1e-6); radiance is the FP32 forward model with
                  FP32 Box-Muller noise: 1e-5 norm-wise per spectrum.
  inference    -- against the oracle with the same BF16 storage of layer
                  inputs and weights the only differences are FP32 summation
                  order and the rare BF16 rounding tie it flips: |dz| <= 2e-3.
                  Against the plain FP64 network: BF16 keeps 8 significant
                  bits (relative rounding 2^-9 per stored value), so 2e-2
                  norm-wise.
  gradients    -- products of BF16-stored activations, weights and output
                  errors summed in FP32: 2e-2 norm-wise per layer and a
                  cosine >= 0.999 with the FP64 gradient.
  Adam         -- the first step from zero moments moves each weight by
                  lr * g / (|g| + eps); where the FP64 gradient is
                  clearly signed that is -lr * sign(g) to FP32 rounding.
"""
import time

import numpy as np
import pytest

import oracle
import scenegen
from _helpers import CONVERGED, assert_parity, noisy_spectra
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402

SIZES = (284, 512, 512, 256, 5)


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
    return tab, scene, ff.Prior(1, lo, hi, x0)


@pytest.fixture(scope="module")
def probe(world):
    """Oracle-made spectra, oracle initial weights and normalisation."""
    tab, _, prior = world
    rad, tgt, _ = omlp.generate(tab, prior.lo, prior.hi, prior.x0, 21, 5000, 1024, bg_fraction=0.2)
    feats = omlp.features(rad, 0.0, 1.0, 1e-6)
    mean = feats.mean(0).astype(np.float32)
    inv = (1.0 / feats.std(0)).astype(np.float32)
    p = omlp.init_params(SIZES, 17).astype(np.float32)
    return rad, tgt.astype(np.float32), mean, inv, p


def _net(probe):
    _, _, mean, inv, p = probe
    net = ff.WarmStart(seed=3)
    net.set_params(p)
    net.set_normalization(mean, inv, 1e-6)
    return net


@pytest.mark.parametrize("bg", [0.0, 0.25])
def test_generator_matches_oracle(world, dev, bg):
    tab, scene, prior = world
    P = 3000
    rad, tgt, st = ff.generate(scene, prior, 11, 123456789, P, bg_fraction=bg, states=True)
    torch.cuda.synchronize()
    orad, otgt, ost = omlp.generate(tab, prior.lo, prior.hi, prior.x0, 11, 123456789, P, bg_fraction=bg)
    st = st.cpu().double().numpy()
    np.testing.assert_array_equal(st[:, 0] == 0.0, ost[:, 0] == 0.0)
    np.testing.assert_allclose(st, ost, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(tgt.cpu().double().numpy(), otgt, rtol=0, atol=1e-6)
    g = rad.cpu().double().numpy()
    rel = np.linalg.norm(g - orad, axis=1) / np.linalg.norm(orad, axis=1)
    assert rel.max() < 1e-5, rel.max()
    # noise-free spectra are the plain forward model of the drawn states
    rad0, _ = ff.generate(scene, prior, 11, 123456789, 256, snr=0.0, bg_fraction=bg)
    L = oracle.forward(tab, ost[:256], 1)
    rel0 = np.linalg.norm(rad0.cpu().double().numpy() - L, axis=1) / np.linalg.norm(L, axis=1)
    assert rel0.max() < 1e-5, rel0.max()


def test_fit_normalization(world, dev, probe):
    rad = probe[0]
    net = ff.WarmStart(seed=1)
    net.fit_normalization(torch.from_numpy(rad).to(dev), floor=1e-6)
    torch.cuda.synchronize()
    mean, inv, fl = net.get_normalization()
    v = np.log(np.maximum(rad.astype(np.float64), 1e-6))
    np.testing.assert_allclose(mean, v.mean(0), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(inv, 1.0 / v.std(0), rtol=1e-4)
    assert fl == np.float32(1e-6)


def test_inference_matches_oracle(world, dev, probe):
    rad, _, mean, inv, p = probe
    net = _net(probe)
    z = net.infer(torch.from_numpy(rad).to(dev)).cpu().double().numpy()
    X = omlp.features(rad, mean.astype(np.float64), inv.astype(np.float64), np.float64(np.float32(1e-6)))
    zq, _ = omlp.forward(p.astype(np.float64), SIZES, X, bf16_storage=True)
    assert np.abs(z - zq).max() < 2e-3, np.abs(z - zq).max()
    z64, _ = omlp.forward(p.astype(np.float64), SIZES, X)
    assert np.linalg.norm(z - z64) / np.linalg.norm(z64) < 2e-2
    # a row's result does not depend on the rows batched with it
    z2 = net.infer(torch.from_numpy(rad[100:357]).to(dev)).cpu().double().numpy()
    np.testing.assert_allclose(z2, z[100:357], rtol=0, atol=1e-6)


def test_inference_empty_and_ragged(world, dev, probe):
    net = _net(probe)
    z = net.infer(torch.empty((0, 284), dtype=torch.float32, device=dev))
    assert z.shape == (0, 5)
    rad = probe[0]
    for P in (1, 63, 65, 1000):
        zp = net.infer(torch.from_numpy(rad[:P]).to(dev)).cpu().numpy()
        zf = net.infer(torch.from_numpy(rad).to(dev)).cpu().numpy()[:P]
        np.testing.assert_allclose(zp, zf, rtol=0, atol=1e-6)


@pytest.mark.parametrize("n_in", [283, 281, 7])
def test_inference_input_widths_not_a_multiple_of_four(dev, n_in):
    """Widths that are not a multiple of 4 take the features kernel's
    element-wise path (rows not 16-byte aligned), with a padded tail up to
    the next multiple of 32; a hidden width of 64 takes the 64-wide GEMM."""
    sizes = (n_in, 128, 128, 64, 5)
    rng = np.random.default_rng(n_in)
    rad = rng.lognormal(-3.0, 1.0, (700, n_in)).astype(np.float32)
    feats = omlp.features(rad, 0.0, 1.0, 1e-6)
    mean = feats.mean(0).astype(np.float32)
    inv = (1.0 / feats.std(0)).astype(np.float32)
    p = omlp.init_params(sizes, 5).astype(np.float32)
    net = ff.WarmStart(n_in=n_in, hidden=sizes[1:4], n_out=5, seed=1)
    net.set_params(p)
    net.set_normalization(mean, inv, 1e-6)
    z = net.infer(torch.from_numpy(rad).to(dev)).cpu().double().numpy()
    X = omlp.features(rad, mean.astype(np.float64), inv.astype(np.float64), np.float64(np.float32(1e-6)))
    zq, _ = omlp.forward(p.astype(np.float64), sizes, X, bf16_storage=True)
    assert np.abs(z - zq).max() < 2e-3, np.abs(z - zq).max()


def test_listed_inference_across_chunks(world, dev, probe):
    """More listed rows than one 262,144-row chunk, in a random order: every
    listed row equals the full inference's, the others stay untouched."""
    net = _net(probe)
    big = torch.from_numpy(np.tile(probe[0], (60, 1))).to(dev)         # 300,000 rows
    P = big.shape[0]
    perm = np.random.default_rng(3).permutation(P)[:(1 << 18) + 1234]
    idx = torch.from_numpy(perm.astype(np.int64)).to(dev)
    full = net.infer(big).cpu().numpy()
    z0 = torch.full((P, 5), -7.0, dtype=torch.float32, device=dev)
    net.infer_listed(big, idx, len(perm), z0=z0)
    torch.cuda.synchronize()
    got = z0.cpu().numpy()
    np.testing.assert_array_equal(got[perm], full[perm])
    rest = np.setdiff1d(np.arange(P), perm)
    assert np.all(got[rest] == -7.0)


def test_gradients_match_oracle(world, dev, probe):
    rad, tgt, mean, inv, p = probe
    net = _net(probe)
    loss, g = net.gradients(torch.from_numpy(rad).to(dev), torch.from_numpy(tgt).to(dev))
    torch.cuda.synchronize()
    X = omlp.features(rad, mean.astype(np.float64), inv.astype(np.float64), np.float64(np.float32(1e-6)))
    lref, gref = omlp.loss_and_grads(p.astype(np.float64), SIZES, X, tgt.astype(np.float64))
    assert abs(loss.item() - lref) <= 2e-2 * lref
    g = g.cpu().double().numpy()
    off = 0
    for l, (o, i) in enumerate(omlp.layer_shapes(*SIZES)):
        for n in (o * i, o):
            a, b = g[off:off + n], gref[off:off + n]
            off += n
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            assert rel < 2e-2 and cos > 0.999, (l, n, rel, cos)
    assert off == g.size


def test_adam_first_step(world, dev, probe):
    rad, tgt, mean, inv, p = probe
    net = _net(probe)
    lr = 1e-3
    net.train_step(torch.from_numpy(rad).to(dev), torch.from_numpy(tgt).to(dev), lr)
    torch.cuda.synchronize()
    p1 = net.get_params().astype(np.float64)
    X = omlp.features(rad, mean.astype(np.float64), inv.astype(np.float64), np.float64(np.float32(1e-6)))
    _, gref = omlp.loss_and_grads(p.astype(np.float64), SIZES, X, tgt.astype(np.float64))
    step = p1 - p.astype(np.float64)
    # every weight moves by at most lr (|g| / (|g| + eps) < 1)
    assert np.abs(step).max() <= lr * (1 + 1e-5) + 1e-6
    off = 0
    for o, i in omlp.layer_shapes(*SIZES):
        n = o * i + o
        gl, sl = gref[off:off + n], step[off:off + n]
        off += n
        clear = np.abs(gl) > 0.2 * np.sqrt(np.mean(gl * gl))
        assert clear.mean() > 0.3
        np.testing.assert_allclose(sl[clear], -lr * np.sign(gl[clear]), rtol=0, atol=lr * 1e-3 + 2e-7)


@pytest.fixture(scope="module")
def trained(world, dev):
    """A network trained on the scene's own generated spectra (fire only)."""
    _, scene, prior = world
    net = ff.WarmStart(seed=1)
    nrad, _ = ff.generate(scene, prior, 999, 0, 16384)
    net.fit_normalization(nrad)
    t0 = time.perf_counter()
    hist = net.train(scene, prior, steps=1500, batch=2048, seed=2, lr=1e-3, lr_final=1e-5)
    torch.cuda.synchronize()
    h = hist.cpu().numpy()
    print(f"\n  trained 1500 x 2048 in {time.perf_counter() - t0:.2f} s; "
          f"loss {h[:20].mean():.4g} -> {h[-50:].mean():.4g}")
    return net, h


def test_training_reduces_loss(world, dev, trained):
    tab, _, prior = world
    net, h = trained
    assert np.all(np.isfinite(h))
    assert h[-50:].mean() < 0.1 * h[:20].mean()
    # held-out oracle-made spectra: the network beats the default start by far
    rad, tgt, _ = omlp.generate(tab, prior.lo, prior.hi, prior.x0, 4242, 0, 2000)
    z = net.infer(torch.from_numpy(rad).to(dev)).cpu().double().numpy()
    zdef = np.clip(oracle.x_to_z(np.asarray(prior.x0)[None, :], prior.lo, prior.hi), -1, 1)
    err_net = np.sqrt(np.mean((z - tgt) ** 2, axis=0))
    err_def = np.sqrt(np.mean((zdef - tgt) ** 2, axis=0))
    print("  held-out rms z error: network", np.round(err_net, 4), "default start", np.round(err_def, 4))
    assert np.all(err_net[:3] < 0.3 * err_def[:3])
    assert np.mean((z - tgt) ** 2) < 0.05 * np.mean((zdef - tgt) ** 2)


def _run(scene, rad, prior, z0, dev):
    ev = torch.zeros(1, dtype=torch.int64, device=dev)
    out = ff.retrieve(scene, rad, prior, z0=z0, evals=ev)
    torch.cuda.synchronize()
    return out.numpy(), int(ev.item())


def test_warm_start_gain_fire_pixels(world, dev, trained):
    """What the network gains: fewer LM iterations and evaluations at the
    oracle's accuracy."""
    tab, scene, prior = world
    net, _ = trained
    X = scenegen.config0_states(4096, scene=5)
    lobs = noisy_spectra(tab, X, 1, 0, 5)
    rad = torch.from_numpy(lobs).to(dev)
    z0 = net.infer(rad)
    plain, ev_plain = _run(scene, rad, prior, None, dev)
    warm, ev_warm = _run(scene, rad, prior, z0, dev)
    cp = (plain["status"] & CONVERGED) != 0
    cw = (warm["status"] & CONVERGED) != 0
    fb = (warm["status"] & ff.ST_USED_FALLBACK) != 0
    print(f"\n  plain: conv {cp.mean():.4f} iters {plain['iters'].mean():.2f} evals {ev_plain}"
          f"\n  warm : conv {cw.mean():.4f} iters {warm['iters'].mean():.2f} evals {ev_warm} fallback {fb.mean():.4f}")
    assert np.all((warm["status"] & ff.ST_WARM_START) != 0)
    assert cw.mean() >= cp.mean() - 0.002
    assert warm["iters"].mean() < 0.6 * plain["iters"].mean()
    assert ev_warm < 0.6 * ev_plain
    assert fb.mean() < 0.02
    # accuracy: the warm-started fit reaches the oracle's (default-start) minimum
    ref = oracle.retrieve(tab, lobs, 1, prior.lo, prior.hi, prior.x0)
    assert_parity(warm, ref, tab=tab, lobs=lobs, min_same=0.98, label="warm start")


def test_warm_start_wall_time(world, dev, trained):
    """Network inference plus warm-started LM (fallback on) takes less wall
    time than the plain LM on a batch of the headline scene's size, where
    each lane of the persistent grid drains about twenty pixels."""
    tab, scene, prior = world
    net, _ = trained
    X = scenegen.config0_states(4096, scene=5)
    rad = torch.from_numpy(noisy_spectra(tab, X, 1, 0, 5)).to(dev)
    big = rad.repeat(640, 1).contiguous()                    # 2,621,440 pixels
    t = {}
    for name in ("plain", "warm", "plain", "warm"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        zz = net.infer(big) if name == "warm" else None
        ff.retrieve(scene, big, prior, z0=zz)
        torch.cuda.synchronize()
        t[name] = time.perf_counter() - t0
    print(f"\n  2,621,440 px: plain {t['plain'] * 1e3:.1f} ms, warm (network + LM) {t['warm'] * 1e3:.1f} ms")
    assert t["warm"] < 0.8 * t["plain"]


def test_warm_start_on_clustered_fire_scene(dev):
    """A scene that is 97 % background (f = 0 truth), with the warm start
    routed by the front end as the benchmark runs it: the network gives
    starts to the fire candidates only (HFDI >= -0.1, Sec. 2.1) and every
    other pixel starts from the default x0.  Convergence stays at least as
    high as with the default start everywhere, fire pixels need far fewer
    iterations, and the whole scene costs fewer evaluations."""
    atm = scenegen.make_atmosphere(1, 0)
    tab = oracle.band_tables(atm)
    scene = ff.Scene(atm)
    lo, hi, x0 = scenegen.default_prior(1)
    prior = ff.Prior(1, lo, hi, x0)
    states, fire = scenegen.config1_states()
    idx = scenegen.subsample(1, 0, len(states), 20000)
    lobs = noisy_spectra(tab, states[idx], 1, 1, 7)
    isf = fire[idx]
    net = ff.WarmStart(seed=1)
    net.fit_normalization(ff.generate(scene, prior, 999, 0, 16384, bg_fraction=0.3)[0])
    net.train(scene, prior, steps=1500, batch=2048, seed=2, bg_fraction=0.3, lr=1e-3, lr_final=1e-5)
    rad = torch.from_numpy(lobs).to(dev)
    z0, n_cand = net.infer_routed(scene, rad)
    torch.cuda.synchronize()
    routed = ~np.isnan(z0[:, 0].cpu().numpy())
    assert routed.sum() == n_cand and routed[isf].mean() > 0.5 and routed[~isf].mean() < 0.05
    plain, ev_plain = _run(scene, rad, prior, None, dev)
    warm, ev_warm = _run(scene, rad, prior, z0, dev)
    cp = (plain["status"] & CONVERGED) != 0
    cw = (warm["status"] & CONVERGED) != 0
    # pixels without a start are solved exactly as the plain retrieval solves them
    for k in ("state", "rrr", "iters", "status"):
        np.testing.assert_array_equal(warm[k][~routed], plain[k][~routed])
    assert np.all((warm["status"][routed] & ff.ST_WARM_START) != 0)
    print(f"\n  {n_cand} candidates ({routed[isf].sum()} of {isf.sum()} fire pixels)"
          f"\n  plain: conv {cp.mean():.4f} (fire {cp[isf].mean():.4f}) iters bg {plain['iters'][~isf].mean():.2f} "
          f"fire {plain['iters'][isf].mean():.2f} evals/px {ev_plain / len(idx):.2f}"
          f"\n  warm : conv {cw.mean():.4f} (fire {cw[isf].mean():.4f}) iters bg {warm['iters'][~isf].mean():.2f} "
          f"fire {warm['iters'][isf].mean():.2f} evals/px {ev_warm / len(idx):.2f} "
          f"fallback {((warm['status'] & ff.ST_USED_FALLBACK) != 0).mean():.4f}")
    assert cw.mean() >= cp.mean()
    assert cw[isf].mean() >= cp[isf].mean() - 0.01
    assert warm["iters"][routed & isf].mean() < 0.6 * plain["iters"][routed & isf].mean()
    assert ev_warm < ev_plain
    # accuracy on the fire pixels against the oracle from the default start
    sel = np.flatnonzero(isf)[:1500]
    ref = oracle.retrieve(tab, lobs[sel], 1, lo, hi, x0)
    sub = {k: v[sel] for k, v in warm.items() if v is not None}
    assert_parity(sub, ref, tab=tab, lobs=lobs[sel], min_same=0.97, label="warm start, clustered-fire scene")


def test_checkpoint_resume_is_bitwise(world, dev, tmp_path):
    """Training is deterministic, and a run saved halfway (weights,
    normalisation, Adam moments and step counts: ff_warmstart_save),
    reloaded (ff_warmstart_load) and continued with the second span of the
    same schedule ends bitwise equal to the uninterrupted run."""
    tab, scene, prior = world
    total, half, batch = 240, 110, 512

    def fresh():
        n = ff.WarmStart(seed=3)
        n.fit_normalization(ff.generate(scene, prior, 77, 0, 4096, bg_fraction=0.3)[0])
        return n

    a = fresh()
    a.train(scene, prior, steps=total, batch=batch, seed=5, bg_fraction=0.3)
    torch.cuda.synchronize()
    b = fresh()
    b.train(scene, prior, steps=total, batch=batch, seed=5, bg_fraction=0.3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.get_params(), b.get_params())
    c = fresh()
    c.train(scene, prior, steps=total, batch=batch, seed=5, bg_fraction=0.3, n_steps=half)
    torch.cuda.synchronize()
    assert c.steps_done == half
    path = str(tmp_path / "half.ffws")
    c.save(path)
    c.close()
    d = ff.WarmStart.load(path)
    assert d.sizes == a.sizes and d.steps_done == half
    d.train(scene, prior, steps=total, batch=batch, seed=5, bg_fraction=0.3, first_step=d.steps_done)
    torch.cuda.synchronize()
    assert d.steps_done == total
    np.testing.assert_array_equal(d.get_params(), a.get_params())
    for x, y in zip(d.get_normalization(), a.get_normalization()):
        np.testing.assert_array_equal(x, y)
    # and the resumed network infers the same starts
    X = scenegen.config0_states(256, scene=9)
    rad = torch.from_numpy(noisy_spectra(tab, X, 1, 0, 9)).to(dev)
    np.testing.assert_array_equal(d.infer(rad).cpu().numpy(), a.infer(rad).cpu().numpy())
