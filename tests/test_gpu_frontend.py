"""GPU tests of the fire-candidate front end (Sec. 2.1) through the C ABI:
the HFDI values and the candidate list against the oracle (bit-exact: both
sides evaluate the index in IEEE float32 and compare the threshold in
double), and the listed retrieval against the full retrieval and the
oracle."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import assert_parity, noisy_spectra

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def clustered(dev):
    """A 160 x 203 clustered-fire scene (3 % fire in blobs, the rest f = 0),
    oracle-made spectra with SNR-300 noise; P = 32,480 is not a multiple of
    the 4,096-pixel tile."""
    atm = scenegen.make_atmosphere(1, 0)
    tab = oracle.band_tables(atm)
    states, fire = scenegen.config1_states(160, 203, scene=3)
    lobs = noisy_spectra(tab, states, 1, 1, 3)
    return atm, tab, states, fire, lobs


def _cands(scene, lobs, dev, threshold=-0.1):
    rad = torch.from_numpy(np.ascontiguousarray(lobs)).to(dev)
    idx, cnt, h = ff.hfdi_candidates(scene, rad, threshold)
    torch.cuda.synchronize()
    n = int(cnt.item())
    return rad, idx, cnt, idx[:n].cpu().numpy(), h.cpu().numpy()


def test_hfdi_and_candidates_match_the_oracle_exactly(clustered, dev):
    atm, tab, states, fire, lobs = clustered
    lobs = lobs.copy()
    ia, ib = oracle.nearest_band(tab.lam, 2430.0), oracle.nearest_band(tab.lam, 2061.0)
    lobs[5] = 0.0                    # 0/0
    lobs[6, ia] = np.nan             # non-finite
    lobs[7, ib] = -lobs[7, ia]       # zero sum, nonzero difference
    scene = ff.Scene(atm)
    for thr in (-0.1, -0.3, 0.0):
        _, _, _, got, h = _cands(scene, lobs, dev, thr)
        want, hw = oracle.hfdi_candidates(tab, lobs, thr)
        np.testing.assert_array_equal(h, hw)          # NaNs compare equal here
        np.testing.assert_array_equal(got, want)
        print(f"threshold {thr}: {len(want)} candidates of {len(lobs)}")
    # with saturation levels on the index bands
    lsat = np.full(tab.B, np.inf, np.float32)
    lsat[ia] = np.float32(np.percentile(lobs[:, ia][np.isfinite(lobs[:, ia])], 90))
    lsat[ib] = np.float32(np.percentile(lobs[:, ib], 95))
    atm_s = scenegen.make_atmosphere(1, 0, sat_level=lsat)
    tab_s = oracle.band_tables(atm_s)
    _, _, _, got, h = _cands(ff.Scene(atm_s), lobs, dev)
    want, _ = oracle.hfdi_candidates(tab_s, lobs)
    np.testing.assert_array_equal(got, want)
    assert len(want) > len(oracle.hfdi_candidates(tab, lobs)[0])


@pytest.mark.parametrize("P", [0, 1, 4095, 4096, 4097, 70000])
def test_candidate_list_sizes(dev, P):
    atm = scenegen.make_atmosphere(0, 0)
    tab = oracle.band_tables(atm)
    rng = np.random.default_rng(P)
    lobs = rng.uniform(0.0, 1.0, (P, tab.B)).astype(np.float32)
    _, idx, cnt, got, h = _cands(ff.Scene(atm), lobs, dev)
    want, hw = oracle.hfdi_candidates(tab, lobs)
    assert int(cnt.item()) == len(want)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(h, hw)


def test_candidates_without_index_values_and_scratch_reuse(dev):
    """The writing pass takes the candidate decisions the counting pass kept
    in the stream's scratch, so the list must not depend on whether the
    index values are written, nor on what an earlier call of another size
    left in that scratch: calls of 70,000, 1,000 and 70,000 pixels in a row on
    one stream, with and without index values, each equal to the oracle."""
    atm = scenegen.make_atmosphere(0, 0)
    tab = oracle.band_tables(atm)
    scene = ff.Scene(atm)
    rng = np.random.default_rng(11)
    lobs = rng.uniform(0.0, 1.0, (70000, tab.B)).astype(np.float32)
    stream = torch.cuda.Stream(device=dev)
    for P, thr, values in ((70000, -0.1, False), (1000, 0.2, True), (70000, 0.05, False), (70000, -0.1, True)):
        rad = torch.from_numpy(np.ascontiguousarray(lobs[:P])).to(dev)
        with torch.cuda.stream(stream):
            idx, cnt, h = ff.hfdi_candidates(scene, rad, thr, with_index_values=values, stream=stream)
        torch.cuda.synchronize()
        want, hw = oracle.hfdi_candidates(tab, lobs[:P], thr)
        n = int(cnt.item())
        print(f"  P={P} threshold {thr} values {values}: {n} candidates")
        assert n == len(want)
        np.testing.assert_array_equal(idx[:n].cpu().numpy(), want)
        if values:
            np.testing.assert_array_equal(h.cpu().numpy(), hw)
        else:
            assert h is None


def test_listed_retrieval_equals_the_full_retrieval(clustered, dev):
    """Listed rows get exactly the full retrieval's outputs (same kernel,
    same launch shape); rows not listed are left untouched; list entries
    outside [0, P) are skipped."""
    atm, tab, states, fire, lobs = clustered
    scene = ff.Scene(atm)
    prior = ff.default_prior(1)
    rad, idx, cnt, cands, _ = _cands(scene, lobs, dev)
    for lpp in (1, 4):
        opts = ff.default_options(lanes_per_pixel=lpp)
        full = ff.retrieve(scene, rad, prior, options=opts).numpy()
        out = ff.allocate_outputs(len(lobs), 1, dev)
        for t in (out.state, out.cov, out.moments, out.rrr):
            t.fill_(-7.0)
        out.iters.fill_(-7)
        out.status.fill_(-7)
        evals = torch.zeros(1, dtype=torch.int64, device=dev)
        ff.retrieve_listed(scene, rad, idx, cnt, prior, options=opts, outputs=out, evals=evals)
        torch.cuda.synchronize()
        r = out.numpy()
        for k in ("state", "cov", "moments", "rrr", "iters", "status"):
            np.testing.assert_array_equal(r[k][cands], full[k][cands])
        rest = np.setdiff1d(np.arange(len(lobs)), cands)
        assert np.all(r["state"][rest] == -7.0) and np.all(r["status"][rest] == -7)
        assert int(evals.item()) == int((full["iters"][cands] + 1).sum())
    # entries outside [0, P) are skipped, a count above P is clamped to P
    bad = torch.tensor([-1, len(lobs) + 5, int(cands[0])], dtype=torch.int64, device=dev)
    big = torch.tensor([3], dtype=torch.int64, device=dev)
    out = ff.allocate_outputs(len(lobs), 1, dev)
    out.status.fill_(-7)
    ff.retrieve_listed(scene, rad, bad, big, prior, outputs=out)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert st[cands[0]] == full["status"][cands[0]]
    assert np.sum(st != -7) == 1


def test_listed_retrieval_matches_the_oracle(clustered, dev):
    """The candidates' retrievals against the FP64 oracle on the same rows."""
    atm, tab, states, fire, lobs = clustered
    scene = ff.Scene(atm)
    prior = ff.default_prior(1)
    rad, idx, cnt, cands, _ = _cands(scene, lobs, dev)
    out = ff.retrieve_listed(scene, rad, idx, cnt, prior)
    torch.cuda.synchronize()
    r = {k: v[cands] for k, v in out.numpy().items() if v is not None}
    ref = oracle.retrieve(tab, lobs[cands], 1, prior.lo, prior.hi, prior.x0)
    rec = np.isin(np.nonzero(fire)[0], cands).mean()
    print(f"{len(cands)} candidates, fire recall {rec:.3f}, background candidates {(~fire[cands]).sum()}")
    assert_parity(r, ref, tab=tab, lobs=lobs[cands], min_same=0.97, label="listed")


@pytest.fixture(scope="module")
def frontend_net(clustered, dev):
    """A network trained on the scene's own generated spectra, with a share
    of background samples (as for the clustered-fire benchmark)."""
    atm = clustered[0]
    scene = ff.Scene(atm)
    prior = ff.default_prior(1)
    net = ff.WarmStart(seed=1)
    net.fit_normalization(ff.generate(scene, prior, 999, 0, 16384, bg_fraction=0.3)[0])
    net.train(scene, prior, steps=1500, batch=2048, seed=2, bg_fraction=0.3, lr=1e-3, lr_final=1e-5)
    torch.cuda.synchronize()
    return net


def test_listed_inference_equals_the_full_inference(clustered, dev, frontend_net):
    """ff_mlp_infer_listed writes exactly the full inference's rows at the
    listed pixels, leaves the other rows untouched and skips entries outside
    [0, P)."""
    atm, tab, states, fire, lobs = clustered
    scene = ff.Scene(atm)
    net = frontend_net
    rad, idx, cnt, cands, _ = _cands(scene, lobs, dev)
    n = len(cands)
    full = net.infer(rad).cpu().numpy()
    z0 = torch.full((len(lobs), 5), -7.0, dtype=torch.float32, device=dev)
    net.infer_listed(rad, idx, n, z0=z0)
    torch.cuda.synchronize()
    got = z0.cpu().numpy()
    np.testing.assert_array_equal(got[cands], full[cands])
    rest = np.setdiff1d(np.arange(len(lobs)), cands)
    assert np.all(got[rest] == -7.0)
    # nothing listed: nothing written; entries outside [0, P) skipped
    z1 = torch.full((len(lobs), 5), -7.0, dtype=torch.float32, device=dev)
    net.infer_listed(rad, idx, 0, z0=z1)
    bad = torch.tensor([-1, len(lobs), len(lobs) + 5, int(cands[0])], dtype=torch.int64, device=dev)
    net.infer_listed(rad, bad, 4, z0=z1)
    torch.cuda.synchronize()
    g1 = z1.cpu().numpy()
    np.testing.assert_array_equal(g1[cands[0]], full[cands[0]])
    assert np.sum(np.any(g1 != -7.0, axis=1)) == 1


def test_warm_started_candidates(clustered, dev, frontend_net):
    """The paper's pipeline with the learned start: HFDI candidates, the
    network on the listed rows only, LM on the listed rows from those starts
    (fallback on).  The listed warm retrieval equals the full warm retrieval
    on the listed rows; against the plain listed retrieval it takes fewer
    iterations and converges as often; its fits reach the FP64 oracle's
    (default-start) minimum."""
    atm, tab, states, fire, lobs = clustered
    scene = ff.Scene(atm)
    prior = ff.default_prior(1)
    net = frontend_net
    rad, idx, cnt, cands, _ = _cands(scene, lobs, dev)
    z0 = net.infer(rad)
    net.infer_listed(rad, idx, len(cands), z0=z0)
    full = ff.retrieve(scene, rad, prior, z0=z0).numpy()
    warm = ff.retrieve_listed(scene, rad, idx, cnt, prior, z0=z0)
    plain = ff.retrieve_listed(scene, rad, idx, cnt, prior)
    torch.cuda.synchronize()
    w = {k: v[cands] for k, v in warm.numpy().items() if v is not None}
    p = {k: v[cands] for k, v in plain.numpy().items() if v is not None}
    for k in ("state", "cov", "moments", "rrr", "iters", "status"):
        np.testing.assert_array_equal(w[k], full[k][cands])
    assert np.all((w["status"] & ff.ST_WARM_START) != 0)
    cw = (w["status"] & ff.ST_CONVERGED) != 0
    cp = (p["status"] & ff.ST_CONVERGED) != 0
    fb = (w["status"] & ff.ST_USED_FALLBACK) != 0
    isf = fire[cands]
    print(f"\n  {len(cands)} candidates ({isf.sum()} fire): plain conv {cp.mean():.4f} iters {p['iters'].mean():.2f} "
          f"(fire {p['iters'][isf].mean():.2f}); warm conv {cw.mean():.4f} iters {w['iters'].mean():.2f} "
          f"(fire {w['iters'][isf].mean():.2f}) fallback {fb.mean():.4f}")
    assert cw.mean() >= cp.mean() - 0.002
    assert w["iters"].mean() < 0.7 * p["iters"].mean()
    assert w["iters"][isf].mean() < 0.6 * p["iters"][isf].mean()
    ref = oracle.retrieve(tab, lobs[cands], 1, prior.lo, prior.hi, prior.x0)
    assert_parity(w, ref, tab=tab, lobs=lobs[cands], min_same=0.95, label="warm-started candidates")
