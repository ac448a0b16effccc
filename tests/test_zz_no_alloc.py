"""ff_retrieve_batch_noalloc (queue counters and launch descriptors in the
library's fixed device array) gives bitwise the outputs of
ff_retrieve_batch, on two calls in a row, the second with a smaller input
(the array keeps the first call's contents, so the counters must be cleared
by the call itself)."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import noisy_spectra

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402

KEYS = ("state", "cov", "moments", "rrr", "iters", "status")


def _batch(dev, sizes, cfg=6):
    scenes, rads = [], []
    for s, P in enumerate(sizes):
        atm = scenegen.make_atmosphere(cfg, s % 3)
        tab = oracle.band_tables(atm)
        X = scenegen.config0_states(max(P, 1), scene=40 + s)[:P]
        scenes.append(ff.Scene(atm))
        rads.append(torch.from_numpy(noisy_spectra(tab, X, 1, cfg, s)).to(dev).reshape(P, tab.B))
    return scenes, rads


def _outputs(rads, model, dev, fill):
    outs = [ff.allocate_outputs(r.shape[0], model, dev) for r in rads]
    for o in outs:
        for t in (o.state, o.cov, o.moments, o.rrr):
            t.fill_(fill)
        o.iters.fill_(-5)
        o.status.fill_(-5)
    return outs


def _compare(a, b):
    for x, y in zip(a, b):
        x, y = x.numpy(), y.numpy()
        for k in KEYS:
            np.testing.assert_array_equal(x[k], y[k], err_msg=k)


def _pair(scenes, rads, prior, opts, z0s, dev, stream):
    ref = _outputs(rads, prior.model, dev, -7.0)
    got = _outputs(rads, prior.model, dev, 3.0)
    ev_ref = torch.zeros(1, dtype=torch.int64, device=dev)
    ev_got = torch.zeros(1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    ff.retrieve_batch(scenes, rads, prior, z0s=z0s, options=opts, outputs=ref, evals=ev_ref, stream=stream)
    ff.retrieve_batch_noalloc(scenes, rads, got, prior, z0s=z0s, options=opts, evals=ev_got, stream=stream)
    torch.cuda.synchronize()
    _compare(got, ref)
    assert ev_got.item() == ev_ref.item() > 0
    return got


@pytest.mark.parametrize("lanes", [1, 4])
def test_noalloc_matches_retrieve_batch_on_two_calls(lanes):
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    print(f"noalloc: lanes {lanes}", flush=True)
    prior = ff.default_prior(1)
    opts = ff.default_options(lanes_per_pixel=lanes, block_size=64)
    stream = torch.cuda.Stream(device=dev)
    # first call: 20 scenes (two launches of <= 16), an empty and a one-pixel scene
    sizes = [300, 0, 1, 77, 128] + [20 + 9 * k for k in range(15)]
    scenes, rads = _batch(dev, sizes)
    out1 = _pair(scenes, rads, prior, opts, None, dev, stream)
    assert sum(int(((o.numpy()["status"] & ff.ST_CONVERGED) != 0).sum()) for o in out1) > 0.8 * sum(sizes)
    # second call, smaller: 3 scenes, fewer pixels, per-pixel starts (with fallback)
    scenes2, rads2 = scenes[3:6], [r[: max(1, r.shape[0] // 3)] for r in rads[3:6]]
    g = torch.Generator(device="cpu").manual_seed(11)
    z0s = [(torch.rand((r.shape[0], 5), generator=g) * 2 - 1).to(dev) for r in rads2]
    _pair(scenes2, rads2, prior, opts, z0s, dev, stream)
    # and once more on the default stream
    _pair(scenes2[:1], rads2[:1], prior, opts, None, dev, None)


def test_noalloc_fp64_two_component():
    dev = torch.device("cuda:0")
    print("noalloc: fp64, two components", flush=True)
    prior = ff.default_prior(2)
    atm = scenegen.make_atmosphere(6, 0)
    tab = oracle.band_tables(atm)
    X = scenegen.config2_states(96, scene=3)
    X[:, 0] = np.maximum(X[:, 0], 1e-3)
    rad = torch.from_numpy(noisy_spectra(tab, X, 2, 6, 0)).to(dev)
    sc = ff.Scene(atm)
    opts = ff.default_options(precision=ff.PRECISION_FP64, lanes_per_pixel=2)
    _pair([sc, sc], [rad, rad[:40]], prior, opts, None, dev, None)
    _pair([sc], [rad[:17]], prior, opts, None, dev, None)
