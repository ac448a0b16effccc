"""Graph-captured pipeline (ff_pipeline_*): every replay equals the eager
launch sequence bitwise, also after the radiance buffers are rewritten in
place, with eager library work and synchronisations between replays."""
import numpy as np
import pytest

import oracle
import scenegen
from _helpers import noisy_spectra

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402

KEYS = ("state", "cov", "moments", "rrr", "iters", "status")


def _batch(dev, sizes=(70, 1, 333)):
    scenes, rads = [], []
    for s, P in enumerate(sizes):
        atm = scenegen.make_atmosphere(4, s)
        tab = oracle.band_tables(atm)
        X = scenegen.config0_states(P, scene=10 + s)
        scenes.append(ff.Scene(atm))
        rads.append(torch.from_numpy(noisy_spectra(tab, X, 1, 4, s)).to(dev))
    return scenes, rads


def _same(outs, ref):
    for o, r in zip(outs, ref):
        o, r = o.numpy(), r.numpy()
        for k in KEYS:
            np.testing.assert_array_equal(o[k], r[k], err_msg=k)


@pytest.mark.parametrize("warm", [False, True, "mixed"])
def test_pipeline_replays_match_eager(warm):
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    scenes, rads = _batch(dev)
    prior = ff.default_prior(1)
    opts = ff.default_options(lanes_per_pixel=4)
    net = None
    if warm:
        net = ff.WarmStart(seed=1)
        net.fit_normalization(ff.generate(scenes[0], prior, 9, 0, 4096)[0])
        net.train(scenes[0], prior, steps=200, batch=1024, seed=2)
        torch.cuda.synchronize()          # training runs on the default stream
    stream = torch.cuda.Stream(device=dev)
    evals = torch.zeros(1, dtype=torch.int64, device=dev)
    # one network per scene; "mixed": the middle scene starts from x0
    nets = None if not warm else [net, None if warm == "mixed" else net, net]

    def eager():
        with torch.cuda.stream(stream):
            z0s = None if nets is None else [None if n is None else n.infer(r, stream=stream)
                                             for n, r in zip(nets, rads)]
            outs = ff.retrieve_batch(scenes, rads, prior, z0s=z0s, options=opts, stream=stream)
        torch.cuda.synchronize()
        return outs

    pipe = ff.Pipeline(scenes, rads, prior, net=nets, options=opts, evals=evals, stream=stream)
    torch.cuda.synchronize()
    ref = eager()
    _same(pipe.outputs, ref)                      # the eager pass inside create
    n0 = evals.item()
    assert n0 > 0
    for rep in range(3):
        for o in pipe.outputs:                    # clear the outputs with a fill kernel
            for t in (o.state, o.cov, o.moments, o.rrr):
                t.fill_(-7.0)
        torch.cuda.synchronize()
        pipe.launch()
        torch.cuda.synchronize()
        _same(pipe.outputs, ref)
        eager()                                   # eager library work between replays
    assert evals.item() == 4 * n0                 # create + three replays
    # serving pattern: new spectra written into the bound buffers
    with torch.no_grad():
        rads[0].mul_(1.01)
        rads[2].copy_(torch.flip(rads[2], dims=[0]))
    torch.cuda.synchronize()
    ref2 = eager()
    pipe.launch()
    torch.cuda.synchronize()
    _same(pipe.outputs, ref2)
    assert not np.array_equal(ref2[0].numpy()["state"], ref[0].numpy()["state"])
    pipe.close()


def test_routed_pipeline_matches_eager_routing():
    """The routed pipeline (front end + network on the candidates, inside the
    graph, the candidate count never read back) equals the eager routed
    sequence -- ff_hfdi_candidates, the network on the listed rows, the
    retrieval with NaN rows for every other pixel -- bitwise in every output
    (the status bits included, so the same rows start from the network), on
    every replay; a scene that is mostly background keeps most of its rows
    without a start."""
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    scenes, rads = _batch(dev)
    atm = scenegen.make_atmosphere(1, 0)
    tab = oracle.band_tables(atm)
    states, fire = scenegen.config1_states(64, 1234, scene=0)
    idx = scenegen.subsample(1, 3, len(states), 3000)
    scenes.append(ff.Scene(atm))
    rads.append(torch.from_numpy(noisy_spectra(tab, states[idx], 1, 1, 3)).to(dev))
    prior = ff.default_prior(1)
    opts = ff.default_options(lanes_per_pixel=4)
    net = ff.WarmStart(seed=1)
    net.fit_normalization(ff.generate(scenes[0], prior, 9, 0, 4096)[0])
    net.train(scenes[0], prior, steps=200, batch=1024, seed=2)
    torch.cuda.synchronize()
    nets = [net, None, net, net]
    stream = torch.cuda.Stream(device=dev)
    evals = torch.zeros(1, dtype=torch.int64, device=dev)

    def eager():
        z0s = []
        for n, sc, r in zip(nets, scenes, rads):
            z0s.append(None if n is None else n.infer_routed(sc, r, -0.1, stream=stream)[0])
        with torch.cuda.stream(stream):
            outs = ff.retrieve_batch(scenes, rads, prior, z0s=z0s, options=opts, stream=stream)
        torch.cuda.synchronize()
        return outs, z0s

    pipe = ff.Pipeline(scenes, rads, prior, net=nets, options=opts, evals=evals, stream=stream, route=-0.1)
    torch.cuda.synchronize()
    ref, z0s = eager()
    _same(pipe.outputs, ref)
    n0 = evals.item()
    routed = ~np.isnan(z0s[3][:, 0].cpu().numpy())
    assert 0 < routed.sum() < 0.5 * len(routed)      # mostly background
    st = pipe.outputs[3].numpy()["status"].astype(np.int64)
    assert np.array_equal((st & ff.ST_WARM_START) != 0, routed)
    for rep in range(3):
        for o in pipe.outputs:
            for t in (o.state, o.cov, o.moments, o.rrr):
                t.fill_(-7.0)
        torch.cuda.synchronize()
        pipe.launch()
        torch.cuda.synchronize()
        _same(pipe.outputs, ref)
        eager()
    assert evals.item() == 4 * n0
    pipe.close()


def test_pipeline_argument_checks():
    dev = torch.device("cuda:0")
    scenes, rads = _batch(dev, sizes=(8,))
    net = ff.WarmStart(n_in=100, seed=1)                    # inputs != 284 bands
    with pytest.raises(ff.FirefitError):
        ff.Pipeline(scenes, rads, ff.default_prior(1), net=net)
    with pytest.raises(ff.FirefitError):                    # routed with a NaN threshold
        ff.Pipeline(scenes, rads, ff.default_prior(1), net=ff.WarmStart(seed=1), route=float("nan"))
    # routed without any network: nothing to route, the plain pipeline's outputs
    plain = ff.Pipeline(scenes, rads, ff.default_prior(1))
    routed = ff.Pipeline(scenes, rads, ff.default_prior(1), route=ff.HFDI_THRESHOLD)
    torch.cuda.synchronize()
    for k in KEYS:
        np.testing.assert_array_equal(routed.outputs[0].numpy()[k], plain.outputs[0].numpy()[k])
    plain.close()
    routed.close()
    # the default (null) stream is fine for create and launch
    pipe = ff.Pipeline(scenes, rads, ff.default_prior(1), stream=torch.cuda.default_stream(dev))
    ref = pipe.outputs[0].numpy()
    pipe.launch()
    torch.cuda.synchronize()
    for k in KEYS:
        np.testing.assert_array_equal(pipe.outputs[0].numpy()[k], ref[k])
    pipe.close()


def test_release_scratch_then_retrieve_again():
    """ff_release_scratch frees the per-stream buffers; the next call on the
    same stream allocates afresh and gives the same result."""
    dev = torch.device("cuda:0")
    scenes, rads = _batch(dev, sizes=(40,))
    stream = torch.cuda.Stream(device=dev)
    a = ff.retrieve(scenes[0], rads[0], ff.default_prior(1), stream=stream)
    torch.cuda.synchronize()
    assert ff.lib().ff_release_scratch() == ff.FF_OK
    b = ff.retrieve(scenes[0], rads[0], ff.default_prior(1), stream=stream)
    torch.cuda.synchronize()
    for k in KEYS:
        np.testing.assert_array_equal(a.numpy()[k], b.numpy()[k])


def test_release_scratch_keeps_a_live_pipelines_buffer():
    """ff_release_scratch frees the per-stream buffers but not the one a live
    pipeline's graph binds: replays after the release still match the eager
    result bitwise."""
    dev = torch.device("cuda:0")
    scenes, rads = _batch(dev, sizes=(50, 7))
    prior = ff.default_prior(1)
    stream = torch.cuda.Stream(device=dev)
    pipe = ff.Pipeline(scenes, rads, prior, options=ff.default_options(lanes_per_pixel=2), stream=stream)
    torch.cuda.synchronize()
    ref = [o.numpy() for o in pipe.outputs]
    assert ff.lib().ff_release_scratch() == ff.FF_OK
    for o in pipe.outputs:
        o.state.fill_(-3.0)
    torch.cuda.synchronize()
    pipe.launch(stream)
    torch.cuda.synchronize()
    for o, r in zip(pipe.outputs, ref):
        o = o.numpy()
        for k in KEYS:
            np.testing.assert_array_equal(o[k], r[k], err_msg=k)
    pipe.close()
