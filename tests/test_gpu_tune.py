"""Launch-shape autotuner (ff_tune): the choice is valid, stored in and read
back from its JSON table, and the tuned launch still matches the oracle."""
import json

import numpy as np
import pytest

import oracle
import scenegen
from _helpers import assert_parity, noisy_spectra

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402


def test_tune_choice_cache_and_parity(tmp_path):
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    atm = scenegen.make_atmosphere(0, 0)
    tab = oracle.band_tables(atm)
    scene = ff.Scene(atm)
    lo, hi, x0 = scenegen.default_prior(1)
    prior = ff.Prior(1, lo, hi, x0)
    X = scenegen.config0_states(4096)[:1500]
    lobs = noisy_spectra(tab, X, 1, 0, 0)
    rad = torch.from_numpy(lobs).to(dev)
    path = str(tmp_path / "tuning.json")
    opts, ms = ff.tune([scene], [rad], prior, cache_path=path)
    print(f"\n  chosen: lanes/pixel {opts.lanes_per_pixel} block {opts.block_size} "
          f"blocks/CU {opts.blocks_per_cu} schedule {opts.schedule}: {ms:.3f} ms")
    assert opts.lanes_per_pixel in (1, 2, 4, 8, 16, 32, 64)
    assert opts.block_size in (64, 128, 256) and opts.blocks_per_cu in (0, 1)
    assert opts.n_quad == 32 and ms > 0
    table = json.load(open(path))
    assert len(table) == 1
    (key, entry), = table.items()
    assert "/B284/model1/" in key and key.endswith("/plain/P2^10")
    assert entry["lanes_per_pixel"] == opts.lanes_per_pixel and entry["ms"] == pytest.approx(ms, rel=1e-5)
    # a second call is a table hit: same choice, same recorded time
    opts2, ms2 = ff.tune([scene], [rad], prior, cache_path=path)
    assert (opts2.lanes_per_pixel, opts2.block_size, opts2.blocks_per_cu, opts2.schedule) == \
        (opts.lanes_per_pixel, opts.block_size, opts.blocks_per_cu, opts.schedule)
    assert ms2 == pytest.approx(ms, rel=1e-5)
    # a warm-start batch is a different entry
    z0 = torch.tensor(np.clip(oracle.x_to_z(X, lo, hi), -1, 1), dtype=torch.float32, device=dev)
    ff.tune([scene], [rad], prior, z0s=[z0], cache_path=path)
    assert len(json.load(open(path))) == 2
    # the tuned launch still reaches the oracle's fits
    ref = oracle.retrieve(tab, lobs, 1, lo, hi, x0)
    out = ff.retrieve(scene, rad, prior, options=opts)
    torch.cuda.synchronize()
    assert_parity(out.numpy(), ref, min_t=500, label="tuned")
