"""The FP32 LM kernel drops work a wave does not need: the saturation mask
when no pixel of the wave has a saturated band, and (one-component model)
the 1/(1 - S rho) factor when every pixel's table has S = 0.  Both shortcuts
must give the general path's sums bit for bit, whatever else shares the wave.

* S = 0: the same scene retrieved as a plain scene (shortcut taken) and
  through the per-pixel-atmosphere path with that scene as its only
  atmosphere (general path, the factor formed) -- bitwise equal outputs.
* mask: a scene with a finite saturation level and a few pixels lifted
  above it in one band; the waves holding them take the masked path, and
  every other pixel must equal its result from the same batch with those
  pixels left clean (every wave unmasked)."""
import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_07580_amd as ff  # noqa: E402

KEYS = ("state", "cov", "moments", "rrr", "iters", "status")


def _equal(a, b, rows=None):
    for k in KEYS:
        x, y = a[k], b[k]
        if rows is not None:
            x, y = x[rows], y[rows]
        np.testing.assert_array_equal(x, y, err_msg=k)      # NaN-aware


def _scene_radiance(P, seed, sat_level=None):
    atm = scenegen.make_atmosphere(1, seed, sat_level=sat_level)
    tab = oracle.band_tables(atm)
    states, _ = scenegen.config1_states(P // 64, 64, scene=seed, fire_fraction=0.1)
    L = oracle.forward(tab, states, 1)
    noise = scenegen.noise_normals(1, seed, len(states), tab.B)
    return atm, (L * (1.0 + noise / 300.0)).astype(np.float32)


@pytest.mark.parametrize("lanes", [1, 4])
def test_s_zero_shortcut_equals_general_path(lanes):
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    atm, lobs = _scene_radiance(4096, 31)
    assert not np.any(atm.s_sph)
    scene = ff.Scene(atm)
    rad = torch.from_numpy(lobs).to(dev)
    prior = ff.default_prior(1)
    opts = ff.default_options(lanes_per_pixel=lanes)
    fast = ff.retrieve(scene, rad, prior, options=opts).numpy()
    idx = torch.zeros(rad.shape[0], dtype=torch.int32, device=dev)
    general = ff.retrieve_atm_indexed([scene], idx, rad, prior, options=opts).numpy()
    torch.cuda.synchronize()
    conv = (fast["status"] & ff.ST_CONVERGED) != 0
    print(f"\n  L={lanes}: {conv.sum()} of {len(conv)} converged")
    assert conv.mean() > 0.9
    _equal(fast, general)


@pytest.mark.parametrize("lanes", [1, 4])
def test_unmasked_band_loop_equals_masked(lanes):
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    atm0, lobs = _scene_radiance(4096, 32)
    band = 150
    sat = np.full(lobs.shape[1], np.inf, np.float32)
    sat[band] = float(lobs[:, band].max()) * 1.5           # above every clean pixel
    atm = scenegen.make_atmosphere(1, 32, sat_level=sat)
    scene = ff.Scene(atm)
    lifted = np.arange(7, lobs.shape[0], 97)              # one pixel in ~97: many waves masked
    dirty = lobs.copy()
    dirty[lifted, band] = sat[band] * 2.0
    prior = ff.default_prior(1)
    opts = ff.default_options(lanes_per_pixel=lanes)
    clean_out = ff.retrieve(scene, torch.from_numpy(lobs).to(dev), prior, options=opts).numpy()
    dirty_out = ff.retrieve(scene, torch.from_numpy(dirty).to(dev), prior, options=opts).numpy()
    torch.cuda.synchronize()
    others = np.ones(lobs.shape[0], bool)
    others[lifted] = False
    print(f"\n  L={lanes}: {len(lifted)} pixels with a saturated band, {others.sum()} compared")
    _equal(clean_out, dirty_out, others)
    # the lifted pixels were solved on the remaining bands
    assert np.mean((dirty_out["status"][lifted] & ff.ST_CONVERGED) != 0) > 0.8
