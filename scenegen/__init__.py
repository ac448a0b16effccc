"""Seeded synthetic inputs for the fire-temperature retrieval.

This module only *draws* inputs: instrument band grids, the high-resolution
solar irradiance and transmittance that stand in for a per-scene 6S look-up
table (paper Sec. 2.2, eq. (solar)), true per-pixel states, fire masks and
the standard-normal noise draws.  It holds none of the retrieval's own
arithmetic (no forward model, no quadrature, no band resampling, no solver):
radiance is made from the drawn states by whichever forward model the caller
owns.  Both the FP64 oracle and the GPU library consume what this module
returns, and neither is imported here.

Seeds: ``numpy.random.Generator(PCG64(SeedSequence([cfg, scene, stream])))``
with stream ids ``STREAM_*`` below, so any array can be regenerated alone.

The paper's AVIRIS-3 scenes, endmember library and 6S tables are not
available; the shapes and value distributions below follow the workload
definitions of the benchmark configurations (284 bands over 380-2500 nm,
Gaussian SRF of 8.5 nm FWHM, lognormal sub-pixel temperatures, linear
reflectance, a 5778 K blackbody sun scaled to 1361 W m^-2, a 0.9
transmittance with Gaussian absorption dips, SNR-300 noise).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

STREAM_PARAMS = 0
STREAM_NOISE = 1
STREAM_MASK = 2
STREAM_DIPS = 3
STREAM_SUBSAMPLE = 4

MODEL_LOGNORMAL_1 = 1  # state (f, m, s, rho0, rho1)
MODEL_LOGNORMAL_2 = 2  # state (f, eta, m_s, s_s, m_h, s_h, rho0, rho1)
MODEL_GAUSS_GRID_2 = 3  # state (f, eta, mu_s, sig_s, mu_h, sig_h, rho0, rho1)
MODEL_ENDMEMBER_1 = 4  # state (f, m, s, x_gv, x_npv, x_soil1, x_soil2, x_char)
MODEL_FULL = 5  # state (f, eta, mu_s, sig_s, mu_h, sig_h, x_gv, x_npv, x_soil1, x_soil2, x_char)

N_STATE = {MODEL_LOGNORMAL_1: 5, MODEL_LOGNORMAL_2: 8, MODEL_GAUSS_GRID_2: 8, MODEL_ENDMEMBER_1: 8,
           MODEL_FULL: 11}

STATE_NAMES = {
    MODEL_LOGNORMAL_1: ("f", "m", "s", "rho0", "rho1"),
    MODEL_LOGNORMAL_2: ("f", "eta", "m_s", "s_s", "m_h", "s_h", "rho0", "rho1"),
    MODEL_GAUSS_GRID_2: ("f", "eta", "mu_s", "sig_s", "mu_h", "sig_h", "rho0", "rho1"),
    MODEL_ENDMEMBER_1: ("f", "m", "s", "x_gv", "x_npv", "x_soil1", "x_soil2", "x_char"),
    MODEL_FULL: ("f", "eta", "mu_s", "sig_s", "mu_h", "sig_h", "x_gv", "x_npv", "x_soil1", "x_soil2", "x_char"),
}

# Exact SI constants (2019 redefinition) used to define the synthetic sun.
_H = 6.62607015e-34
_C = 299792458.0
_KB = 1.380649e-23
_SIGMA_SB = 2.0 * math.pi**5 * _KB**4 / (15.0 * _H**3 * _C**2)

T_SUN = 5778.0
SOLAR_CONSTANT = 1361.0

# Absorption dips of the synthetic transmittance: centre and Gaussian width (nm).
DIP_CENTRES_NM = (940.0, 1140.0, 1380.0, 1880.0)
DIP_WIDTHS_NM = (15.0, 20.0, 40.0, 50.0)
DIP_DEPTH_RANGE = (0.3, 0.95)
T_CONTINUUM = 0.9


def rng_for(cfg: int, scene: int, stream: int) -> np.random.Generator:
    """Independent PCG64 stream for (configuration, scene, stream id)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, scene, stream])))


# --------------------------------------------------------------------------
# Instrument
# --------------------------------------------------------------------------
def band_grid(n_bands: int = 284, lo_nm: float = 380.0, hi_nm: float = 2500.0,
              fwhm_nm: float = 8.5):
    """Band centres uniformly spaced over [lo, hi] and a constant FWHM."""
    lam = np.linspace(lo_nm, hi_nm, n_bands, dtype=np.float64)
    fwhm = np.full(n_bands, fwhm_nm, dtype=np.float64)
    return lam, fwhm


def hires_grid(lo_nm: float = 350.0, hi_nm: float = 2550.0, step_nm: float = 0.5):
    n = int(round((hi_nm - lo_nm) / step_nm)) + 1
    return lo_nm + step_nm * np.arange(n, dtype=np.float64)


# --------------------------------------------------------------------------
# Atmosphere stand-in (replaces the per-scene 6S table of paper Sec. 2.2)
# --------------------------------------------------------------------------
def solar_irradiance(lam_nm: np.ndarray) -> np.ndarray:
    """Top-of-atmosphere irradiance, W m^-2 nm^-1: a 5778 K blackbody whose
    integral over all wavelengths is 1361 W m^-2 (pi * B integrates to
    sigma T^4, so the scale is 1361 / (sigma T^4))."""
    lam = lam_nm * 1e-9
    x = _H * _C / (lam * _KB * T_SUN)
    b = 2.0 * _H * _C**2 / lam**5 / np.expm1(x) * 1e-9
    return SOLAR_CONSTANT / (_SIGMA_SB * T_SUN**4) * math.pi * b


def draw_dip_depths(cfg: int, scene: int) -> np.ndarray:
    rng = rng_for(cfg, scene, STREAM_DIPS)
    return rng.uniform(DIP_DEPTH_RANGE[0], DIP_DEPTH_RANGE[1], size=len(DIP_CENTRES_NM))


def transmittance(lam_nm: np.ndarray, depths: np.ndarray) -> np.ndarray:
    """0.9 times a product of (1 - d_i * Gaussian dip): never negative."""
    t = np.full_like(lam_nm, T_CONTINUUM)
    for c, w, d in zip(DIP_CENTRES_NM, DIP_WIDTHS_NM, depths):
        t *= 1.0 - d * np.exp(-0.5 * ((lam_nm - c) / w) ** 2)
    return t


@dataclass
class Atmosphere:
    """High-resolution atmosphere + instrument description of one scene."""
    wavelength_nm: np.ndarray      # band centres [B]
    fwhm_nm: np.ndarray            # band FWHM [B]
    hr_lambda_nm: np.ndarray       # high-resolution grid [H]
    e_solar: np.ndarray            # [H] W m^-2 nm^-1
    tau_down: np.ndarray           # [H]
    tau_up: np.ndarray             # [H]
    rho_atm: np.ndarray            # [H]
    s_sph: np.ndarray              # [H]
    cos_sza: float = 1.0
    sat_level: np.ndarray | None = None   # [B] float32 or None (no saturation)
    dip_depths: np.ndarray = field(default_factory=lambda: np.zeros(4))

    @property
    def n_bands(self) -> int:
        return int(self.wavelength_nm.shape[0])


def make_atmosphere(cfg: int, scene: int = 0, n_bands: int = 284,
                    rho_atm: float = 0.0, s_sph: float = 0.0, cos_sza: float = 1.0,
                    sat_level=None) -> Atmosphere:
    """Synthetic scene atmosphere: blackbody sun, one transmittance used for
    both paths, no path reflectance and no spherical albedo by default."""
    lam, fwhm = band_grid(n_bands)
    hr = hires_grid()
    depths = draw_dip_depths(cfg, scene)
    t = transmittance(hr, depths)
    return Atmosphere(
        wavelength_nm=lam, fwhm_nm=fwhm, hr_lambda_nm=hr,
        e_solar=solar_irradiance(hr), tau_down=t.copy(), tau_up=t.copy(),
        rho_atm=np.full_like(hr, rho_atm), s_sph=np.full_like(hr, s_sph),
        cos_sza=float(cos_sza),
        sat_level=None if sat_level is None else np.asarray(sat_level, np.float32),
        dip_depths=depths)


# --------------------------------------------------------------------------
# Prior box and default start (the affine map of paper eq. (affine) needs
# finite bounds for every state variable)
# --------------------------------------------------------------------------
def default_prior(model: int):
    """(lo, hi, x0) in physical units for the given model."""
    if model == MODEL_LOGNORMAL_1:
        lo = np.array([0.0, 350.0, 1.0, -0.2, -5e-4])
        hi = np.array([0.5, 2200.0, 500.0, 1.0, 5e-4])
        x0 = np.array([0.01, 1000.0, 150.0, 0.2, 0.0])
    elif model == MODEL_LOGNORMAL_2:
        lo = np.array([0.0, 0.0, 350.0, 1.0, 900.0, 1.0, -0.2, -5e-4])
        hi = np.array([0.5, 1.0, 900.0, 500.0, 2200.0, 500.0, 1.0, 5e-4])
        x0 = np.array([0.01, 0.5, 650.0, 150.0, 1200.0, 150.0, 0.2, 0.0])
    elif model == MODEL_GAUSS_GRID_2:
        lo = np.array([0.0, 0.0, 350.0, 10.0, 900.0, 10.0, -0.2, -5e-4])
        hi = np.array([0.5, 1.0, 900.0, 500.0, 2200.0, 500.0, 1.0, 5e-4])
        x0 = np.array([0.01, 0.5, 650.0, 150.0, 1200.0, 150.0, 0.2, 0.0])
    elif model == MODEL_ENDMEMBER_1:
        # the surface fractions live on [0, 1] and start at the simplex centre
        lo = np.array([0.0, 350.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0])
        hi = np.array([0.5, 2200.0, 500.0, 1.0, 1.0, 1.0, 1.0, 1.0])
        x0 = np.array([0.01, 1000.0, 150.0, 0.2, 0.2, 0.2, 0.2, 0.2])
    elif model == MODEL_FULL:
        # the Gaussian-mixture box and start, fractions as for model 4
        lo = np.array([0.0, 0.0, 350.0, 10.0, 900.0, 10.0] + [0.0] * 5)
        hi = np.array([0.5, 1.0, 900.0, 500.0, 2200.0, 500.0] + [1.0] * 5)
        x0 = np.array([0.01, 0.5, 650.0, 150.0, 1200.0, 150.0] + [0.2] * 5)
    else:
        raise ValueError(f"unknown model {model}")
    return lo, hi, x0


# --------------------------------------------------------------------------
# True states
# --------------------------------------------------------------------------
def draw_states_lognormal1(rng: np.random.Generator, n: int) -> np.ndarray:
    """f ~ logU[1e-4, 0.3], m ~ U[600, 1400] K, s ~ U[50, 300] K,
    rho0 ~ U[0.05, 0.4], rho1 ~ U[-1e-4, 1e-4] /nm.  Shape [n, 5]."""
    f = np.exp(rng.uniform(math.log(1e-4), math.log(0.3), n))
    m = rng.uniform(600.0, 1400.0, n)
    s = rng.uniform(50.0, 300.0, n)
    r0 = rng.uniform(0.05, 0.4, n)
    r1 = rng.uniform(-1e-4, 1e-4, n)
    return np.stack([f, m, s, r0, r1], axis=1)


def draw_states_lognormal2(rng: np.random.Generator, n: int) -> np.ndarray:
    """Two-component stress states: f ~ logU[1e-5, 1e-3], eta ~ U[0.05, 0.95],
    smouldering mean U[500, 800] K, flaming mean U[900, 1500] K, both spreads
    U[50, 300] K, reflectance as in the one-component draw.  Shape [n, 8]."""
    f = np.exp(rng.uniform(math.log(1e-5), math.log(1e-3), n))
    eta = rng.uniform(0.05, 0.95, n)
    ms = rng.uniform(500.0, 800.0, n)
    ss = rng.uniform(50.0, 300.0, n)
    mh = rng.uniform(900.0, 1500.0, n)
    sh = rng.uniform(50.0, 300.0, n)
    r0 = rng.uniform(0.05, 0.4, n)
    r1 = rng.uniform(-1e-4, 1e-4, n)
    return np.stack([f, eta, ms, ss, mh, sh, r0, r1], axis=1)


def draw_states_gauss_grid2(rng: np.random.Generator, n: int) -> np.ndarray:
    """States of the Gaussian-mixture model: f ~ logU[1e-4, 0.1], eta ~
    U[0.05, 0.95], smouldering mean U[450, 850] K, flaming mean U[950, 1700]
    K, spreads U[30, 250] K, reflectance as in the one-component draw.
    Shape [n, 8]."""
    f = np.exp(rng.uniform(math.log(1e-4), math.log(0.1), n))
    eta = rng.uniform(0.05, 0.95, n)
    ms = rng.uniform(450.0, 850.0, n)
    ss = rng.uniform(30.0, 250.0, n)
    mh = rng.uniform(950.0, 1700.0, n)
    sh = rng.uniform(30.0, 250.0, n)
    r0 = rng.uniform(0.05, 0.4, n)
    r1 = rng.uniform(-1e-4, 1e-4, n)
    return np.stack([f, eta, ms, ss, mh, sh, r0, r1], axis=1)


def draw_states_endmember1(rng: np.random.Generator, n: int) -> np.ndarray:
    """One lognormal fire component over the endmember surface: f, m, s as in
    the one-component draw, surface fractions ~ Dirichlet(0.7, ..., 0.7) (a
    sparse mix: many pixels have fractions near zero).  Shape [n, 8]."""
    f = np.exp(rng.uniform(math.log(1e-4), math.log(0.3), n))
    m = rng.uniform(600.0, 1400.0, n)
    s = rng.uniform(50.0, 300.0, n)
    x = rng.dirichlet(np.full(5, 0.7), n)
    return np.concatenate([np.stack([f, m, s], axis=1), x], axis=1)


def draw_states_full(rng: np.random.Generator, n: int) -> np.ndarray:
    """The paper's full state: the Gaussian-mixture draw for f, eta and the
    two components, surface fractions ~ Dirichlet(0.7, ..., 0.7).
    Shape [n, 11]."""
    th = draw_states_gauss_grid2(rng, n)[:, :6]
    x = rng.dirichlet(np.full(5, 0.7), n)
    return np.concatenate([th, x], axis=1)


def endmember_library(hr_lambda_nm: np.ndarray) -> np.ndarray:
    """Five synthetic surface reflectance spectra [5, H] on the
    high-resolution grid, standing in for the paper's fire-relevant library
    (Sec. 2.4: green vegetation, non-photosynthetic vegetation, two soils,
    char/ash), built from smooth logistic edges and Gaussian absorption
    features of the usual shapes:
      0 green vegetation: low visible with a green peak, red edge near 715
        nm to a 0.45 NIR plateau, liquid-water bands at 1450 and 1940 nm;
      1 non-photosynthetic vegetation: a rise from 0.10 to 0.40 with a
        cellulose-lignin feature at 2100 nm;
      2 bright soil: 0.15 rising to 0.45 with a clay feature at 2200 nm;
      3 dark iron-rich soil: 0.06 rising to 0.30 with a ferric feature at
        900 nm;
      4 char/ash: flat and dark, 0.04 rising to 0.08."""
    lam = np.asarray(hr_lambda_nm, np.float64)

    def edge(c, w):
        return 1.0 / (1.0 + np.exp(-(lam - c) / w))

    def dip(c, w, d):
        return 1.0 - d * np.exp(-0.5 * ((lam - c) / w) ** 2)

    gv = (0.04 + 0.05 * np.exp(-0.5 * ((lam - 550.0) / 30.0) ** 2) + 0.41 * edge(715.0, 12.0)
          - 0.20 * edge(1300.0, 60.0)) * dip(1450.0, 60.0, 0.5) * dip(1940.0, 70.0, 0.6)
    npv = (0.10 + 0.30 * edge(900.0, 250.0)) * dip(2100.0, 50.0, 0.25) * dip(1940.0, 60.0, 0.15)
    soil1 = (0.15 + 0.30 * edge(800.0, 300.0)) * dip(2200.0, 25.0, 0.15)
    soil2 = (0.06 + 0.24 * edge(1100.0, 350.0)) * dip(900.0, 80.0, 0.2)
    char = 0.04 + 0.04 * (lam - lam.min()) / (lam.max() - lam.min())
    return np.stack([gv, npv, soil1, soil2, char])


def config5_states(n_pixels: int = 262144, scene: int = 0) -> np.ndarray:
    """The paper's two-Gaussian mixture on the temperature grid."""
    return draw_states_gauss_grid2(rng_for(5, scene, STREAM_PARAMS), n_pixels)


def config0_states(n_pixels: int = 4096, scene: int = 0) -> np.ndarray:
    return draw_states_lognormal1(rng_for(0, scene, STREAM_PARAMS), n_pixels)


def config2_states(n_pixels: int = 262144, scene: int = 0) -> np.ndarray:
    return draw_states_lognormal2(rng_for(2, scene, STREAM_PARAMS), n_pixels)


def fire_mask_blobs(rng: np.random.Generator, rows: int, cols: int,
                    fire_fraction: float = 0.03, smooth_px: float = 6.0) -> np.ndarray:
    """Spatially clustered fire mask: white noise smoothed by a Gaussian of
    ``smooth_px`` pixels, thresholded so that exactly round(fraction * N)
    pixels are on.  Returns bool [rows, cols]."""
    from scipy.ndimage import gaussian_filter
    noise = rng.standard_normal((rows, cols)).astype(np.float32)
    sm = gaussian_filter(noise, smooth_px, mode="wrap")
    n_on = int(round(fire_fraction * rows * cols))
    flat = sm.ravel()
    idx = np.argpartition(-flat, n_on - 1)[:n_on]
    mask = np.zeros(rows * cols, dtype=bool)
    mask[idx] = True
    return mask.reshape(rows, cols)


def config1_states(rows: int = 2048, cols: int = 1234, scene: int = 0,
                   fire_fraction: float = 0.03) -> tuple[np.ndarray, np.ndarray]:
    """Clustered-fire scene: lines x cross-track pixels in row-major order.
    Fire pixels take one-component draws, background pixels f = 0 with the
    same reflectance draws (their m, s are irrelevant and set to the draws).
    Returns (states [P, 5], fire mask [P] bool)."""
    p = rows * cols
    states = draw_states_lognormal1(rng_for(1, scene, STREAM_PARAMS), p)
    mask = fire_mask_blobs(rng_for(1, scene, STREAM_MASK), rows, cols, fire_fraction).ravel()
    states[~mask, 0] = 0.0
    return states, mask


def noise_normals(cfg: int, scene: int, n_pixels: int, n_bands: int) -> np.ndarray:
    """Standard-normal draws [P, B] float32; radiance noise is sigma = L/SNR."""
    rng = rng_for(cfg, scene, STREAM_NOISE)
    return rng.standard_normal((n_pixels, n_bands), dtype=np.float32)


def subsample(cfg: int, scene: int, n_total: int, n_sample: int) -> np.ndarray:
    """Sorted seeded subset of pixel indices (without replacement)."""
    rng = rng_for(cfg, scene, STREAM_SUBSAMPLE)
    return np.sort(rng.choice(n_total, size=min(n_sample, n_total), replace=False))


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n)).astype(np.int64)


def ragged_scene_sizes(n_scenes: int = 16, lo: int = 10_000, hi: int = 2_500_000,
                       cfg: int = 4) -> np.ndarray:
    """Pixel counts of a ragged multi-scene batch, log-uniform in [lo, hi]."""
    return log_uniform_int(rng_for(cfg, 0, STREAM_PARAMS), lo, hi, n_scenes)


# ----------------------------------------------------------------------------
# Ragged multi-scene batch: 16 scenes, pixel counts log-uniform in
# [10k, 2.5M]; four atmospheres (one per flight line, scene s uses s % 4);
# the four smallest scenes are coarse-resolution versions of a 15x finer
# truth (each coarse pixel is the footprint of 15 x 15 fine pixels, so its
# temperature distribution is a sub-pixel mixture of the fine-scale draws).
# ----------------------------------------------------------------------------
RAGGED_BLOCK = 15
RAGGED_ATMOSPHERES = 4


def config4_layout(n_scenes: int = 16, n_block_averaged: int = 4) -> list[dict]:
    """Per-scene shape: rows x cols coarse pixels (near-square, rows*cols <=
    the drawn count), atmosphere id and block size (1 or RAGGED_BLOCK)."""
    sizes = ragged_scene_sizes(n_scenes)
    smallest = set(np.argsort(sizes, kind="stable")[:n_block_averaged].tolist())
    out = []
    for s, p in enumerate(sizes.tolist()):
        cols = max(1, int(math.isqrt(int(p))))
        rows = max(1, int(p) // cols)
        out.append({"scene": s, "rows": rows, "cols": cols, "pixels": rows * cols,
                    "atmosphere": s % RAGGED_ATMOSPHERES,
                    "block": RAGGED_BLOCK if s in smallest else 1})
    return out


def config4_states(spec: dict, fire_fraction: float = 0.03) -> tuple[np.ndarray, np.ndarray]:
    """Truth of one ragged-batch scene at its finest resolution: (states
    [rows*block * cols*block, 5], fire mask) in row-major order of the fine
    grid, clustered fire blobs as in the clustered-fire scene."""
    r, c = spec["rows"] * spec["block"], spec["cols"] * spec["block"]
    states = draw_states_lognormal1(rng_for(4, spec["scene"], STREAM_PARAMS), r * c)
    mask = fire_mask_blobs(rng_for(4, spec["scene"], STREAM_MASK), r, c, fire_fraction).ravel()
    states[~mask, 0] = 0.0
    return states, mask


def block_footprints(rows: int, cols: int, block: int) -> np.ndarray:
    """Index map [rows*cols, block*block]: the fine pixels (row-major on the
    fine grid of rows*block x cols*block) inside each coarse pixel."""
    fr = np.arange(rows)[:, None, None, None] * block + np.arange(block)[None, None, :, None]
    fc = np.arange(cols)[None, :, None, None] * block + np.arange(block)[None, None, None, :]
    return (fr * (cols * block) + fc).reshape(rows * cols, block * block)
