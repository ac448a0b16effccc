"""Shared test helpers: seeded oracle-made spectra and parity comparisons.

Every pixel that both runs (the GPU and the FP64 oracle, on the same float32
radiance) converge on is checked, in one of these ways:

  * Loss, where the fit is determined (the oracle's posterior s.d. of every
    state variable below a quarter of its box).  The oracle evaluates its
    loss (Sec. 2.5 eq. loss, FP64, the same masked bands) at the GPU's
    state, and the GPU must end at a fit at least as good as the oracle's
    own up to the resolution of the cost: F(x_gpu) <= F(x_oracle) + 3e-3 s^2
    (s^2 = F / (N_valid - n), one chi^2 unit).  The GPU forms the thermal
    term in FP32, whose ~1e-7 relative rounding per band (~3e-5 s per
    residual where the fire dominates the radiance) moves F by ~1e-3 chi^2
    units, a few 1e-6 of F.
  * Loss, in distribution, where some variable is not determined (an
    undetected fire's temperature, f < 1e-4; the components of a mixture
    that the data cannot separate): the loss is flat along that direction
    and the stop rule ends at a point set by the solve's trajectory (the
    oracle's own end point moves by up to ~10 chi^2 units under 1e-7
    relative perturbations of its input).  At 1e-3, 0.1 and 1 chi^2 units
    the GPU may end worse than the oracle no more often than it ends
    better (x1.5, +5).
  * Same minimum.  A pixel is at the oracle's minimum when the relative
    radiance residuals agree to 1e-5 and every variable the data determine
    lies within 3 posterior s.d. of the oracle's value.  There:
      - E[T] within 0.5 K wherever it is identified: both fits have
        f >= 1e-4, neither has an unidentified (zero-Jacobian-column)
        variable, and the oracle's posterior s.d. of E[T] is <= 100 K;
      - f within 1e-4 wherever the oracle's posterior s.d. of f is <= 1e-3
        at a full-rank solution (at f = 0 the temperature columns vanish and
        a large f at the lower temperature bound can fit equally: the
        area-temperature degeneracy, Sec. 4);
      - the relative radiance residual within 1e-5 (by definition);
      - the Gauss-Newton posterior where E[T] is compared, every variable is
        determined and the two states agree to 0.05 posterior s.d. (the
        covariance is a function of the state): the s.d. within 5 % and the
        correlations among them within 0.05 (J^T J is accumulated in FP32
        and its inverse amplifies that rounding by the condition number,
        up to ~1e4 for the five-endmember surface).
    Where E[T] or f differ by more than their tolerance at the same
    minimum, the GPU's end point must fit strictly better than the oracle's
    (by more than the loss resolution): a solve from another start can stop
    further along a flat direction than the default-start oracle did.
  * Pixels at another minimum are covered by the loss checks (a different
    start, or an FP32 trajectory, may end in another basin of nearly equal
    cost).
"""
import numpy as np

import oracle
import scenegen

CONVERGED = oracle.ST_CONVERGED
SD_T_MAX = 100.0
SD_F_MAX = 1e-3
T_TOL = 0.5          # K
F_TOL = 1e-4
RRR_TOL = 1e-5
LOSS_TOL_CHI2 = 3e-3  # loss resolution of an FP32 thermal term, chi^2 units
F_DETECT = 1e-4      # fire fractions below this are not detections (the f tolerance)
COV_SD_TOL = 0.05
COV_STATE_SD = 0.05
COV_CORR_TOL = 0.05
BASIN_SD = 3.0


def noisy_spectra(tab, states, model, cfg, scene, snr=300.0):
    """Oracle forward model + SNR noise (sigma = L / snr), float32."""
    L = oracle.forward(tab, states, model)
    if snr is None:
        return L.astype(np.float32)
    noise = scenegen.noise_normals(cfg, scene, len(states), tab.B)
    return (L * (1.0 + noise / snr)).astype(np.float32)


def loss_at(tab, lobs, state, model, q=32):
    """The oracle's loss (eq. loss) at physical states [P, n] on radiance
    lobs [P, B] (float32, widened): sum over the unsaturated bands of
    (L_obs - L(x))^2, and the number of those bands."""
    lobs = np.ascontiguousarray(lobs, np.float32)
    L = oracle.forward(tab, np.asarray(state, np.float64), model, q=q)
    r = lobs.astype(np.float64) - L
    used = np.ones(lobs.shape, bool) if tab.lsat is None else lobs < tab.lsat[None, :]
    r = np.where(used, r, 0.0)
    return (r * r).sum(axis=1), used.sum(axis=1)


def posterior_sd(ref, model):
    """Oracle posterior s.d. of (E[T], f) by the delta method on its covariance."""
    n = oracle.n_state(model)
    C = oracle.unpack_cov(ref.cov, n)
    sd_f = np.sqrt(np.abs(C[:, 0, 0]))
    if model in (1, 4):                  # one lognormal component: E[T] = m
        sd_t = np.sqrt(np.abs(C[:, 1, 1]))
    else:
        x = ref.state
        g = np.zeros_like(x)
        g[:, 1] = x[:, 4] - x[:, 2]      # dE/deta = m_h - m_s
        g[:, 2] = 1.0 - x[:, 1]          # dE/dm_s
        g[:, 4] = x[:, 1]                # dE/dm_h
        sd_t = np.sqrt(np.abs(np.einsum("pi,pij,pj->p", g, C, g)))
    return np.nan_to_num(sd_t, nan=np.inf), np.nan_to_num(sd_f, nan=np.inf)


def _both(gpu, ref):
    gst = gpu["status"].astype(np.int64)
    return ((gst & CONVERGED) != 0) & ref.converged


def identifiable(gpu, ref, model=1, f_min=F_DETECT):
    """(both converged, E[T] comparable) masks -- see the module docstring."""
    gst = gpu["status"].astype(np.int64)
    both = _both(gpu, ref)
    sd_t, _ = posterior_sd(ref, model)
    ok = both & (gpu["state"][:, 0] >= f_min) & (ref.state[:, 0] >= f_min)
    ok &= (gst & oracle.ST_COVSING) == 0
    ok &= (ref.status.astype(np.int64) & oracle.ST_COVSING) == 0
    ok &= sd_t <= SD_T_MAX
    return both, ok


def f_comparable(gpu, ref, model=1):
    both = _both(gpu, ref)
    _, sd_f = posterior_sd(ref, model)
    full_rank = (ref.status.astype(np.int64) & oracle.ST_COVSING) == 0
    return both & (sd_f <= SD_F_MAX) & full_rank


def same_minimum(gpu, ref, tol=RRR_TOL, model=1):
    both = _both(gpu, ref)
    n = oracle.n_state(model)
    sd = np.sqrt(np.abs(np.diagonal(oracle.unpack_cov(ref.cov, n), axis1=1, axis2=2)))
    near = np.abs(gpu["state"][:, :n] - ref.state) <= BASIN_SD * sd
    near |= ~np.isfinite(sd)                 # unidentified variables are not compared
    return both & (np.abs(gpu["rrr"] - ref.rrr) <= tol) & near.all(axis=1)


def _box(model):
    lo, hi, _ = scenegen.default_prior(model)
    return hi - lo


def determined(ref, model=1):
    """[P, n] mask of the variables the data determine: the oracle's
    posterior s.d. is finite and below a quarter of the variable's box."""
    n = oracle.n_state(model)
    sd = np.sqrt(np.abs(np.diagonal(oracle.unpack_cov(ref.cov, n), axis1=1, axis2=2)))
    return np.isfinite(sd) & (sd < 0.25 * _box(model)[None, :]), sd


def covariance_report(gpu, ref, mask, model=1):
    """Largest relative difference of the posterior s.d. and largest
    correlation difference over the variables the data determine (oracle
    s.d. < a quarter of the variable's box) on the masked pixels whose two
    states agree to COV_STATE_SD posterior s.d."""
    n = oracle.n_state(model)
    det, sd = determined(ref, model)
    close = np.all(np.abs(gpu["state"][:, :n] - ref.state) <= COV_STATE_SD * sd, axis=1)
    mask = mask & close & det.all(axis=1)
    if not mask.any():
        return 0.0, 0.0, 0
    Cg = oracle.unpack_cov(np.asarray(gpu["cov"], np.float64), n)[mask]
    Co = oracle.unpack_cov(ref.cov, n)[mask]
    dg = np.sqrt(np.abs(np.diagonal(Cg, axis1=1, axis2=2)))
    do = np.sqrt(np.abs(np.diagonal(Co, axis1=1, axis2=2)))
    det = np.isfinite(do) & (do < 0.25 * _box(model)[None, :]) & (do > 0)
    rel = np.where(det, np.abs(dg / np.where(det, do, 1.0) - 1.0), 0.0)
    rg = Cg / (dg[:, :, None] * dg[:, None, :])
    ro = Co / (do[:, :, None] * do[:, None, :])
    pair = det[:, :, None] & det[:, None, :]
    dr = np.where(pair, np.abs(rg - ro), 0.0)
    return float(np.nan_to_num(rel, nan=np.inf).max()), float(np.nan_to_num(dr, nan=np.inf).max()), int(det.sum())


def parity_report(gpu, ref, model=1, tab=None, lobs=None, q=32):
    """Dict of the parity statistics used by the tests (loss statistics when
    the oracle's tables and the radiance are given)."""
    both, ok = identifiable(gpu, ref, model)
    same = same_minimum(gpu, ref, model=model)
    t_ok = ok & same
    f_ok = f_comparable(gpu, ref, model) & same
    dT = np.abs(gpu["moments"][:, 0] - ref.moments[:, 0])
    df = np.abs(gpu["state"][:, 0] - ref.state[:, 0])
    drrr = np.abs(gpu["rrr"] - ref.rrr)
    rep = {
        "both": int(both.sum()), "same_min": int(same.sum()),
        "same_frac": float(same.sum() / max(both.sum(), 1)),
        "t_n": int(t_ok.sum()), "dT_max": float(dT[t_ok].max()) if t_ok.any() else 0.0,
        "dT_p99": float(np.percentile(dT[t_ok], 99)) if t_ok.any() else 0.0,
        "f_n": int(f_ok.sum()), "df_max": float(df[f_ok].max()) if f_ok.any() else 0.0,
        "drrr_max_same": float(drrr[same].max()) if same.any() else 0.0,
        "dT_over_tol": int((dT > T_TOL)[t_ok].sum()), "df_over_tol": int((df > F_TOL)[f_ok].sum()),
        "t_mask": t_ok, "f_mask": f_ok, "both_mask": both, "same_mask": same,
    }
    if "cov" in gpu and gpu["cov"] is not None:
        rep["cov_sd_rel_max"], rep["cov_corr_max"], rep["cov_n"] = covariance_report(gpu, ref, t_ok, model)
    if tab is not None and lobs is not None:
        idx = np.where(both)[0]
        Fg = np.full(len(both), np.nan)
        Fo = np.full(len(both), np.nan)
        nv = np.zeros(len(both), np.int64)
        if len(idx):
            Fg[idx], nv[idx] = loss_at(tab, lobs[idx], gpu["state"][idx], model, q)
            Fo[idx], _ = loss_at(tab, lobs[idx], ref.state[idx], model, q)
        n = oracle.n_state(model)
        s2 = Fo / np.maximum(nv - n, 1)
        dchi = (Fg - Fo) / s2
        worse = both & (dchi > LOSS_TOL_CHI2)
        det, _ = determined(ref, model)
        flat = both & ~det.all(axis=1)
        rep["loss_worse"] = int(worse.sum())
        rep["determined"] = int((both & ~flat).sum())
        rep["loss_worse_determined"] = int((worse & ~flat).sum())
        rep["flat"] = int(flat.sum())
        for thr in (1e-3, 0.1, 1.0):
            rep[f"flat_worse_{thr:g}"] = int((flat & (dchi > thr)).sum())
            rep[f"flat_better_{thr:g}"] = int((flat & (dchi < -thr)).sum())
        rep["dchi2_max"] = float(np.nanmax(dchi[both])) if both.any() else 0.0
        rep["dchi2_min"] = float(np.nanmin(dchi[both])) if both.any() else 0.0
        rep["dchi2_max_determined"] = float(np.nanmax(dchi[both & ~flat])) if (both & ~flat).any() else 0.0
        rep["worse_mask"] = worse & ~flat
        rep["dchi2"] = dchi
    return rep


def assert_parity(gpu, ref, model=1, tab=None, lobs=None, min_same=0.99, min_t=1, label="", q=32,
                  cov=True, flat_worse_frac=None):
    """The parity gate of the module docstring; tab and lobs (the oracle's
    tables and the float32 radiance both runs retrieved) are required.
    flat_worse_frac: instead of the symmetric test on fits with a flat
    direction, a bound on the share of pixels whose GPU fit ends more than
    one chi^2 unit worse than the oracle's (a known shortfall, stated by the
    caller)."""
    assert tab is not None and lobs is not None, "the loss check needs the tables and the radiance"
    rep = parity_report(gpu, ref, model, tab, lobs, q)
    print(label, {k: v for k, v in rep.items() if not k.endswith("_mask") and k != "dchi2"})
    assert rep["same_frac"] >= min_same, rep["same_frac"]
    assert rep["t_n"] >= min_t and rep["f_n"] >= min_t
    # values at the same minimum; a difference beyond the tolerance is
    # allowed only where the GPU's end point fits strictly better
    better = rep["dchi2"] < -LOSS_TOL_CHI2
    dT = np.abs(gpu["moments"][:, 0] - ref.moments[:, 0])
    df = np.abs(gpu["state"][:, 0] - ref.state[:, 0])
    off_t = rep["t_mask"] & (dT > T_TOL)
    off_f = rep["f_mask"] & (df > F_TOL)
    off = (off_t | off_f) & ~better
    if flat_worse_frac is not None:
        # a known flat-direction shortfall: such pixels count against its bound
        flat = rep["both_mask"] & ~determined(ref, model)[0].all(axis=1)
        assert (off & flat).sum() + rep["flat_worse_1"] <= flat_worse_frac * rep["both"] + 1
        off &= ~flat
    assert not off.any(), (dT[off], df[off], rep["dchi2"][off])
    rep["value_excused_better"] = int(((off_t | off_f) & better).sum())
    assert rep["drrr_max_same"] <= RRR_TOL
    # every determined fit ends as good as the oracle's
    assert rep["loss_worse_determined"] == 0, (rep["loss_worse_determined"], rep["dchi2_max_determined"])
    # fits with a flat direction: no worse than the oracle in distribution
    if flat_worse_frac is None:
        for thr in (1e-3, 0.1, 1.0):
            w, b = rep[f"flat_worse_{thr:g}"], rep[f"flat_better_{thr:g}"]
            assert w <= 1.5 * b + 5, (thr, w, b)
    else:
        assert rep["flat_worse_1"] <= flat_worse_frac * rep["both"], (rep["flat_worse_1"], rep["both"])
    if cov and "cov_sd_rel_max" in rep:
        assert rep["cov_sd_rel_max"] <= COV_SD_TOL, rep["cov_sd_rel_max"]
        assert rep["cov_corr_max"] <= COV_CORR_TOL, rep["cov_corr_max"]
    return rep
