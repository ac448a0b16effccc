"""FP64 CPU oracle for the fire-temperature inversion.

TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it; the product path never does.  It shares no code
with the GPU library (``paper_2608_07580_amd``) and does not import it.

Parts (Keely et al., real-time physics inversion of VSWIR fire spectra):
  * ``gauss_hermite``: physicists' Gauss-Hermite rule, nodes by the
    Golub-Welsch eigenvalue method (eigenvalues of the symmetric Jacobi matrix
    of the Hermite recurrence), weights by the Christoffel function.  Used to
    integrate the lognormal temperature pdf of the thermal term, Sec. 2.2
    eq. (thermal).
  * ``band_tables``: Gaussian spectral-response resampling of the
    high-resolution atmosphere onto the instrument bands (Sec. 2.4 resamples
    spectra onto the instrument grid with a Gaussian SRF) and the per-band
    factors of eq. (solar).
  * ``forward`` / ``retrieve``: the C oracle (``oracle.c``): forward model of
    eq. (fm)/(solar)/(thermal) with the analytic Jacobian, the masked loss of
    eq. (loss) minimised in the z coordinate of eq. (affine) by
    Levenberg-Marquardt, Gauss-Newton covariance and mixture moments.
  * ``adam_retrieve`` / ``paper_stages``: the paper's staged Adam (Sec. 2.5,
    eq. adam) in the C oracle.
  * ``hfdi`` / ``hfdi_candidates``: the fire-candidate index of Sec. 2.1.
  * ``coarsen``: block-mean aggregation and the Quantile Error Curve of the
    resolution-rescaling analysis.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# status bits of the retrieval (same meaning as the public status word)
ST_GTOL, ST_XTOL, ST_FTOL, ST_MAXITER = 1, 2, 4, 8
ST_NONFINITE, ST_DAMPING, ST_COVSING, ST_ATBOUND = 16, 32, 64, 128
ST_NODOF = 1024
ST_CONVERGED = ST_GTOL | ST_XTOL | ST_FTOL

LAMBDA_REF_NM = 1440.0


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2, IEEE)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        L.orc_planck.restype = C.c_double
        L.orc_planck.argtypes = [C.c_double, C.c_double, dp]
        L.orc_planck_many.restype = None
        L.orc_planck_many.argtypes = [C.c_long, dp, dp, dp, dp]
        L.orc_forward.restype = C.c_int
        L.orc_forward.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp, C.c_int, dp, dp,
                                  C.c_int, C.c_long, dp, dp, dp, C.c_int]
        L.orc_retrieve.restype = C.c_int
        L.orc_retrieve.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp, fp, C.c_int, dp, dp,
                                   C.c_int, dp, dp, dp, dp, C.c_long, fp,
                                   C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_int,
                                   dp, dp, dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_uint)]
        L.orc_adam_retrieve.restype = C.c_int
        L.orc_adam_retrieve.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp, fp, C.c_int, dp, dp,
                                        C.c_int, dp, dp, dp, dp, C.c_long, fp,
                                        C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_uint), dp, dp,
                                        dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                        dp, dp, dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_uint)]
        L.orc_max_threads.restype = C.c_int
        L.orc_project_simplex.restype = None
        L.orc_project_simplex.argtypes = [C.c_int, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


# ----------------------------------------------------------------------------
# Gauss-Hermite rule (Golub & Welsch 1969)
# ----------------------------------------------------------------------------
def _orthonormal_hermite(q: int, x):
    """p_0..p_q at x, orthonormal for the weight e^{-x^2}:
    p_0 = pi^-1/4, p_{j+1} = sqrt(2/(j+1)) x p_j - sqrt(j/(j+1)) p_{j-1}."""
    p = np.empty((q + 1,) + np.shape(x))
    p[0] = np.pi ** -0.25
    if q >= 1:
        p[1] = np.sqrt(2.0) * x * p[0]
    for j in range(1, q):
        p[j + 1] = np.sqrt(2.0 / (j + 1)) * x * p[j] - np.sqrt(j / (j + 1.0)) * p[j - 1]
    return p


def gauss_hermite(q: int = 32):
    """Nodes x_k and weights w_k with sum_k w_k f(x_k) ~ int e^{-x^2} f(x) dx.

    Golub-Welsch: the monic Hermite recurrence p_{k+1} = x p_k - (k/2) p_{k-1}
    gives a symmetric tridiagonal Jacobi matrix (zero diagonal, off-diagonal
    sqrt(k/2)) whose eigenvalues are the nodes.  The nodes get one Newton
    polish on the orthonormal p_q (p_q' = sqrt(2q) p_{q-1}), and the weights
    come from the Christoffel function w_k = 1 / sum_{j<q} p_j(x_k)^2, which
    keeps full relative accuracy for the ~1e-23 tail weights."""
    k = np.arange(1, q, dtype=np.float64)
    J = np.diag(np.sqrt(k / 2.0), 1) + np.diag(np.sqrt(k / 2.0), -1)
    x = np.linalg.eigvalsh(J)
    x = 0.5 * (x - x[::-1])                      # exact symmetry about 0
    p = _orthonormal_hermite(q, x)
    x = x - p[q] / (np.sqrt(2.0 * q) * p[q - 1])
    x = 0.5 * (x - x[::-1])
    p = _orthonormal_hermite(q, x)
    w = 1.0 / np.sum(p[:q] ** 2, axis=0)
    w = 0.5 * (w + w[::-1])
    return x, w


# ----------------------------------------------------------------------------
# Band tables: Gaussian SRF resampling of the high-resolution atmosphere
# ----------------------------------------------------------------------------
@dataclass
class Tables:
    lam: np.ndarray    # band centre [B] nm
    K: np.ndarray      # E cos(sza) / pi   [B]
    tau2: np.ndarray   # tau_down * tau_up [B]
    tup: np.ndarray    # tau_up [B]
    ratm: np.ndarray   # rho_atm [B]
    S: np.ndarray      # spherical albedo [B]
    lsat: np.ndarray | None  # [B] float32 saturation level, or None
    endm: np.ndarray | None = None  # [5, B] endmember reflectance (model 4), or None

    @property
    def B(self):
        return int(self.lam.shape[0])


def srf_matrix(lam_b, fwhm_b, hr_lam):
    """Row-normalised Gaussian response of each band on the high-resolution
    grid, truncated at +-4 sigma (sigma = FWHM / (2 sqrt(2 ln 2)))."""
    sig = np.asarray(fwhm_b, np.float64) / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    d = hr_lam[None, :] - np.asarray(lam_b, np.float64)[:, None]
    w = np.exp(-0.5 * (d / sig[:, None]) ** 2)
    w[np.abs(d) > 4.0 * sig[:, None]] = 0.0
    s = w.sum(axis=1)
    if np.any(s <= 0):
        raise ValueError("a band's response window holds no high-resolution sample")
    return w / s[:, None]


def band_tables(atm, endmembers=None) -> Tables:
    """Per-band factors of eq. (solar): each atmospheric quantity is resampled
    to band resolution separately; tau2 = resampled tau_down * resampled tau_up.
    ``endmembers`` [5, H] on the high-resolution grid are resampled with the
    same responses (Sec. 2.4)."""
    W = srf_matrix(atm.wavelength_nm, atm.fwhm_nm, atm.hr_lambda_nm)
    endm = None
    if endmembers is not None:
        e = np.asarray(endmembers, np.float64)
        assert e.shape == (N_ENDMEMBERS, W.shape[1])
        endm = np.ascontiguousarray(e @ W.T)
    E = W @ atm.e_solar
    tdn = W @ atm.tau_down
    tup = W @ atm.tau_up
    ratm = W @ atm.rho_atm
    S = W @ atm.s_sph
    return Tables(lam=np.ascontiguousarray(atm.wavelength_nm, np.float64),
                  K=E * atm.cos_sza / np.pi, tau2=tdn * tup, tup=tup, ratm=ratm, S=S,
                  lsat=None if atm.sat_level is None else np.asarray(atm.sat_level, np.float32),
                  endm=endm)


# ----------------------------------------------------------------------------
# Physics helpers
# ----------------------------------------------------------------------------
def planck(lam_nm, T, with_derivative: bool = False):
    """Planck radiance W m^-2 sr^-1 nm^-1 (and T dB/dT) from the C oracle."""
    lam_nm, T = np.broadcast_arrays(np.asarray(lam_nm, np.float64), np.asarray(T, np.float64))
    lam_c = np.ascontiguousarray(lam_nm.ravel())
    T_c = np.ascontiguousarray(T.ravel())
    out = np.empty_like(lam_c)
    der = np.empty_like(lam_c) if with_derivative else None
    lib().orc_planck_many(lam_c.size, _dp(lam_c), _dp(T_c), _dp(out), _dp(der))
    if with_derivative:
        return out.reshape(lam_nm.shape), der.reshape(lam_nm.shape)
    return out.reshape(lam_nm.shape)


N_ENDMEMBERS = 5          # Sec. 2.4: the library's five spectra
SIMPLEX_FIRST = 3         # model 4: state (f, m, s, x_surf,1 .. x_surf,5)


def simplex_first(model: int) -> int:
    """First surface fraction of the model's state (model 4: after f, m, s;
    model 5: after f, eta, mu_s, sig_s, mu_h, sig_h), or -1."""
    return {4: 3, 5: 6}.get(model, -1)


def n_state(model: int) -> int:
    return {1: 5, 2: 8, 3: 8, 4: 8, 5: 11}[model]


def project_simplex(v):
    """Euclidean projection of v onto the unit simplex {x >= 0, sum x = 1},
    the step applied to the surface fractions (Sec. 2.5)."""
    x = np.ascontiguousarray(v, np.float64).copy()
    lib().orc_project_simplex(x.size, _dp(x))
    return x


def _endm(tab: Tables, model: int):
    if simplex_first(model) < 0:
        return None
    if tab.endm is None:
        raise ValueError("the endmember models need the band tables' endmember spectra")
    return np.ascontiguousarray(tab.endm, np.float64)


def grid_nodes(G: int):
    """Temperature grid of the Gaussian-mixture model (model 3): G uniform
    nodes over [350, 2200] K (Sec. 2.2)."""
    return 350.0 + (2200.0 - 350.0) * np.arange(G) / (G - 1)


def x_to_z(x, lo, hi):
    """eq. (affine): z = 2 (x - lo) / (hi - lo) - 1."""
    return 2.0 * (np.asarray(x) - lo) / (hi - lo) - 1.0


def z_to_x(z, lo, hi):
    """eq. (affine) inverse: x = lo + (hi - lo)(z + 1) / 2."""
    return lo + 0.5 * (hi - lo) * (np.asarray(z) + 1.0)


def mixture_moments(eta, mu_hot, sd_hot, mu_smol, sd_smol):
    """Sec. 2.2 moment matching of the two-component mixture:
    E[T] = eta mu_hot + (1-eta) mu_smol,
    Var[T] = eta sd_hot^2 + (1-eta) sd_smol^2 + eta (1-eta)(mu_hot - mu_smol)^2."""
    et = eta * mu_hot + (1.0 - eta) * mu_smol
    var = eta * sd_hot**2 + (1.0 - eta) * sd_smol**2 + eta * (1.0 - eta) * (mu_hot - mu_smol) ** 2
    return et, np.sqrt(var)


def forward(tab: Tables, state, model: int, q: int = 32, jacobian: bool = False,
            nthreads: int = 0):
    """Model radiance [P, B] (and dL/dx [P, B, n]) for physical states [P, n]."""
    n = n_state(model)
    st = np.ascontiguousarray(np.atleast_2d(state), dtype=np.float64)
    assert st.shape[1] == n
    P = st.shape[0]
    gx, gw = gauss_hermite(q)
    L = np.empty((P, tab.B))
    J = np.empty((P, tab.B, n)) if jacobian else None
    endm = _endm(tab, model)
    rc = lib().orc_forward(tab.B, _dp(tab.lam), _dp(tab.K), _dp(tab.tau2), _dp(tab.tup),
                           _dp(tab.ratm), _dp(tab.S), _dp(endm), q, _dp(gx), _dp(gw), model, P,
                           _dp(st), _dp(L), _dp(J), nthreads)
    if rc != 0:
        raise ValueError("orc_forward: bad arguments")
    return (L, J) if jacobian else L


@dataclass
class LMOptions:
    max_iter: int = 50
    xtol: float = 1e-6
    ftol: float = 1e-8     # predicted relative decrease of an accepted step (~3e-6 chi^2 at SNR 300)
    # while the fire fraction is below f_detect (the fraction tolerance: no
    # detectable fire, the thermal variables unidentified) the decrease test
    # uses ftol_undetected, the resolution of an FP32 thermal term (1e-6 F)
    ftol_undetected: float = 1e-6
    f_detect: float = 1e-4
    gtol: float = 1e-10
    kappa: float = 1e-5
    tau: float = 1e-6      # initial damping mu_0 = tau * max diag(J^T J)


@dataclass
class Result:
    state: np.ndarray
    cov: np.ndarray
    moments: np.ndarray
    rrr: np.ndarray
    iters: np.ndarray
    status: np.ndarray

    @property
    def converged(self):
        return (self.status & ST_CONVERGED) != 0


def retrieve(tab: Tables, lobs, model: int, lo, hi, x0, z0=None, q: int = 32,
             opts: LMOptions | None = None, nthreads: int = 0) -> Result:
    """FP64 Levenberg-Marquardt retrieval of every pixel of lobs [P, B] (float32)."""
    opts = opts or LMOptions()
    n = n_state(model)
    lobs = np.ascontiguousarray(lobs, dtype=np.float32)
    P = lobs.shape[0]
    assert lobs.shape[1] == tab.B
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    x0 = np.ascontiguousarray(x0, np.float64)
    z0c = None if z0 is None else np.ascontiguousarray(z0, np.float64).reshape(P, n)
    gx, gw = gauss_hermite(q)
    out = Result(state=np.empty((P, n)), cov=np.empty((P, n * (n + 1) // 2)),
                 moments=np.empty((P, 2)), rrr=np.empty(P),
                 iters=np.empty(P, np.int32), status=np.empty(P, np.uint32))
    lsat = None if tab.lsat is None else np.ascontiguousarray(tab.lsat, np.float32)
    endm = _endm(tab, model)
    rc = lib().orc_retrieve(tab.B, _dp(tab.lam), _dp(tab.K), _dp(tab.tau2), _dp(tab.tup),
                            _dp(tab.ratm), _dp(tab.S), _dp(endm), _fp(lsat), q, _dp(gx), _dp(gw),
                            model, _dp(lo), _dp(hi), _dp(x0), _dp(z0c), P, _fp(lobs),
                            opts.max_iter, opts.xtol, opts.ftol, opts.gtol, opts.kappa,
                            opts.tau, opts.ftol_undetected, opts.f_detect, nthreads, _dp(out.state), _dp(out.cov), _dp(out.moments),
                            _dp(out.rrr), out.iters.ctypes.data_as(C.POINTER(C.c_int)),
                            out.status.ctypes.data_as(C.POINTER(C.c_uint)))
    if rc != 0:
        raise ValueError("orc_retrieve: bad arguments")
    return out


@dataclass
class AdamStage:
    """One stage of the paper's optimiser (Sec. 2.5): ``steps`` Adam updates of
    the variables in ``free`` (indices) at learning rate ``lr``; the gradient is
    scaled to at most ``clip`` in global norm (<= 0: no clip); variable j's loss
    runs over the used bands with window[j][0] <= lambda <= window[j][1] nm;
    ``zset`` maps a variable to the z it takes when the stage starts."""
    steps: int
    lr: float
    free: tuple
    window: dict            # j -> (lo_nm, hi_nm) for the free variables
    clip: float = 1.0
    zset: dict | None = None


ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8     # eq. (adam) defaults


# Sec. 2.5: band windows of the two stages (nm).  Stage 1 fits over the
# whole VSWIR range; in stage 2 the flaming component's variables see
# [900, 1800], the smouldering component's [1500, 2500], and the variables
# shared by both (f, eta) the union of the two.
OMEGA_1 = (350.0, 2500.0)
OMEGA_HOT = (900.0, 1800.0)
OMEGA_SMOL = (1500.0, 2500.0)
OMEGA_2 = (900.0, 2500.0)
ADAM_CLIP = 1.0     # maximum global gradient norm (the printed value is lost)


def paper_stages(model: int, lo, hi, x0, clip: float = ADAM_CLIP):
    """The two Adam stages of Sec. 2.5 on this model's state.

    Stage 1 (30 steps, lr 0.03, window OMEGA_1) fits the reflectance, the
    thermal fraction f and one temperature with the spread held at its lower
    bound (a near-delta distribution: the single temperature of stage 1);
    for the two-component model that temperature is the flaming mean with
    eta held at 1.  Stage 2 (100 steps, lr 0.015) holds the reflectance and
    fits f and the temperature distribution, whose spreads (and eta) restart
    from the prior start x0; the one-component model's f, m, s use OMEGA_2,
    the two-component model's flaming (m_h, s_h) and smouldering (m_s, s_s)
    variables their own windows.  With the endmember surface (models 4 and
    5) the surface fractions take the reflectance's place in stage 1, as the
    paper's stage-1 state {x_surf, alpha_1, T_1} has them; for model 5 (the
    paper's full forward model) the two stages free exactly the paper's
    state vectors x_1 and x_2."""
    z0 = x_to_z(np.asarray(x0, np.float64), np.asarray(lo, np.float64), np.asarray(hi, np.float64))
    if model == 1:
        s1 = AdamStage(30, 0.03, (0, 1, 3, 4), {j: OMEGA_1 for j in (0, 1, 3, 4)}, clip, {2: -1.0})
        s2 = AdamStage(100, 0.015, (0, 1, 2), {j: OMEGA_2 for j in (0, 1, 2)}, clip, {2: float(z0[2])})
    elif model == 4:
        surf = (0, 1, 3, 4, 5, 6, 7)
        s1 = AdamStage(30, 0.03, surf, {j: OMEGA_1 for j in surf}, clip, {2: -1.0})
        s2 = AdamStage(100, 0.015, (0, 1, 2), {j: OMEGA_2 for j in (0, 1, 2)}, clip, {2: float(z0[2])})
    elif model == 5:
        # the paper's own state vectors: x_1 = {x_surf, alpha_1, T_1} and
        # x_2 = {mu_hot, sig_hot, mu_smol, sig_smol, eta, alpha}
        surf = (0, 4, 6, 7, 8, 9, 10)
        s1 = AdamStage(30, 0.03, surf, {j: OMEGA_1 for j in surf}, clip, {1: 1.0, 5: -1.0})
        win = {0: OMEGA_2, 1: OMEGA_2, 2: OMEGA_SMOL, 3: OMEGA_SMOL, 4: OMEGA_HOT, 5: OMEGA_HOT}
        s2 = AdamStage(100, 0.015, (0, 1, 2, 3, 4, 5), win, clip,
                       {1: float(z0[1]), 3: float(z0[3]), 5: float(z0[5])})
    elif model in (2, 3):
        s1 = AdamStage(30, 0.03, (0, 4, 6, 7), {j: OMEGA_1 for j in (0, 4, 6, 7)}, clip,
                       {1: 1.0, 5: -1.0})
        win = {0: OMEGA_2, 1: OMEGA_2, 2: OMEGA_SMOL, 3: OMEGA_SMOL, 4: OMEGA_HOT, 5: OMEGA_HOT}
        s2 = AdamStage(100, 0.015, (0, 1, 2, 3, 4, 5), win, clip,
                       {1: float(z0[1]), 3: float(z0[3]), 5: float(z0[5])})
    else:
        raise ValueError(f"unknown model {model}")
    return [s1, s2]


def adam_retrieve(tab: Tables, lobs, model: int, lo, hi, x0, stages, z0=None, q: int = 32,
                  beta1: float = ADAM_BETA1, beta2: float = ADAM_BETA2, eps: float = ADAM_EPS,
                  nthreads: int = 0) -> Result:
    """FP64 staged-Adam retrieval (Sec. 2.5, eq. adam) of every pixel of lobs
    [P, B]; outputs as ``retrieve`` (iters = Adam steps taken)."""
    n = n_state(model)
    lobs = np.ascontiguousarray(lobs, dtype=np.float32)
    P = lobs.shape[0]
    assert lobs.shape[1] == tab.B
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    x0 = np.ascontiguousarray(x0, np.float64)
    z0c = None if z0 is None else np.ascontiguousarray(z0, np.float64).reshape(P, n)
    k = len(stages)
    steps = np.array([s.steps for s in stages], np.int32)
    free = np.array([sum(1 << j for j in s.free) for s in stages], np.uint32)
    lr = np.array([s.lr for s in stages], np.float64)
    clip = np.array([s.clip for s in stages], np.float64)
    wlo = np.zeros((max(k, 1), n))
    whi = np.zeros((max(k, 1), n))
    zset = np.full((max(k, 1), n), np.nan)
    for i, s in enumerate(stages):
        for j in s.free:
            wlo[i, j], whi[i, j] = s.window[j]
        for j, v in (s.zset or {}).items():
            zset[i, j] = v
    gx, gw = gauss_hermite(q)
    out = Result(state=np.empty((P, n)), cov=np.empty((P, n * (n + 1) // 2)),
                 moments=np.empty((P, 2)), rrr=np.empty(P),
                 iters=np.empty(P, np.int32), status=np.empty(P, np.uint32))
    lsat = None if tab.lsat is None else np.ascontiguousarray(tab.lsat, np.float32)
    endm = _endm(tab, model)
    rc = lib().orc_adam_retrieve(
        tab.B, _dp(tab.lam), _dp(tab.K), _dp(tab.tau2), _dp(tab.tup), _dp(tab.ratm), _dp(tab.S),
        _dp(endm), _fp(lsat), q, _dp(gx), _dp(gw), model, _dp(lo), _dp(hi), _dp(x0), _dp(z0c), P,
        _fp(lobs), k, steps.ctypes.data_as(C.POINTER(C.c_int)),
        free.ctypes.data_as(C.POINTER(C.c_uint)), _dp(lr), _dp(clip), _dp(wlo), _dp(whi),
        _dp(zset), beta1, beta2, eps, nthreads, _dp(out.state), _dp(out.cov), _dp(out.moments),
        _dp(out.rrr), out.iters.ctypes.data_as(C.POINTER(C.c_int)),
        out.status.ctypes.data_as(C.POINTER(C.c_uint)))
    if rc != 0:
        raise ValueError("orc_adam_retrieve: bad arguments")
    return out


# ----------------------------------------------------------------------------
# Fire-candidate pre-filter (Sec. 2.1)
# ----------------------------------------------------------------------------
HFDI_LAMBDA_NM = (2430.0, 2061.0)
HFDI_THRESHOLD = -0.1


def nearest_band(lam, target_nm: float) -> int:
    """Index of the band centre nearest target_nm (the lower index on a tie)."""
    return int(np.argmin(np.abs(np.asarray(lam, np.float64) - target_nm)))


def hfdi(tab: Tables, lobs):
    """Sec. 2.1: HFDI = (L(2430) - L(2061)) / (L(2430) + L(2061)) per pixel,
    L(lambda) the radiance of the nearest band, in float32 arithmetic (the
    precision of the radiance), with IEEE results for a zero sum."""
    lobs = np.asarray(lobs, np.float32)
    a = lobs[:, nearest_band(tab.lam, HFDI_LAMBDA_NM[0])]
    b = lobs[:, nearest_band(tab.lam, HFDI_LAMBDA_NM[1])]
    with np.errstate(divide="ignore", invalid="ignore"):
        return (a - b) / (a + b)


def hfdi_candidates(tab: Tables, lobs, threshold: float = HFDI_THRESHOLD):
    """Candidate pixels in increasing order: HFDI >= threshold (compared in
    double), or either HFDI band saturated (Sec. 2.1 keeps saturated
    candidates: saturation there itself indicates hot emission)."""
    lobs = np.asarray(lobs, np.float32)
    h = hfdi(tab, lobs)
    keep = h.astype(np.float64) >= threshold
    if tab.lsat is not None:
        ia, ib = nearest_band(tab.lam, HFDI_LAMBDA_NM[0]), nearest_band(tab.lam, HFDI_LAMBDA_NM[1])
        keep |= (lobs[:, ia] >= tab.lsat[ia]) | (lobs[:, ib] >= tab.lsat[ib])
    return np.nonzero(keep)[0].astype(np.int64), h


def max_threads() -> int:
    return int(lib().orc_max_threads())


def unpack_cov(packed, n):
    """Packed upper triangle (row-major) -> full symmetric [.., n, n]."""
    packed = np.asarray(packed)
    out = np.empty(packed.shape[:-1] + (n, n))
    pos = 0
    for i in range(n):
        for j in range(i, n):
            out[..., i, j] = packed[..., pos]
            out[..., j, i] = packed[..., pos]
            pos += 1
    return out
