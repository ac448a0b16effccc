"""firefit: per-pixel full-physics inversion of VSWIR radiance for sub-pixel
fire temperature on AMD Instinct MI355X (gfx950).

Thin Python binding of the C-ABI library ``libfirefit.so`` (``include/firefit.h``):
argument marshalling only.  Every step of the retrieval -- band resampling,
forward model, Jacobian, reductions, damped solves, covariance, moments --
runs in the library's HIP kernels.  torch is used for device memory and
streams.  There is no CPU fallback: if the library is not built, importing
works but every call raises.
"""
from __future__ import annotations

import ctypes as C
from contextlib import nullcontext as _nullcontext
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfirefit.so")

FF_OK, FF_EINVAL, FF_EDEVICE, FF_ENOMEM, FF_EUNSUPPORTED = 0, -1, -2, -3, -4
MODEL_LOGNORMAL_1, MODEL_LOGNORMAL_2, MODEL_GAUSS_GRID_2, MODEL_ENDMEMBER_1, MODEL_FULL = 1, 2, 3, 4, 5
N_ENDMEMBERS = 5
PRECISION_FP32, PRECISION_FP64 = 0, 1
SCHEDULE_PERSISTENT, SCHEDULE_STATIC = 0, 1
ACCUMULATE_FP32, ACCUMULATE_FP64 = 0, 1
MAX_STATE = 11
TABLE_COLS = 12

ST_CONVERGED_GTOL, ST_CONVERGED_XTOL, ST_CONVERGED_FTOL = 1, 2, 4
ST_MAX_ITER, ST_NONFINITE_INPUT, ST_DAMPING_OVERFLOW = 8, 16, 32
ST_COV_SINGULAR, ST_AT_BOUND, ST_USED_FALLBACK, ST_WARM_START, ST_NO_DOF = 64, 128, 256, 512, 1024
ST_BAD_ATMOSPHERE = 2048
MAX_ATMOSPHERES = 16
ST_CONVERGED = ST_CONVERGED_GTOL | ST_CONVERGED_XTOL | ST_CONVERGED_FTOL

N_STATE = {MODEL_LOGNORMAL_1: 5, MODEL_LOGNORMAL_2: 8, MODEL_GAUSS_GRID_2: 8, MODEL_ENDMEMBER_1: 8,
           MODEL_FULL: 11}

# exported symbols of include/firefit.h
EXPORTS = ("ff_version", "ff_status_string", "ff_last_error", "ff_options_default",
           "ff_prior_default", "ff_gauss_hermite", "ff_scene_create", "ff_scene_destroy",
           "ff_scene_n_bands", "ff_scene_band_tables", "ff_forward", "ff_retrieve_scene",
           "ff_retrieve_batch", "ff_retrieve", "ff_tune",
           "ff_mlp_create", "ff_mlp_destroy", "ff_mlp_n_params", "ff_mlp_get_params",
           "ff_mlp_set_params", "ff_mlp_set_normalization", "ff_mlp_get_normalization",
           "ff_mlp_fit_normalization", "ff_mlp_infer", "ff_mlp_infer_listed", "ff_mlp_gradients",
           "ff_mlp_train_step",
           "ff_mlp_generate", "ff_mlp_train", "ff_pipeline_create", "ff_pipeline_launch", "ff_pipeline_z0",
           "ff_pipeline_destroy", "ff_release_scratch", "ff_adam_options_default", "ff_adam_retrieve_batch",
           "ff_hfdi_candidates", "ff_retrieve_listed", "ff_retrieve_atm_indexed", "ff_block_mean", "ff_qec",
           "ff_scene_set_endmembers", "ff_scene_endmembers", "ff_tune_quadrature",
           "ff_retrieve_batch_noalloc", "ff_mlp_train_span", "ff_mlp_steps_done", "ff_warmstart_save",
           "ff_warmstart_load", "ff_mlp_sizes", "ff_valu_rates", "ff_pipeline_create_routed")


class FirefitError(RuntimeError):
    pass


# ----------------------------------------------------------------------------
# C structures (layout of include/firefit.h)
# ----------------------------------------------------------------------------
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


class ffSrf(C.Structure):
    _fields_ = [("n_bands", C.c_int32), ("wavelength_nm", _dp), ("fwhm_nm", _dp)]


class ffAtmosphere(C.Structure):
    _fields_ = [("n_hr", C.c_int32), ("lambda_nm", _dp), ("e_solar", _dp), ("tau_down", _dp),
                ("tau_up", _dp), ("rho_atm", _dp), ("s_sph", _dp), ("cos_sza", C.c_double),
                ("sat_level", _fp)]


class ffPrior(C.Structure):
    _fields_ = [("model", C.c_int32), ("lo", C.c_double * MAX_STATE),
                ("hi", C.c_double * MAX_STATE), ("x0", C.c_double * MAX_STATE)]


class ffOptions(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("precision", C.c_int32), ("n_quad", C.c_int32),
                ("schedule", C.c_int32), ("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("fallback", C.c_int32), ("accumulate", C.c_int32), ("lanes_per_pixel", C.c_int32),
                ("warm_max_iter", C.c_int32),
                ("xtol", C.c_double),
                ("ftol", C.c_double), ("gtol", C.c_double), ("kappa", C.c_double),
                ("tau", C.c_double), ("ftol_undetected", C.c_double), ("f_detect", C.c_double)]


MAX_ADAM_STAGES = 4


class ffAdamStage(C.Structure):
    _fields_ = [("steps", C.c_int32), ("free_mask", C.c_uint32), ("lr", C.c_double), ("clip_norm", C.c_double),
                ("window_lo_nm", C.c_double * MAX_STATE), ("window_hi_nm", C.c_double * MAX_STATE),
                ("z_start", C.c_double * MAX_STATE)]


class ffAdamOptions(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("precision", C.c_int32), ("accumulate", C.c_int32),
                ("n_quad", C.c_int32), ("block_size", C.c_int32), ("lanes_per_pixel", C.c_int32),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("stage", ffAdamStage * MAX_ADAM_STAGES)]


class ffOutputs(C.Structure):
    _fields_ = [("state", C.c_void_p), ("cov_packed", C.c_void_p), ("moments", C.c_void_p),
                ("rrr", C.c_void_p), ("iters", C.c_void_p), ("status", C.c_void_p),
                ("state_f64", C.c_void_p)]


_lib = None


def lib():
    """The loaded C library; raises FirefitError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FirefitError(f"{LIB_PATH} is missing: build it with paper_2608_07580_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        L.ff_version.restype = C.c_char_p
        L.ff_status_string.restype = C.c_char_p
        L.ff_status_string.argtypes = [C.c_int32]
        L.ff_last_error.restype = C.c_char_p
        L.ff_options_default.argtypes = [C.POINTER(ffOptions)]
        L.ff_prior_default.argtypes = [C.c_int32, C.POINTER(ffPrior)]
        L.ff_gauss_hermite.argtypes = [C.c_int32, _dp, _dp]
        L.ff_scene_create.argtypes = [C.POINTER(ffSrf), C.POINTER(ffAtmosphere), C.POINTER(C.c_void_p)]
        L.ff_scene_destroy.argtypes = [C.c_void_p]
        L.ff_scene_destroy.restype = None
        L.ff_scene_n_bands.argtypes = [C.c_void_p]
        L.ff_scene_band_tables.argtypes = [C.c_void_p, _dp]
        L.ff_scene_set_endmembers.argtypes = [C.c_void_p, C.c_int32, _dp, _dp]
        L.ff_tune_quadrature.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.c_int32, C.POINTER(ffPrior), C.POINTER(C.c_void_p),
                                         C.POINTER(ffOptions), C.POINTER(ffOutputs), C.POINTER(ffOutputs),
                                         C.c_char_p, C.c_int32, _dp, C.c_void_p]
        L.ff_scene_endmembers.argtypes = [C.c_void_p, _dp]
        L.ff_forward.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ff_retrieve_scene.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(ffPrior),
                                        C.c_void_p, C.POINTER(ffOptions), C.POINTER(ffOutputs),
                                        C.c_void_p, C.c_void_p]
        L.ff_retrieve_batch.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_int64), C.c_int32, C.POINTER(ffPrior),
                                        C.POINTER(C.c_void_p), C.POINTER(ffOptions),
                                        C.POINTER(ffOutputs), C.c_void_p, C.c_void_p]
        L.ff_retrieve_batch_noalloc.argtypes = L.ff_retrieve_batch.argtypes
        L.ff_retrieve.argtypes = [C.c_void_p, C.c_int64, C.POINTER(ffSrf), C.POINTER(ffAtmosphere),
                                  C.POINTER(ffPrior), C.c_void_p, C.POINTER(ffOptions),
                                  C.POINTER(ffOutputs), C.c_void_p]
        L.ff_tune.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_int32,
                              C.POINTER(ffPrior), C.POINTER(C.c_void_p), C.POINTER(ffOptions),
                              C.POINTER(ffOutputs), C.c_char_p, C.c_int32, _dp, C.c_void_p]
        vp = C.c_void_p
        L.ff_mlp_create.argtypes = [C.c_int32] * 5 + [C.c_uint64, C.POINTER(vp)]
        L.ff_mlp_destroy.argtypes = [vp]
        L.ff_mlp_destroy.restype = None
        L.ff_mlp_n_params.argtypes = [vp]
        L.ff_mlp_n_params.restype = C.c_int64
        L.ff_mlp_get_params.argtypes = [vp, _fp]
        L.ff_mlp_set_params.argtypes = [vp, _fp]
        L.ff_mlp_set_normalization.argtypes = [vp, _fp, _fp, C.c_float]
        L.ff_mlp_get_normalization.argtypes = [vp, _fp, _fp, _fp]
        L.ff_mlp_fit_normalization.argtypes = [vp, vp, C.c_int64, C.c_float, vp]
        L.ff_mlp_infer.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.ff_mlp_infer_listed.argtypes = [vp, vp, C.c_int64, vp, C.c_int64, vp, vp]
        L.ff_mlp_gradients.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
        L.ff_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, vp, vp]
        L.ff_mlp_generate.argtypes = [vp, C.POINTER(ffPrior), C.c_uint64, C.c_uint64, C.c_int64, C.c_double,
                                      C.c_double, vp, vp, vp, vp]
        L.ff_mlp_train.argtypes = [vp, vp, C.POINTER(ffPrior), C.c_int64, C.c_int32, C.c_uint64, C.c_double,
                                   C.c_double, C.c_float, C.c_float, vp, vp]
        L.ff_mlp_train_span.argtypes = [vp, vp, C.POINTER(ffPrior), C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                        C.c_uint64, C.c_double, C.c_double, C.c_float, C.c_float, vp, vp]
        L.ff_mlp_steps_done.argtypes = [vp]
        L.ff_mlp_steps_done.restype = C.c_int64
        L.ff_warmstart_save.argtypes = [vp, C.c_char_p]
        L.ff_warmstart_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.ff_mlp_sizes.argtypes = [vp, C.POINTER(C.c_int32)]
        L.ff_valu_rates.argtypes = [_dp, C.c_int32, vp]
        L.ff_pipeline_create.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32,
                                         C.POINTER(ffPrior), C.POINTER(vp), C.POINTER(ffOptions),
                                         C.POINTER(ffOutputs), vp, vp, C.POINTER(vp)]
        L.ff_pipeline_create_routed.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32,
                                                C.POINTER(ffPrior), C.POINTER(vp), C.c_double, C.POINTER(ffOptions),
                                                C.POINTER(ffOutputs), vp, vp, C.POINTER(vp)]
        L.ff_pipeline_launch.argtypes = [vp, vp]
        L.ff_pipeline_z0.argtypes = [vp]
        L.ff_pipeline_z0.restype = vp
        L.ff_pipeline_destroy.argtypes = [vp]
        L.ff_pipeline_destroy.restype = None
        L.ff_adam_options_default.argtypes = [C.POINTER(ffPrior), C.POINTER(ffAdamOptions)]
        L.ff_adam_retrieve_batch.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                             C.POINTER(C.c_int64), C.c_int32, C.POINTER(ffPrior),
                                             C.POINTER(C.c_void_p), C.POINTER(ffAdamOptions),
                                             C.POINTER(ffOutputs), C.c_void_p, C.c_void_p]
        L.ff_hfdi_candidates.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]
        L.ff_retrieve_listed.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.POINTER(ffPrior), C.c_void_p, C.POINTER(ffOptions),
                                         C.POINTER(ffOutputs), C.c_void_p, C.c_void_p]
        L.ff_retrieve_atm_indexed.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                              C.POINTER(ffPrior), C.c_void_p, C.POINTER(ffOptions),
                                              C.POINTER(ffOutputs), C.c_void_p, C.c_void_p]
        L.ff_block_mean.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
        L.ff_qec.argtypes = [C.c_void_p] * 8 + [C.c_int32] * 4 + [C.c_double, C.c_int32, C.c_int32, _dp] + \
            [C.c_void_p] * 4
        for name in ("ff_tune_quadrature", "ff_scene_set_endmembers", "ff_scene_endmembers", "ff_block_mean", "ff_qec", "ff_retrieve_atm_indexed", "ff_hfdi_candidates", "ff_retrieve_listed", "ff_adam_options_default", "ff_adam_retrieve_batch",
                     "ff_pipeline_create", "ff_pipeline_create_routed", "ff_pipeline_launch", "ff_release_scratch",
                     "ff_gauss_hermite", "ff_scene_create", "ff_scene_band_tables", "ff_forward",
                     "ff_retrieve_scene", "ff_retrieve_batch", "ff_retrieve_batch_noalloc", "ff_retrieve",
                     "ff_prior_default", "ff_tune",
                     "ff_mlp_create", "ff_mlp_get_params", "ff_mlp_set_params", "ff_mlp_set_normalization",
                     "ff_mlp_get_normalization", "ff_mlp_fit_normalization", "ff_mlp_infer",
                     "ff_mlp_infer_listed", "ff_mlp_gradients", "ff_mlp_train_step", "ff_mlp_generate", "ff_mlp_train",
                     "ff_mlp_train_span", "ff_warmstart_save", "ff_warmstart_load", "ff_mlp_sizes",
                     "ff_valu_rates"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != FF_OK:
        msg = lib().ff_last_error().decode()
        raise FirefitError(f"{what}: {lib().ff_status_string(rc).decode()} ({rc}): {msg}")


VALU_RATE_NAMES = ("fma_f32", "exp2_f32", "rcp_f32", "fma_f64", "cvt_f32_f64", "planck_node")


def valu_rates(stream=None) -> dict:
    """ff_valu_rates: sustained lane-operations per second on the current device."""
    r = np.zeros(6)
    _check(lib().ff_valu_rates(r.ctypes.data_as(_dp), 6, _stream_handle(stream)), "ff_valu_rates")
    return dict(zip(VALU_RATE_NAMES, r.tolist()))


def version() -> str:
    return lib().ff_version().decode()


def gauss_hermite(q: int = 32):
    x = np.empty(q)
    w = np.empty(q)
    _check(lib().ff_gauss_hermite(q, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp)), "ff_gauss_hermite")
    return x, w


def default_options(**kw) -> ffOptions:
    o = ffOptions()
    lib().ff_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


@dataclass
class Prior:
    model: int
    lo: np.ndarray
    hi: np.ndarray
    x0: np.ndarray

    def to_c(self) -> ffPrior:
        p = ffPrior()
        p.model = self.model
        n = N_STATE[self.model]
        for j in range(MAX_STATE):
            p.lo[j] = float(self.lo[j]) if j < n else 0.0
            p.hi[j] = float(self.hi[j]) if j < n else 1.0
            p.x0[j] = float(self.x0[j]) if j < n else 0.5
        return p


def default_prior(model: int = MODEL_LOGNORMAL_1) -> Prior:
    p = ffPrior()
    _check(lib().ff_prior_default(model, C.byref(p)), "ff_prior_default")
    n = N_STATE[model]
    return Prior(model, np.array(p.lo[:n]), np.array(p.hi[:n]), np.array(p.x0[:n]))


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class Scene:
    """Per-scene band tables on the current device (ff_scene)."""

    def __init__(self, atmosphere):
        a = atmosphere
        self._keep = [np.ascontiguousarray(x, np.float64) for x in
                      (a.wavelength_nm, a.fwhm_nm, a.hr_lambda_nm, a.e_solar, a.tau_down,
                       a.tau_up, a.rho_atm, a.s_sph)]
        lam, fwhm, hr, e, tdn, tup, ratm, ssph = self._keep
        sat = None if getattr(a, "sat_level", None) is None else np.ascontiguousarray(a.sat_level, np.float32)
        self._sat = sat
        srf = ffSrf(len(lam), lam.ctypes.data_as(_dp), fwhm.ctypes.data_as(_dp))
        atm = ffAtmosphere(len(hr), hr.ctypes.data_as(_dp), e.ctypes.data_as(_dp),
                           tdn.ctypes.data_as(_dp), tup.ctypes.data_as(_dp), ratm.ctypes.data_as(_dp),
                           ssph.ctypes.data_as(_dp), float(a.cos_sza),
                           sat.ctypes.data_as(_fp) if sat is not None else None)
        h = C.c_void_p()
        _check(lib().ff_scene_create(C.byref(srf), C.byref(atm), C.byref(h)), "ff_scene_create")
        self.handle = h
        self.n_bands = int(lib().ff_scene_n_bands(h))

    def band_tables(self) -> np.ndarray:
        out = np.empty((self.n_bands, TABLE_COLS))
        _check(lib().ff_scene_band_tables(self.handle, out.ctypes.data_as(_dp)), "ff_scene_band_tables")
        return out

    def set_endmembers(self, hr_lambda_nm, reflectance):
        """ff_scene_set_endmembers: the library [N_ENDMEMBERS, n_hr] on the
        high-resolution grid, resampled to the bands on the device."""
        lam = np.ascontiguousarray(hr_lambda_nm, np.float64)
        refl = np.ascontiguousarray(reflectance, np.float64)
        if refl.shape != (N_ENDMEMBERS, lam.size):
            raise ValueError("reflectance must be [N_ENDMEMBERS, n_hr]")
        _check(lib().ff_scene_set_endmembers(self.handle, lam.size, lam.ctypes.data_as(_dp),
                                             refl.ctypes.data_as(_dp)), "ff_scene_set_endmembers")
        return self

    def endmembers(self) -> np.ndarray:
        """ff_scene_endmembers: the band-resampled library [N_ENDMEMBERS, n_bands]."""
        out = np.empty((N_ENDMEMBERS, self.n_bands))
        _check(lib().ff_scene_endmembers(self.handle, out.ctypes.data_as(_dp)), "ff_scene_endmembers")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().ff_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward(scene: Scene, state, model: int = MODEL_LOGNORMAL_1, n_quad: int = 32,
            jacobian: bool = False, stream=None):
    """Model radiance [P, B] (and dL/dx [P, B, n]) at device states [P, n]
    (float32 -> FP32 kernels, float64 -> FP64 kernels)."""
    torch = _torch()
    n = N_STATE[model]
    assert state.is_cuda and state.dim() == 2 and state.shape[1] == n and state.is_contiguous()
    prec = PRECISION_FP64 if state.dtype == torch.float64 else PRECISION_FP32
    assert state.dtype in (torch.float32, torch.float64)
    P = state.shape[0]
    L = torch.empty((P, scene.n_bands), dtype=state.dtype, device=state.device)
    J = torch.empty((P, scene.n_bands, n), dtype=state.dtype, device=state.device) if jacobian else None
    _check(lib().ff_forward(scene.handle, model, prec, n_quad, _ptr(state), P, _ptr(L), _ptr(J),
                            _stream_handle(stream)), "ff_forward")
    return (L, J) if jacobian else L


@dataclass
class Outputs:
    state: object
    cov: object
    moments: object
    rrr: object
    iters: object
    status: object
    state_f64: object | None = None

    def to_c(self) -> ffOutputs:
        return ffOutputs(_ptr(self.state), _ptr(self.cov), _ptr(self.moments), _ptr(self.rrr),
                         _ptr(self.iters), _ptr(self.status), _ptr(self.state_f64))

    def numpy(self) -> dict:
        d = {k: getattr(self, k) for k in ("state", "cov", "moments", "rrr", "iters", "status", "state_f64")}
        return {k: (None if v is None else v.cpu().numpy()) for k, v in d.items()}


def allocate_outputs(P: int, model: int, device, state_f64: bool = False) -> Outputs:
    torch = _torch()
    n = N_STATE[model]
    return Outputs(state=torch.empty((P, n), dtype=torch.float32, device=device),
                   cov=torch.empty((P, n * (n + 1) // 2), dtype=torch.float32, device=device),
                   moments=torch.empty((P, 2), dtype=torch.float32, device=device),
                   rrr=torch.empty(P, dtype=torch.float32, device=device),
                   iters=torch.empty(P, dtype=torch.int32, device=device),
                   status=torch.empty(P, dtype=torch.int32, device=device),
                   state_f64=torch.empty((P, n), dtype=torch.float64, device=device) if state_f64 else None)


def retrieve(scene: Scene, radiance, prior: Prior | None = None, z0=None, options: ffOptions | None = None,
             outputs: Outputs | None = None, evals=None, stream=None, state_f64: bool = False) -> Outputs:
    """Levenberg-Marquardt retrieval of every pixel of radiance [P, B] float32 (device)."""
    torch = _torch()
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    options = options or default_options()
    assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
    assert radiance.dim() == 2 and radiance.shape[1] == scene.n_bands
    P = radiance.shape[0]
    if z0 is not None:
        assert z0.is_cuda and z0.dtype == torch.float32 and z0.is_contiguous()
        assert tuple(z0.shape) == (P, N_STATE[prior.model])
    out = outputs or allocate_outputs(P, prior.model, radiance.device, state_f64)
    pc = prior.to_c()
    oc = out.to_c()
    _check(lib().ff_retrieve_scene(scene.handle, _ptr(radiance), P, C.byref(pc), _ptr(z0),
                                   C.byref(options), C.byref(oc), _ptr(evals), _stream_handle(stream)),
           "ff_retrieve_scene")
    return out


NOALLOC_MAX_SCENES = 64


def retrieve_batch(scenes, radiances, prior: Prior | None = None, z0s=None, options: ffOptions | None = None,
                   outputs=None, evals=None, stream=None) -> list:
    """One launch sequence over a ragged batch of scenes (same band count)."""
    return _retrieve_batch("ff_retrieve_batch", scenes, radiances, prior, z0s, options, outputs, evals, stream)


def retrieve_batch_noalloc(scenes, radiances, outputs, prior: Prior | None = None, z0s=None,
                           options: ffOptions | None = None, evals=None, stream=None) -> list:
    """ff_retrieve_batch_noalloc: the same retrieval with the library's fixed
    device array as scratch (the caller passes the outputs)."""
    return _retrieve_batch("ff_retrieve_batch_noalloc", scenes, radiances, prior, z0s, options, outputs, evals,
                           stream)


def _retrieve_batch(fn, scenes, radiances, prior, z0s, options, outputs, evals, stream) -> list:
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    options = options or default_options()
    ns = len(scenes)
    outs = outputs or [allocate_outputs(r.shape[0], prior.model, r.device) for r in radiances]
    sc = (C.c_void_p * ns)(*[s.handle.value for s in scenes])
    rd = (C.c_void_p * ns)(*[r.data_ptr() for r in radiances])
    Ps = (C.c_int64 * ns)(*[r.shape[0] for r in radiances])
    z0p = None
    if z0s is not None:
        z0p = (C.c_void_p * ns)(*[0 if z is None else z.data_ptr() for z in z0s])
    oc = (ffOutputs * ns)(*[o.to_c() for o in outs])
    pc = prior.to_c()
    _check(getattr(lib(), fn)(sc, rd, Ps, ns, C.byref(pc), z0p, C.byref(options), oc, _ptr(evals),
                              _stream_handle(stream)), fn)
    return outs


HFDI_THRESHOLD = -0.1


def hfdi_candidates(scene: Scene, radiance, threshold: float = HFDI_THRESHOLD, with_index_values: bool = True,
                    stream=None):
    """Fire-candidate pre-filter (ff_hfdi_candidates) on radiance [P, B]
    float32 (device).  Returns (index [P] int64 whose first count entries are
    the candidates in increasing order, count [1] int64, hfdi [P] float32 or
    None), all on the device; the count is not read back."""
    torch = _torch()
    assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
    assert radiance.dim() == 2 and radiance.shape[1] == scene.n_bands
    P = radiance.shape[0]
    index = torch.empty(P, dtype=torch.int64, device=radiance.device)
    count = torch.empty(1, dtype=torch.int64, device=radiance.device)
    h = torch.empty(P, dtype=torch.float32, device=radiance.device) if with_index_values else None
    _check(lib().ff_hfdi_candidates(scene.handle, _ptr(radiance), P, float(threshold), _ptr(h), _ptr(index),
                                    _ptr(count), _stream_handle(stream)), "ff_hfdi_candidates")
    return index, count, h


def retrieve_listed(scene: Scene, radiance, index, count, prior: Prior | None = None, z0=None,
                    options: ffOptions | None = None, outputs: Outputs | None = None, evals=None,
                    stream=None, state_f64: bool = False) -> Outputs:
    """Retrieve only the rows listed by (index, count) (ff_retrieve_listed);
    outputs are [P]-sized and unlisted rows are left as they were."""
    torch = _torch()
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    options = options or default_options()
    assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
    assert radiance.dim() == 2 and radiance.shape[1] == scene.n_bands
    P = radiance.shape[0]
    assert index.is_cuda and index.dtype == torch.int64 and index.numel() >= 1 and index.is_contiguous()
    assert count.is_cuda and count.dtype == torch.int64 and count.numel() == 1
    if z0 is not None:
        assert z0.is_cuda and z0.dtype == torch.float32 and z0.is_contiguous()
        assert tuple(z0.shape) == (P, N_STATE[prior.model])
    out = outputs or allocate_outputs(P, prior.model, radiance.device, state_f64)
    pc = prior.to_c()
    oc = out.to_c()
    _check(lib().ff_retrieve_listed(scene.handle, _ptr(radiance), P, _ptr(index), _ptr(count), C.byref(pc),
                                    _ptr(z0), C.byref(options), C.byref(oc), _ptr(evals),
                                    _stream_handle(stream)), "ff_retrieve_listed")
    return out


def retrieve_atm_indexed(atmospheres, atm_index, radiance, prior: Prior | None = None, z0=None,
                         options: ffOptions | None = None, outputs: Outputs | None = None, evals=None,
                         stream=None, state_f64: bool = False) -> Outputs:
    """Retrieval with a per-pixel atmosphere (ff_retrieve_atm_indexed): pixel p
    uses atmospheres[atm_index[p]] (atm_index: [P] int32 device tensor)."""
    torch = _torch()
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    options = options or default_options()
    assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
    P = radiance.shape[0]
    assert atm_index.is_cuda and atm_index.dtype == torch.int32 and atm_index.numel() == P
    if z0 is not None:
        assert z0.is_cuda and z0.dtype == torch.float32 and z0.is_contiguous()
    out = outputs or allocate_outputs(P, prior.model, radiance.device, state_f64)
    na = len(atmospheres)
    sc = (C.c_void_p * na)(*[s.handle.value for s in atmospheres])
    pc = prior.to_c()
    oc = out.to_c()
    _check(lib().ff_retrieve_atm_indexed(sc, na, _ptr(atm_index), _ptr(radiance), P, C.byref(pc), _ptr(z0),
                                         C.byref(options), C.byref(oc), _ptr(evals), _stream_handle(stream)),
           "ff_retrieve_atm_indexed")
    return out


QEC_LEVELS = (0.05, 0.10, 0.25, 0.50, 0.75, 0.90, 0.95)


def block_mean(radiance, rows: int, cols: int, block: int = 12, stream=None):
    """Coarse radiance [(rows // block) * (cols // block), B] float32 from fine
    radiance [rows * cols, B] (ff_block_mean)."""
    torch = _torch()
    assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
    assert radiance.shape[0] == rows * cols
    B = radiance.shape[1]
    out = torch.empty(((rows // block) * (cols // block), B), dtype=torch.float32, device=radiance.device)
    _check(lib().ff_block_mean(_ptr(radiance), rows, cols, B, block, _ptr(out), _stream_handle(stream)),
           "ff_block_mean")
    return out


def qec(fine: Outputs, coarse: Outputs, rows: int, cols: int, block: int = 12, f_min: float = 1e-4,
        min_fine: int = 5, levels=QEC_LEVELS, fine_mask=None, coarse_mask=None, stream=None):
    """Quantile Error Curves of every coarse pixel (ff_qec): (empirical [K, L],
    mixture [K, L], n_used [K]) device tensors, NaN where not evaluated.
    fine_mask / coarse_mask: optional uint8 device tensors restricting the
    pixels that take part."""
    torch = _torch()
    K = (rows // block) * (cols // block)
    n = fine.state.shape[1]
    lv = np.ascontiguousarray(levels, np.float64)
    dev = fine.state.device
    emp = torch.empty((K, len(lv)), dtype=torch.float32, device=dev)
    mix = torch.empty_like(emp)
    n_used = torch.empty(K, dtype=torch.int32, device=dev)
    for m, size in ((fine_mask, fine.state.shape[0]), (coarse_mask, K)):
        if m is not None:
            assert m.is_cuda and m.dtype == torch.uint8 and m.numel() == size and m.is_contiguous()
    _check(lib().ff_qec(_ptr(fine.moments), _ptr(fine.state), _ptr(fine.status), _ptr(fine_mask),
                        _ptr(coarse.moments), _ptr(coarse.state), _ptr(coarse.status), _ptr(coarse_mask), n,
                        rows, cols, block, float(f_min), min_fine,
                        len(lv), lv.ctypes.data_as(_dp), _ptr(emp), _ptr(mix), _ptr(n_used),
                        _stream_handle(stream)), "ff_qec")
    return emp, mix, n_used


def adam_options(prior: Prior | None = None, **kw) -> ffAdamOptions:
    """The paper's two-stage Adam schedule for `prior` (ff_adam_options_default);
    keyword arguments override top-level fields."""
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    o = ffAdamOptions()
    pc = prior.to_c()
    _check(lib().ff_adam_options_default(C.byref(pc), C.byref(o)), "ff_adam_options_default")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def set_adam_stages(opts: ffAdamOptions, stages) -> ffAdamOptions:
    """Replace the stages of `opts`.  Each stage is a mapping with keys
    steps, lr, free (variable indices), window ({j: (lo_nm, hi_nm)}), and
    optionally clip (default 1.0) and zset ({j: z at the stage start})."""
    if len(stages) > MAX_ADAM_STAGES:
        raise ValueError(f"at most {MAX_ADAM_STAGES} stages")
    opts.n_stages = len(stages)
    for k in range(MAX_ADAM_STAGES):
        st = ffAdamStage()
        for j in range(MAX_STATE):
            st.z_start[j] = float("nan")
        if k < len(stages):
            d = stages[k]
            st.steps = int(d["steps"])
            st.lr = float(d["lr"])
            st.clip_norm = float(d.get("clip", 1.0))
            for j in d["free"]:
                st.free_mask |= 1 << j
                st.window_lo_nm[j], st.window_hi_nm[j] = d["window"][j]
            for j, v in (d.get("zset") or {}).items():
                st.z_start[j] = float(v)
        opts.stage[k] = st
    return opts


def adam_retrieve_batch(scenes, radiances, prior: Prior | None = None, z0s=None,
                        options: ffAdamOptions | None = None, outputs=None, evals=None, stream=None) -> list:
    """The paper's staged-Adam solver over a ragged batch (ff_adam_retrieve_batch)."""
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    options = options or adam_options(prior)
    ns = len(scenes)
    outs = outputs or [allocate_outputs(r.shape[0], prior.model, r.device) for r in radiances]
    sc = (C.c_void_p * ns)(*[s.handle.value for s in scenes])
    rd = (C.c_void_p * ns)(*[r.data_ptr() for r in radiances])
    Ps = (C.c_int64 * ns)(*[r.shape[0] for r in radiances])
    z0p = None
    if z0s is not None:
        z0p = (C.c_void_p * ns)(*[0 if z is None else z.data_ptr() for z in z0s])
    oc = (ffOutputs * ns)(*[o.to_c() for o in outs])
    pc = prior.to_c()
    _check(lib().ff_adam_retrieve_batch(sc, rd, Ps, ns, C.byref(pc), z0p, C.byref(options), oc, _ptr(evals),
                                        _stream_handle(stream)), "ff_adam_retrieve_batch")
    return outs


def adam_retrieve(scene: Scene, radiance, prior: Prior | None = None, z0=None,
                  options: ffAdamOptions | None = None, outputs: Outputs | None = None, evals=None,
                  stream=None, state_f64: bool = False) -> Outputs:
    """The paper's staged-Adam solver on every pixel of radiance [P, B] float32 (device)."""
    torch = _torch()
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
    assert radiance.dim() == 2 and radiance.shape[1] == scene.n_bands
    P = radiance.shape[0]
    if z0 is not None:
        assert z0.is_cuda and z0.dtype == torch.float32 and z0.is_contiguous()
        assert tuple(z0.shape) == (P, N_STATE[prior.model])
    out = outputs or allocate_outputs(P, prior.model, radiance.device, state_f64)
    return adam_retrieve_batch([scene], [radiance], prior, None if z0 is None else [z0], options, [out],
                               evals, stream)[0]


TUNE_IGNORE_CACHE = 1


def tune(scenes, radiances, prior: Prior | None = None, z0s=None, options: ffOptions | None = None,
         cache_path: str | None = None, retune: bool = False, stream=None):
    """Launch-shape autotuner (ff_tune) on a batch: returns (options, best_ms).

    `scenes`/`radiances`/`z0s` are lists (one scene: lists of one).  The
    chosen lanes per pixel, workgroup size, workgroups per CU and schedule
    are written into a copy of `options`; with `cache_path` the choice is
    read from / stored in that JSON table."""
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    opts = ffOptions()
    C.memmove(C.byref(opts), C.byref(options or default_options()), C.sizeof(ffOptions))
    ns = len(scenes)
    outs = [allocate_outputs(r.shape[0], prior.model, r.device) for r in radiances]
    sc = (C.c_void_p * ns)(*[s.handle.value for s in scenes])
    rd = (C.c_void_p * ns)(*[r.data_ptr() for r in radiances])
    Ps = (C.c_int64 * ns)(*[r.shape[0] for r in radiances])
    z0p = None
    if z0s is not None:
        z0p = (C.c_void_p * ns)(*[0 if z is None else z.data_ptr() for z in z0s])
    oc = (ffOutputs * ns)(*[o.to_c() for o in outs])
    pc = prior.to_c()
    ms = C.c_double(0.0)
    _check(lib().ff_tune(sc, rd, Ps, ns, C.byref(pc), z0p, C.byref(opts), oc,
                         None if cache_path is None else os.fsencode(cache_path),
                         TUNE_IGNORE_CACHE if retune else 0, C.byref(ms), _stream_handle(stream)), "ff_tune")
    return opts, ms.value


def tune_quadrature(scenes, radiances, prior: Prior | None = None, z0s=None, options: ffOptions | None = None,
                    cache_path: str | None = None, retune: bool = False, stream=None):
    """Quadrature-order choice (ff_tune_quadrature): returns (options, report)
    with report = {chosen order, its ms, requested order's ms, agreeing
    share, and per tested order (24, 16) its share and ms}."""
    prior = prior or default_prior(MODEL_LOGNORMAL_1)
    opts = ffOptions()
    C.memmove(C.byref(opts), C.byref(options or default_options()), C.sizeof(ffOptions))
    ns = len(scenes)
    ref = [allocate_outputs(r.shape[0], prior.model, r.device) for r in radiances]
    tri = [allocate_outputs(r.shape[0], prior.model, r.device) for r in radiances]
    sc = (C.c_void_p * ns)(*[s.handle.value for s in scenes])
    rd = (C.c_void_p * ns)(*[r.data_ptr() for r in radiances])
    Ps = (C.c_int64 * ns)(*[r.shape[0] for r in radiances])
    z0p = None
    if z0s is not None:
        z0p = (C.c_void_p * ns)(*[0 if z is None else z.data_ptr() for z in z0s])
    oref = (ffOutputs * ns)(*[o.to_c() for o in ref])
    otri = (ffOutputs * ns)(*[o.to_c() for o in tri])
    pc = prior.to_c()
    rep = np.zeros(8)
    _check(lib().ff_tune_quadrature(sc, rd, Ps, ns, C.byref(pc), z0p, C.byref(opts), oref, otri,
                                    None if cache_path is None else os.fsencode(cache_path),
                                    TUNE_IGNORE_CACHE if retune else 0, rep.ctypes.data_as(_dp),
                                    _stream_handle(stream)), "ff_tune_quadrature")
    report = {"n_quad": int(rep[0]), "ms": float(rep[1]), "ms_requested": float(rep[2]), "share": float(rep[3]),
              "tested": {24: {"share": float(rep[4]), "ms": float(rep[5])},
                         16: {"share": float(rep[6]), "ms": float(rep[7])}}}
    return opts, report


# ----------------------------------------------------------------------------
# learned warm start
# ----------------------------------------------------------------------------
def generate(scene: Scene, prior: Prior, seed: int, offset: int, P: int, snr: float = 300.0,
             bg_fraction: float = 0.0, device=None, stream=None, states: bool = False):
    """Training spectra of the one-component model (ff_mlp_generate)."""
    torch = _torch()
    device = device or torch.device("cuda:0")
    rad = torch.empty((P, scene.n_bands), dtype=torch.float32, device=device)
    tgt = torch.empty((P, 5), dtype=torch.float32, device=device)
    st = torch.empty((P, 5), dtype=torch.float32, device=device) if states else None
    pc = prior.to_c()
    _check(lib().ff_mlp_generate(scene.handle, C.byref(pc), seed, offset, P, snr, bg_fraction, _ptr(rad),
                                 _ptr(tgt), _ptr(st), _stream_handle(stream)), "ff_mlp_generate")
    return (rad, tgt, st) if states else (rad, tgt)


class WarmStart:
    """The warm-start network (ff_mlp) on the current device."""

    def __init__(self, n_in: int = 284, hidden=(512, 512, 256), n_out: int = 5, seed: int = 0, _handle=None):
        h = C.c_void_p()
        if _handle is None:
            _check(lib().ff_mlp_create(n_in, hidden[0], hidden[1], hidden[2], n_out, seed, C.byref(h)),
                   "ff_mlp_create")
        else:
            h = _handle
        self.handle = h
        self.sizes = (n_in, hidden[0], hidden[1], hidden[2], n_out)
        self.n_params = int(lib().ff_mlp_n_params(h))

    def close(self):
        if getattr(self, "handle", None):
            lib().ff_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, np.float32)
        _check(lib().ff_mlp_get_params(self.handle, p.ctypes.data_as(_fp)), "ff_mlp_get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.shape == (self.n_params,)
        _check(lib().ff_mlp_set_params(self.handle, p.ctypes.data_as(_fp)), "ff_mlp_set_params")

    def set_normalization(self, mean, inv_std, floor: float):
        mean = np.ascontiguousarray(mean, np.float32)
        inv_std = np.ascontiguousarray(inv_std, np.float32)
        _check(lib().ff_mlp_set_normalization(self.handle, mean.ctypes.data_as(_fp), inv_std.ctypes.data_as(_fp),
                                              floor), "ff_mlp_set_normalization")

    def get_normalization(self):
        n = self.sizes[0]
        mean = np.empty(n, np.float32)
        inv = np.empty(n, np.float32)
        fl = np.empty(1, np.float32)
        _check(lib().ff_mlp_get_normalization(self.handle, mean.ctypes.data_as(_fp), inv.ctypes.data_as(_fp),
                                              fl.ctypes.data_as(_fp)), "ff_mlp_get_normalization")
        return mean, inv, float(fl[0])

    def fit_normalization(self, radiance, floor: float = 1e-6, stream=None):
        _check(lib().ff_mlp_fit_normalization(self.handle, _ptr(radiance), radiance.shape[0], floor,
                                              _stream_handle(stream)), "ff_mlp_fit_normalization")

    def infer(self, radiance, stream=None):
        torch = _torch()
        z0 = torch.empty((radiance.shape[0], self.sizes[4]), dtype=torch.float32, device=radiance.device)
        _check(lib().ff_mlp_infer(self.handle, _ptr(radiance), radiance.shape[0], _ptr(z0), _stream_handle(stream)),
               "ff_mlp_infer")
        return z0

    def infer_listed(self, radiance, index, n_listed: int, z0=None, stream=None):
        """z0 rows of the first n_listed pixels named by index (ff_mlp_infer_listed);
        z0 [P, n_out] is allocated (unlisted rows then undefined) or updated in place."""
        torch = _torch()
        assert radiance.is_cuda and radiance.dtype == torch.float32 and radiance.is_contiguous()
        assert index.is_cuda and index.dtype == torch.int64 and index.is_contiguous()
        assert 0 <= n_listed <= index.numel()
        P = radiance.shape[0]
        if z0 is None:
            z0 = torch.empty((P, self.sizes[4]), dtype=torch.float32, device=radiance.device)
        assert z0.is_cuda and z0.dtype == torch.float32 and z0.is_contiguous()
        assert tuple(z0.shape) == (P, self.sizes[4])
        _check(lib().ff_mlp_infer_listed(self.handle, _ptr(radiance), P, _ptr(index), int(n_listed), _ptr(z0),
                                         _stream_handle(stream)), "ff_mlp_infer_listed")
        return z0

    def infer_routed(self, scene, radiance, threshold: float = HFDI_THRESHOLD, z0=None, stream=None):
        """Starts for the fire candidates only: the front end's index (Sec. 2.1,
        ff_hfdi_candidates) picks the pixels, the network (ff_mlp_infer_listed)
        gives their start rows, every other row is NaN (no start: solved from
        x0).  Returns (z0 [P, n_out], number of candidates); the candidate
        count is read back to the host (one synchronisation of the stream)."""
        torch = _torch()
        P = radiance.shape[0]
        idx, cnt, _ = hfdi_candidates(scene, radiance, threshold, with_index_values=False, stream=stream)
        if z0 is None:
            z0 = torch.empty((P, self.sizes[4]), dtype=torch.float32, device=radiance.device)
        with torch.cuda.stream(stream) if stream is not None else _nullcontext():
            z0.fill_(float("nan"))
            n = int(cnt.item())
        self.infer_listed(radiance, idx, n, z0=z0, stream=stream)
        return z0, n

    def gradients(self, radiance, target, stream=None):
        torch = _torch()
        loss = torch.zeros(1, dtype=torch.float64, device=radiance.device)
        g = torch.empty(self.n_params, dtype=torch.float32, device=radiance.device)
        self._pending = (loss, g)
        _check(lib().ff_mlp_gradients(self.handle, _ptr(radiance), _ptr(target), radiance.shape[0], _ptr(loss),
                                      _ptr(g), _stream_handle(stream)), "ff_mlp_gradients")
        return loss, g

    def train_step(self, radiance, target, lr: float, stream=None):
        torch = _torch()
        loss = torch.zeros(1, dtype=torch.float64, device=radiance.device)
        self._pending = loss
        _check(lib().ff_mlp_train_step(self.handle, _ptr(radiance), _ptr(target), radiance.shape[0], lr, _ptr(loss),
                                       _stream_handle(stream)), "ff_mlp_train_step")
        return loss

    def train(self, scene: Scene, prior: Prior, steps: int, batch: int = 2048, seed: int = 1, snr: float = 300.0,
              bg_fraction: float = 0.0, lr: float = 1e-3, lr_final: float = 1e-5, stream=None, device=None,
              first_step: int = 0, n_steps: int | None = None):
        """Steps [first_step, first_step + n_steps) of a schedule of `steps`
        steps (ff_mlp_train_span; default: the whole schedule)."""
        torch = _torch()
        device = device or torch.device("cuda:0")
        n_steps = steps - first_step if n_steps is None else n_steps
        hist = torch.zeros(max(n_steps, 1), dtype=torch.float64, device=device)
        pc = prior.to_c()
        _check(lib().ff_mlp_train_span(self.handle, scene.handle, C.byref(pc), steps, first_step, n_steps, batch,
                                       seed, snr, bg_fraction, lr, lr_final, _ptr(hist), _stream_handle(stream)),
               "ff_mlp_train_span")
        # the kernels still write hist after this returns: keep it alive even
        # if the caller drops it (its block must not be handed out to a
        # tensor used on another stream meanwhile)
        self._pending = hist
        return hist

    @property
    def steps_done(self) -> int:
        """Schedule steps taken (the first_step of a resumed run)."""
        return int(lib().ff_mlp_steps_done(self.handle))

    def save(self, path: str):
        """Checkpoint (ff_warmstart_save): weights, normalisation, Adam
        moments and step counts."""
        _check(lib().ff_warmstart_save(self.handle, os.fsencode(path)), "ff_warmstart_save")

    @classmethod
    def load(cls, path: str):
        """A network from a checkpoint written by save (ff_warmstart_load)."""
        h = C.c_void_p()
        _check(lib().ff_warmstart_load(os.fsencode(path), C.byref(h)), "ff_warmstart_load")
        sz = (C.c_int32 * 5)()
        _check(lib().ff_mlp_sizes(h, sz), "ff_mlp_sizes")
        return cls(sz[0], (sz[1], sz[2], sz[3]), sz[4], _handle=h)


class Pipeline:
    """Graph-captured (warm start +) retrieval of one batch (ff_pipeline_*).

    The graph binds the radiance tensors, outputs and networks given here;
    rewrite the radiance tensors in place (``rad.copy_(new)``) and call
    ``launch()`` again.  ``outputs`` is a list of Outputs, one per scene.
    ``net``: one WarmStart for every scene, or a list (entries may be None).
    ``route``: an HFDI threshold (the paper: -0.1) to run the network only on
    the front end's candidates (ff_pipeline_create_routed), or None."""

    def __init__(self, scenes, radiances, prior: Prior | None = None, net=None,
                 options: ffOptions | None = None, evals=None, stream=None, route: float | None = None):
        torch = _torch()
        self.prior = prior or default_prior(MODEL_LOGNORMAL_1)
        self.options = options or default_options()
        self.scenes, self.radiances, self.evals = list(scenes), list(radiances), evals
        ns = len(self.scenes)
        self.nets = list(net) if isinstance(net, (list, tuple)) else [net] * ns
        assert len(self.nets) == ns
        self.outputs = [allocate_outputs(r.shape[0], self.prior.model, r.device) for r in self.radiances]
        sc = (C.c_void_p * ns)(*[s.handle.value for s in self.scenes])
        rd = (C.c_void_p * ns)(*[r.data_ptr() for r in self.radiances])
        Ps = (C.c_int64 * ns)(*[r.shape[0] for r in self.radiances])
        oc = (ffOutputs * ns)(*[o.to_c() for o in self.outputs])
        pc = self.prior.to_c()
        self.stream = stream or torch.cuda.current_stream()
        h = C.c_void_p()
        nets = None
        if any(n is not None for n in self.nets):
            nets = (C.c_void_p * ns)(*[None if n is None else n.handle.value for n in self.nets])
        if route is None:
            _check(lib().ff_pipeline_create(sc, rd, Ps, ns, C.byref(pc), nets,
                                            C.byref(self.options), oc, _ptr(evals), _stream_handle(self.stream),
                                            C.byref(h)), "ff_pipeline_create")
        else:
            _check(lib().ff_pipeline_create_routed(sc, rd, Ps, ns, C.byref(pc), nets, float(route),
                                                   C.byref(self.options), oc, _ptr(evals),
                                                   _stream_handle(self.stream), C.byref(h)),
                   "ff_pipeline_create_routed")
        self.handle = h

    def launch(self, stream=None):
        _check(lib().ff_pipeline_launch(self.handle, _stream_handle(stream or self.stream)), "ff_pipeline_launch")

    def close(self):
        if getattr(self, "handle", None):
            lib().ff_pipeline_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
