/*
 * firefit: per-pixel full-physics inversion of VSWIR radiance spectra for
 * sub-pixel fire temperature, on AMD Instinct MI355X (gfx950).
 *
 * Method (Keely et al., "Real-time physics inversion for retrieval of
 * sub-pixel wildfire temperatures from VSWIR imaging spectroscopy"):
 *   forward model   L = L_s + L_t                                     (Sec. 2.2, eq. fm)
 *   solar term      L_s = E cos(sza)/pi [rho_atm + tau_dn tau_up rho/(1 - S rho)]  (eq. solar)
 *   thermal term    L_t = f tau_up int p(T) B(lambda, T) dT                          (eq. thermal)
 *   loss            sum_b m_b (L_obs,b - L_b)^2, m_b = 0 for saturated bands          (Sec. 2.5, eq. loss)
 *   coordinates     z = 2 (x - lo)/(hi - lo) - 1, z clipped to [-1, 1]               (eq. affine)
 *   summary         E[T], sigma[T] of the moment-matched temperature mixture        (Sec. 2.2)
 * p(T) is a lognormal of mean m and s.d. s (FF_MODEL_LOGNORMAL_1) or the
 * eta-weighted mixture of a smouldering and a flaming lognormal
 * (FF_MODEL_LOGNORMAL_2), integrated by Gauss-Hermite quadrature in log T,
 * or the paper's Gaussians on a temperature grid (FF_MODEL_GAUSS_GRID_2).
 * The surface reflectance is linear, rho = rho0 + rho1 (lambda - 1440 nm),
 * or the endmember mixture of Sec. 2.2 (FF_MODEL_ENDMEMBER_1, FF_MODEL_FULL).
 * Each pixel is solved by Levenberg-Marquardt (damped Gauss-Newton on the
 * loss in z, active set for variables held at a bound; with the endmember
 * surface the step keeps the fractions' sum, holds fractions at zero by the
 * sign of their reduced gradient and is shortened so none goes negative),
 * and the Gauss-Newton state covariance is reported; the paper's own
 * solver, staged Adam, is available as ff_adam_retrieve_batch.
 *
 * Conventions for every entry point:
 *  - Return value: ff_status, FF_OK (0) on success, negative on error.  No
 *    entry point throws, aborts or exits.  The message of the last error of
 *    the calling thread is available from ff_last_error().
 *  - Argument errors (NULL pointers where a buffer is required, P < 0,
 *    band-count mismatch, lo >= hi, unknown model/precision/quadrature
 *    order) return FF_EINVAL before anything is launched.  HIP runtime
 *    failures return FF_EDEVICE; allocation failures FF_ENOMEM.
 *  - Device buffers ("_dev") are allocated and owned by the caller (for
 *    example torch tensors' data_ptr()); the library only reads/writes them.
 *    Host buffers ("host") are read during the call only.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*, NULL = default stream) and the call returns without waiting,
 *    except ff_scene_create / ff_scene_band_tables / ff_gauss_hermite /
 *    ff_retrieve, which are synchronous.
 *  - Per-pixel failures are not call errors: they are reported in the
 *    status word of each pixel (FF_ST_* bits).
 *  - P = 0 is a valid no-op.
 *  - Calls on different streams may run concurrently; one scene handle may
 *    be used by several streams at once (it is read-only after creation).
 *    Exceptions: calls that use one warm-start network (ff_mlp_*) share its
 *    activation workspace and must be ordered on one stream, and
 *    ff_retrieve_batch_noalloc calls on one device share its fixed array.
 */
#ifndef FIREFIT_H
#define FIREFIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ff_status;
#define FF_OK 0
#define FF_EINVAL (-1)
#define FF_EDEVICE (-2)
#define FF_ENOMEM (-3)
#define FF_EUNSUPPORTED (-4)

/* Temperature-distribution models and their state vectors (physical units):
 *   FF_MODEL_LOGNORMAL_1: n = 5, x = (f, m, s, rho0, rho1)
 *   FF_MODEL_LOGNORMAL_2: n = 8, x = (f, eta, m_s, s_s, m_h, s_h, rho0, rho1)
 *   FF_MODEL_GAUSS_GRID_2: n = 8, x = (f, eta, mu_s, sig_s, mu_h, sig_h, rho0, rho1)
 *   FF_MODEL_ENDMEMBER_1: n = 8, x = (f, m, s, x_1, x_2, x_3, x_4, x_5)
 *   FF_MODEL_FULL: n = 11, x = (f, eta, mu_s, sig_s, mu_h, sig_h, x_1 .. x_5)
 * f: emitting fraction scaling the thermal term (the paper's alpha),
 * m/s: lognormal mean and s.d. in K, eta: weight of the flaming component,
 * rho0: reflectance at 1440 nm, rho1: reflectance slope per nm.  The
 * lognormal models integrate the Planck radiance by n_quad-node
 * Gauss-Hermite quadrature in log T.  FF_MODEL_GAUSS_GRID_2 is the paper's
 * own form (Sec. 2.2): the eta-weighted mixture of a smouldering and a
 * flaming Gaussian of means mu and s.d. sig, each normalised over a grid of
 * n_quad uniform temperatures spanning [350, 2200] K, and the thermal term
 * the grid sum of the Planck radiance.  FF_MODEL_ENDMEMBER_1 replaces the
 * linear reflectance by the paper's surface mixture (Sec. 2.2, library
 * Sec. 2.4): rho(lambda) = sum_k x_k E_k(lambda) over the scene's
 * FF_N_ENDMEMBERS library spectra (ff_scene_set_endmembers), with the
 * fractions on the unit simplex (x_k >= 0, sum x_k = 1); the thermal term
 * is the one-component lognormal.  FF_MODEL_FULL is the paper's full
 * forward model: the FF_MODEL_GAUSS_GRID_2 thermal term over the endmember
 * surface.  Surface fractions must have the box [0, 1]. */
#define FF_MODEL_LOGNORMAL_1 1
#define FF_MODEL_LOGNORMAL_2 2
#define FF_MODEL_GAUSS_GRID_2 3
#define FF_MODEL_ENDMEMBER_1 4
#define FF_MODEL_FULL 5
#define FF_MAX_STATE 11
#define FF_N_ENDMEMBERS 5

/* Arithmetic of the forward model, Jacobian and reductions.  The damped
 * Cholesky solve and the covariance inversion are FP64 in both. */
#define FF_PRECISION_FP32 0
#define FF_PRECISION_FP64 1

/* Accumulation of the per-band sums J^T J, J^T r, r.r on the FP32 path
 * (the FP64 path always accumulates in FP64). */
#define FF_ACCUMULATE_FP32 0
#define FF_ACCUMULATE_FP64 1

/* Work distribution of the retrieval kernel. */
#define FF_SCHEDULE_PERSISTENT 0   /* resident waves pull pixels from a device queue; a lane refills as its pixel converges */
#define FF_SCHEDULE_STATIC 1       /* one pixel per lane, one launch covers all pixels */

/* Per-pixel status bits. */
#define FF_ST_CONVERGED_GTOL 1u    /* projected gradient small */
#define FF_ST_CONVERGED_XTOL 2u    /* step below xtol in z */
#define FF_ST_CONVERGED_FTOL 4u    /* predicted reduction below ftol * F */
#define FF_ST_MAX_ITER 8u
#define FF_ST_NONFINITE_INPUT 16u  /* NaN/Inf radiance or model: no solve */
#define FF_ST_DAMPING_OVERFLOW 32u
#define FF_ST_COV_SINGULAR 64u     /* some covariance rows are NaN (unidentified variables) */
#define FF_ST_AT_BOUND 128u        /* some z_j = +-1 at the end */
#define FF_ST_USED_FALLBACK 256u   /* the solve from z0 failed; the result is from the default start x0 */
#define FF_ST_WARM_START 512u      /* a per-pixel start z0 was used (see FF_ST_USED_FALLBACK) */
#define FF_ST_NO_DOF 1024u         /* fewer unmasked bands than n + 1: no solve */
#define FF_ST_BAD_ATMOSPHERE 2048u /* per-pixel atmosphere index out of range: no solve */
#define FF_ST_CONVERGED (FF_ST_CONVERGED_GTOL | FF_ST_CONVERGED_XTOL | FF_ST_CONVERGED_FTOL)

/* Columns of the per-band table of a scene (FP64 copy via
 * ff_scene_band_tables).  Row b holds, for band centre lambda_b (nm):
 *   0 lambda_b, 1 K_b = E_b cos(sza)/pi, 2 tau_dn,b tau_up,b, 3 tau_up,b,
 *   4 rho_atm,b, 5 S_b, 6 L_sat,b (+inf when no saturation level),
 * where E, tau, rho_atm, S are the high-resolution atmosphere resampled with
 * the band's Gaussian spectral response (truncated at +-4 sigma, weights
 * normalised to 1).  The remaining columns are internal. */
#define FF_TABLE_COLS 12

/* Instrument: band centres and FWHM (nm), host arrays [n_bands]. */
typedef struct ff_srf {
    int32_t n_bands;
    const double* wavelength_nm;
    const double* fwhm_nm;
} ff_srf;

/* Atmosphere on a uniform high-resolution grid, host arrays [n_hr]:
 * solar irradiance (W m^-2 nm^-1), transmittances, path reflectance and
 * spherical albedo (eq. solar).  sat_level: per-band saturation radiance
 * [n_bands] (bands with L_obs >= level are masked, eq. loss) or NULL. */
typedef struct ff_atmosphere {
    int32_t n_hr;
    const double* lambda_nm;
    const double* e_solar;
    const double* tau_down;
    const double* tau_up;
    const double* rho_atm;
    const double* s_sph;
    double cos_sza;
    const float* sat_level;
} ff_atmosphere;

/* Box and default start, physical units, first n entries used. */
typedef struct ff_prior {
    int32_t model;
    double lo[FF_MAX_STATE];
    double hi[FF_MAX_STATE];
    double x0[FF_MAX_STATE];
} ff_prior;

typedef struct ff_options {
    int32_t max_iter;      /* LM model evaluations after the first (default 50) */
    int32_t precision;     /* FF_PRECISION_* (default FP32) */
    int32_t n_quad;        /* Gauss-Hermite order: 16, 24 or 32 (default 32); FP64 supports 32 */
    int32_t schedule;      /* FF_SCHEDULE_* (default persistent) */
    int32_t block_size;    /* threads per workgroup: 64, 128, 192 or 256 (0 = default 256) */
    int32_t blocks_per_cu; /* persistent grid: workgroups per CU (0 = occupancy limit) */
    int32_t fallback;      /* with a per-pixel start: re-solve failed pixels from x0 (default 1) */
    int32_t accumulate;    /* FF_ACCUMULATE_* for the FP32 path (default FP32) */
    int32_t lanes_per_pixel; /* lanes that share one pixel's evaluation: 1, 2, 4, 8, 16, 32 or 64
                              (0 = default 1); more lanes shorten each pixel's latency at a
                              small replicated cost (results differ only in summation order) */
    int32_t warm_max_iter; /* iteration cap of a solve from a per-pixel start z0 before the fallback
                              to x0 takes over (0 = max_iter; the fallback always gets max_iter) */
    double xtol;           /* default 1e-6 (z units) */
    double ftol;           /* default 1e-8: an accepted step whose predicted reduction is <= ftol F
                              ends the solve (FF_ST_CONVERGED_FTOL) */
    double gtol;           /* default 1e-10 */
    double kappa;          /* accept a step whose predicted reduction is <= kappa F (default 1e-5) */
    double tau;            /* initial damping = tau * max diag(J^T J) (default 1e-6) */
    double ftol_undetected; /* the decrease test's tolerance while the fire fraction (state
                               variable 0) is below f_detect: no detectable fire, the thermal
                               variables unidentified, the loss a noise valley along the
                               area-temperature degeneracy (default 1e-6, the resolution of F
                               with an FP32 thermal term) */
    double f_detect;       /* default 1e-4 (0 = always ftol) */
} ff_options;

/* Outputs, device arrays owned by the caller (any pointer may be NULL to
 * skip that output):
 *   state [P][n] physical units; cov_packed [P][n(n+1)/2] upper triangle of
 *   the state covariance, row-major; moments [P][2] = E[T], sigma[T];
 *   rrr [P] = ||r|| / ||m L_obs||; iters [P] = model evaluations after the
 *   first; status [P] = FF_ST_* bits; state_f64 [P][n] double copy of state. */
typedef struct ff_outputs {
    float* state;
    float* cov_packed;
    float* moments;
    float* rrr;
    int32_t* iters;
    uint32_t* status;
    double* state_f64;
} ff_outputs;

typedef struct ff_scene ff_scene;

const char* ff_version(void);
const char* ff_status_string(ff_status s);
const char* ff_last_error(void);

/* Defaults of ff_options (see field comments).  Host only. */
void ff_options_default(ff_options* opts);

/* Default box and start of a model: f in [0, 0.5], m in [350, 2200] K (the
 * temperature span of the paper's Sec. 2.2 grid), s in [1, 500] K, eta in
 * [0, 1], smouldering mean in [350, 900] K and flaming mean in
 * [900, 2200] K (the 900 K regime split of Sec. 3.4), rho0 in [-0.2, 1],
 * rho1 in [-5e-4, 5e-4] /nm; start f = 0.01, m = 1000, s = 150, eta = 0.5,
 * m_s = 650, m_h = 1200, rho0 = 0.2, rho1 = 0.  FF_MODEL_GAUSS_GRID_2 takes
 * the two-component box and start with the spreads in [10, 500] K.
 * FF_MODEL_ENDMEMBER_1 takes the one-component f, m, s and fractions in
 * [0, 1] starting at 1/5 each; FF_MODEL_FULL the FF_MODEL_GAUSS_GRID_2
 * thermal box and start with those fractions.  FF_EINVAL for an unknown
 * model. */
ff_status ff_prior_default(int32_t model, ff_prior* prior);

/* Gauss-Hermite rule for weight e^{-x^2}: q nodes and weights (host arrays
 * [q]), q in [1, 64].  Used for the lognormal temperature quadrature of
 * eq. (thermal).  Synchronous, host only. */
ff_status ff_gauss_hermite(int32_t q, double* nodes_host, double* weights_host);

/* Build a scene: resample the atmosphere to the bands with a Gaussian SRF
 * and store the per-band factors of eq. (solar) and the Planck constants on
 * the current device.  Synchronous.  *out owns device memory; free it with
 * ff_scene_destroy.  FF_EINVAL if a band's response window (+-4 sigma)
 * contains no high-resolution sample or any array is NULL. */
ff_status ff_scene_create(const ff_srf* srf, const ff_atmosphere* atm, ff_scene** out);
void ff_scene_destroy(ff_scene* scene);
int32_t ff_scene_n_bands(const ff_scene* scene);

/* Copy the scene's FP64 band table to host memory [n_bands][FF_TABLE_COLS].
 * Synchronous. */
ff_status ff_scene_band_tables(const ff_scene* scene, double* out_host);

/* Surface endmember library of the scene (Keely et al. Sec. 2.4): the
 * FF_N_ENDMEMBERS reflectance spectra reflectance_host [FF_N_ENDMEMBERS][n_hr]
 * on the high-resolution grid lambda_nm [n_hr] are resampled to the bands
 * with the scene's Gaussian spectral responses (the same weights as the
 * atmosphere) and kept on the device for FF_MODEL_ENDMEMBER_1.  Host
 * arrays, read during the call; synchronous.  A second call replaces the
 * library.  FF_EINVAL for NULL arrays, n_hr < 1, non-finite values or a
 * band whose response window holds no sample. */
ff_status ff_scene_set_endmembers(ff_scene* scene, int32_t n_hr, const double* lambda_nm,
                                  const double* reflectance_host);

/* Copy the scene's band-resampled library to host memory
 * [FF_N_ENDMEMBERS][n_bands] (FP64).  FF_EINVAL if none was set.
 * Synchronous. */
ff_status ff_scene_endmembers(const ff_scene* scene, double* out_host);

/* Forward model of eq. (fm) at P states.  state_dev: [P][n] physical units,
 * float (FF_PRECISION_FP32) or double (FF_PRECISION_FP64).  radiance_dev:
 * [P][n_bands] of the same type.  jac_dev: [P][n_bands][n] dL/dx of the same
 * type, or NULL.  Asynchronous on stream. */
ff_status ff_forward(const ff_scene* scene, int32_t model, int32_t precision, int32_t n_quad,
                     const void* state_dev, int64_t P, void* radiance_dev, void* jac_dev,
                     void* stream);

/* Retrieve P pixels of one scene.  radiance_dev: [P][n_bands] float32,
 * row-major (band-interleaved by pixel).  z0_dev: [P][n] per-pixel start in
 * z (for example from a learned warm start) or NULL to start every pixel
 * from prior->x0; a row whose first entry is NaN carries no start (that
 * pixel is solved from x0 exactly as without z0: no fallback, no
 * FF_ST_WARM_START), so a warm start can be given to some pixels only.
 * With z0_dev and opts->fallback, pixels whose solve from z0 does not
 * converge are solved again from x0 (FF_ST_USED_FALLBACK).
 * evals_dev: optional uint64 counter that receives += the number of model
 * evaluations performed (NULL to skip).  Asynchronous on stream.  The
 * queue counter and launch descriptor live in a library-owned scratch
 * buffer per (device, stream), allocated on the first call on that stream
 * (which synchronizes it) and reused by later calls, so calls ordered on one
 * stream allocate nothing; calls on one stream must be ordered (they share
 * that buffer).  See ff_release_scratch. */
ff_status ff_retrieve_scene(const ff_scene* scene, const float* radiance_dev, int64_t P,
                            const ff_prior* prior, const float* z0_dev, const ff_options* opts,
                            const ff_outputs* out, unsigned long long* evals_dev, void* stream);

/* Ragged batch: n_scenes scenes (same band count) in one launch sequence;
 * per-scene radiance, start and outputs.  z0_dev may be NULL, or an array
 * of n_scenes pointers (each may be NULL). */
ff_status ff_retrieve_batch(const ff_scene* const* scenes, const float* const* radiance_dev,
                            const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                            const float* const* z0_dev, const ff_options* opts,
                            const ff_outputs* outs, unsigned long long* evals_dev, void* stream);

/* Allocation-free form of ff_retrieve_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels,
 * launch shape and results as ff_retrieve_batch; the queue counters and
 * launch descriptors live in a fixed 16 KiB device array of the library
 * (one copy per device, held until the process ends) instead of the
 * stream's scratch buffer, and the call allocates nothing (the first call
 * on a device for a precision / model / quadrature order copies that
 * quadrature rule into constant memory, synchronously, without
 * allocating).  At most FF_NOALLOC_MAX_SCENES scenes per call (FF_EINVAL
 * beyond).  Every call on one device shares that array and clears its
 * counters first: calls that overlap on one device, on any streams, race
 * and must be ordered by the caller. */
#define FF_NOALLOC_MAX_SCENES 64
ff_status ff_retrieve_batch_noalloc(const ff_scene* const* scenes, const float* const* radiance_dev,
                                    const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                    const float* const* z0_dev, const ff_options* opts,
                                    const ff_outputs* outs, unsigned long long* evals_dev, void* stream);

/* Launch-shape autotuner.  Times ff_retrieve_batch on the given batch
 * (writing its results to outs) for candidate lanes_per_pixel (1..64),
 * block_size (64, 128, 256), blocks_per_cu (occupancy limit or 1) and
 * schedule, one dimension at a time starting from *opts, and writes the
 * fastest into *opts (other fields untouched; n_quad is never changed, since
 * it changes the model).  cache_path: JSON table of earlier choices keyed by
 * device architecture, band count, model, precision, accumulation, n_quad,
 * start kind (z0 given or not) and floor(log2(total pixels)); a hit is
 * applied without timing, a new choice is stored (NULL: no table).
 * flags: FF_TUNE_IGNORE_CACHE re-tunes and overwrites the entry.  best_ms
 * (may be NULL) receives the chosen configuration's time.  Synchronous
 * (waits on stream between candidates). */
#define FF_TUNE_IGNORE_CACHE 1
ff_status ff_tune(const ff_scene* const* scenes, const float* const* radiance_dev, const int64_t* P,
                  int32_t n_scenes, const ff_prior* prior, const float* const* z0_dev, ff_options* opts,
                  const ff_outputs* outs, const char* cache_path, int32_t flags, double* best_ms,
                  void* stream);

/* Quadrature-order choice, the tuner's third dimension (FP32 path of the
 * lognormal models FF_MODEL_LOGNORMAL_1/2 and FF_MODEL_ENDMEMBER_1, whose
 * thermal integral the order only approximates; the grid models' order is
 * their temperature grid and is never changed).  The batch is retrieved at
 * the requested order opts->n_quad into outs_ref and at each lower order of
 * {16, 24} into outs_trial, each at its own launch shape from ff_tune (with
 * cache_path and flags as there).  A lower order is accepted when, on the
 * pixels both runs converge on, at least 99 % agree with the requested
 * order: relative radiance residuals within 1e-5, f within 1e-4, and E[T]
 * within max(0.5 K, 2 % of its posterior s.d. from the requested order's
 * covariance) where both fits have f >= 1e-4; and the converged counts
 * differ by at most 0.5 %.  The fastest accepted order (the requested one if
 * none) and its launch shape are written to opts; report_host[8], if not
 * NULL, receives {chosen order, its time ms, requested order's time ms, the
 * agreeing share of the chosen order (1 for the requested), then share and
 * time ms at order 24 and at order 16 (NaN where not tested; a share of -1
 * means the converged counts differed by more than 0.5 %)}.  Synchronous
 * (copies the per-pixel outputs to the host for the comparison).
 * FF_EUNSUPPORTED for FP64 or a grid model (opts unchanged). */
ff_status ff_tune_quadrature(const ff_scene* const* scenes, const float* const* radiance_dev, const int64_t* P,
                             int32_t n_scenes, const ff_prior* prior, const float* const* z0_dev,
                             ff_options* opts, const ff_outputs* outs_ref, const ff_outputs* outs_trial,
                             const char* cache_path, int32_t flags, double* report_host, void* stream);

/* One-shot form: builds a scene from srf/atm, retrieves, destroys the scene.
 * Synchronous (waits for stream). */
ff_status ff_retrieve(const float* radiance_dev, int64_t P, const ff_srf* srf,
                      const ff_atmosphere* atm, const ff_prior* prior, const float* z0_dev,
                      const ff_options* opts, const ff_outputs* out, void* stream);

/* Per-pixel atmosphere (Keely et al. Sec. 2.3: the atmosphere is cached for
 * the scene on a grid of quantised column water vapour and each pixel takes
 * the entry of its pre-solved water vapour).  atmospheres: n_atm scenes
 * (1 <= n_atm <= FF_MAX_ATMOSPHERES, the same band count), one per quantised
 * atmosphere; atm_index_dev: [P] int32, pixel p is solved with
 * atmospheres[atm_index_dev[p]]; a pixel whose index is outside [0, n_atm)
 * is not solved (NaN outputs, FF_ST_BAD_ATMOSPHERE).  Otherwise as
 * ff_retrieve_scene (radiance [P][n_bands], optional z0, outputs [P]).
 * Asynchronous on stream. */
#define FF_MAX_ATMOSPHERES 16
ff_status ff_retrieve_atm_indexed(const ff_scene* const* atmospheres, int32_t n_atm, const int32_t* atm_index_dev,
                                  const float* radiance_dev, int64_t P, const ff_prior* prior, const float* z0_dev,
                                  const ff_options* opts, const ff_outputs* out, unsigned long long* evals_dev,
                                  void* stream);

/* ------------------------------------------------------------------------
 * Fire-candidate pre-filter (Keely et al. Sec. 2.1).  Per pixel
 *   HFDI = (L(2430 nm) - L(2061 nm)) / (L(2430 nm) + L(2061 nm)),
 * L(lambda) the radiance of the band whose centre is nearest lambda (the
 * lower band index on a tie), in IEEE float32 arithmetic.  A pixel is a
 * candidate when (double)HFDI >= threshold (the paper uses -0.1) or either
 * of the two bands is saturated (L >= the scene's saturation level: the
 * paper keeps such pixels, saturation there being itself a sign of hot
 * emission).  A NaN index (zero sum of zeros, non-finite radiance) is not a
 * candidate unless a band is saturated.
 *   radiance_dev: [P][n_bands] float32; hfdi_dev: [P] float32 index values
 *   or NULL; index_dev: [P] int64, receives the candidates' pixel numbers
 *   in increasing order in its first *count_dev entries; count_dev: one
 *   int64 in device memory, receives the number of candidates.
 * Asynchronous on stream; the count stays on the device (pass it to
 * ff_retrieve_listed without reading it back).  Per-tile counters and the
 * candidate flags (one bit per pixel, kept between the counting and the
 * writing pass) live in the stream's scratch buffer (see
 * ff_retrieve_scene).  FF_EINVAL for NULL
 * arguments, P < 0 or a NaN threshold. */
ff_status ff_hfdi_candidates(const ff_scene* scene, const float* radiance_dev, int64_t P, double threshold,
                             float* hfdi_dev, int64_t* index_dev, int64_t* count_dev, void* stream);

/* Retrieve the listed pixels of one scene: items 0 .. min(*count_dev, P) - 1
 * of index_dev name radiance rows (entries outside [0, P) are skipped); each
 * listed row is solved as by ff_retrieve_scene and its outputs (and its z0
 * row, if z0_dev is given) use the row's own position in the [P]-sized
 * arrays; rows not listed are left untouched.  index_dev and count_dev are
 * device memory, for example from ff_hfdi_candidates; the count is read by
 * the kernel, so nothing waits on the host.  Asynchronous on stream. */
ff_status ff_retrieve_listed(const ff_scene* scene, const float* radiance_dev, int64_t P,
                             const int64_t* index_dev, const int64_t* count_dev, const ff_prior* prior,
                             const float* z0_dev, const ff_options* opts, const ff_outputs* out,
                             unsigned long long* evals_dev, void* stream);

/* ------------------------------------------------------------------------
 * Resolution rescaling (Keely et al.: fine radiance aggregated to a coarse
 * grid in radiance space, both retrieved, and the coarse pixels' Gaussian
 * posteriors compared with the fine retrievals in their footprints by a
 * Quantile Error Curve).  Pixels are row-major images of rows x cols.
 *
 * ff_block_mean: out[(r C + c)][b] = mean of radiance over the block x block
 * fine pixels of coarse pixel (r, c), R = rows / block, C = cols / block
 * (partial blocks at the right and bottom edges are dropped); summed in
 * FP64, rounded once to float32.  block in [1, 32].  Asynchronous. */
ff_status ff_block_mean(const float* radiance_dev, int32_t rows, int32_t cols, int32_t n_bands, int32_t block,
                        float* out_dev, void* stream);

/* ff_qec: per coarse pixel k, QEC_j = Q_coarse(q_j) - Q_fine(q_j) with
 * Q_coarse the quantile of N(E[T]_k, sigma[T]_k) and Q_fine of the fine
 * pixels in k's footprint that take part: qec_emp uses their empirical
 * distribution of E[T] (linear interpolation between order statistics,
 * h = (n - 1) q), qec_mix the equal-weight mixture of their N(E[T], sigma[T])
 * (quantile by bisection to ~1e-9 relative).  A pixel takes part when its
 * status has a convergence bit, its f = state[0] >= f_min and its sigma[T]
 * is finite and positive; a coarse pixel is evaluated when it takes part
 * itself and at least min_fine of its fine pixels do, else its QEC entries
 * are NaN.  fine_mask_dev [rows cols] / coarse_mask_dev [R C] (uint8, may
 * be NULL) restrict the pixels that take part to those with a nonzero entry
 * (for example the fire candidates).  Inputs are the outputs of a retrieval
 * (moments [.][2], state [.][n_state], status); levels_host: n_levels values
 * in (0, 1), n_levels <= 16; outputs [R C][n_levels] float32 and n_used
 * [R C] (fine pixels taking part).  Asynchronous. */
ff_status ff_qec(const float* fine_moments_dev, const float* fine_state_dev, const uint32_t* fine_status_dev,
                 const uint8_t* fine_mask_dev, const float* coarse_moments_dev, const float* coarse_state_dev,
                 const uint32_t* coarse_status_dev, const uint8_t* coarse_mask_dev,
                 int32_t n_state, int32_t rows, int32_t cols, int32_t block, double f_min, int32_t min_fine,
                 int32_t n_levels, const double* levels_host, float* qec_emp_dev, float* qec_mix_dev,
                 int32_t* n_used_dev, void* stream);

/* ------------------------------------------------------------------------
 * The paper's own solver: staged Adam (Keely et al. Sec. 2.5, eq. adam;
 * Kingma & Ba 2015) on the windowed loss of eq. (loss) in the z coordinate of
 * eq. (affine).  Each stage runs a fresh optimiser (t = 1, m = v = 0) for a
 * fixed number of steps on its free variables; the others are held.  Step t:
 *   g   = gradient of the loss in z, where variable j's component sums over
 *         the unsaturated bands with window_lo_nm[j] <= lambda <= window_hi_nm[j]
 *         (g_j = -2 sum_b r_b dL_b/dz_j, r = L_obs - L);
 *   g  *= clip_norm / ||g||  when ||g|| > clip_norm > 0 (norm over free j);
 *   m   = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2;
 *   z_j = clip(z_j - lr (m_j / (1 - beta1^t)) / (sqrt(v_j / (1 - beta2^t)) + eps), -1, 1);
 * for the endmember models the surface fractions are then projected onto the
 * unit simplex (Sec. 2.5), also after the stage's start values are set.
 * Every pixel takes the same number of steps (no convergence test). */
#define FF_MAX_ADAM_STAGES 4

typedef struct ff_adam_stage {
    int32_t steps;                     /* Adam steps of this stage (>= 0) */
    uint32_t free_mask;                /* bit j set: state variable j is updated */
    double lr;                         /* learning rate in z (> 0) */
    double clip_norm;                  /* maximum global gradient norm; <= 0: no clip */
    double window_lo_nm[FF_MAX_STATE]; /* band window of each free variable's gradient */
    double window_hi_nm[FF_MAX_STATE];
    double z_start[FF_MAX_STATE];      /* NaN: carried over; else z_j is set to it
                                          (clipped to [-1, 1]) when the stage starts */
} ff_adam_stage;

typedef struct ff_adam_options {
    int32_t n_stages;        /* 0 .. FF_MAX_ADAM_STAGES */
    int32_t precision;       /* FF_PRECISION_* (default FP32) */
    int32_t accumulate;      /* FF_ACCUMULATE_* for the FP32 path (default FP32) */
    int32_t n_quad;          /* Gauss-Hermite order: 16, 24, 32 (default 32); FP64: 32 */
    int32_t block_size;      /* 64, 128, 192 or 256 (0 = 256) */
    int32_t lanes_per_pixel; /* power of two <= 64 (0 = 1) */
    double beta1, beta2, eps;          /* eq. (adam) defaults 0.9, 0.999, 1e-8 */
    ff_adam_stage stage[FF_MAX_ADAM_STAGES];
} ff_adam_options;

/* The paper's two stages for prior->model, start values taken from prior.
 * Stage 1: 30 steps, lr 0.03, window [350, 2500] nm, frees f, one
 * temperature and the reflectance (rho0, rho1) with the temperature spread
 * at its lower bound -- the single temperature of the first stage (two-
 * component model: the flaming mean, with eta at 1).  Stage 2: 100 steps,
 * lr 0.015, holds the reflectance and frees f and the temperature
 * distribution, spreads (and eta) restarting from x0; windows [900, 1800] nm
 * for the flaming component, [1500, 2500] nm for the smouldering one and
 * their union [900, 2500] nm for f, eta and the one-component model's
 * variables.  clip_norm 1.0 (the paper's value is not legible).  FF_EINVAL
 * for a NULL argument or an invalid prior.  Host only. */
ff_status ff_adam_options_default(const ff_prior* prior, ff_adam_options* opts);

/* Staged-Adam retrieval of a ragged batch (arguments as ff_retrieve_batch,
 * options from ff_adam_options).  Start: z0_dev[s] per pixel, or prior->x0.
 * Outputs as ff_retrieve_batch at the final z over all unsaturated bands;
 * iters = Adam steps taken; status carries FF_ST_NONFINITE_INPUT (radiance
 * or a gradient not finite), FF_ST_NO_DOF, FF_ST_AT_BOUND, FF_ST_COV_SINGULAR
 * and FF_ST_WARM_START, never a convergence bit.  evals_dev receives += the
 * model evaluations (steps + 1 per solved pixel).  Asynchronous on stream;
 * the per-stream scratch of ff_retrieve_batch holds the launch descriptor
 * and the per-stage band lists. */
ff_status ff_adam_retrieve_batch(const ff_scene* const* scenes, const float* const* radiance_dev,
                                 const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                 const float* const* z0_dev, const ff_adam_options* opts,
                                 const ff_outputs* outs, unsigned long long* evals_dev,
                                 void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start.  A multilayer perceptron maps a radiance spectrum to a
 * starting state z0 for the LM solve (which always refines it and falls
 * back to the default start when the solve from z0 fails).  Layers:
 * n_in -> h1 -> h2 -> h3 -> n_out, GELU (tanh form, Hendrycks & Gimpel 2016)
 * after each hidden layer and tanh on the output, so z0 lies in (-1, 1).
 * Input features: u_b = (ln max(L_b, floor) - mean_b) * inv_std_b.
 * Weights: FP32 master copy; BF16 copies feed the matrix-core (MFMA) GEMMs,
 * which accumulate in FP32.  Training: mean squared error in z, Adam
 * (Kingma & Ba; the paper's Sec. 2.5 update with beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8).
 * Parameter vector layout (ff_mlp_get_params / ff_mlp_set_params):
 *   W1 [h1][n_in], b1 [h1], W2 [h2][h1], b2 [h2], W3 [h3][h2], b3 [h3],
 *   W4 [n_out][h3], b4 [n_out]   (row-major, out x in).
 * ------------------------------------------------------------------------ */
typedef struct ff_mlp ff_mlp;

/* Create a network on the current device with weights drawn from a seeded
 * counter-based generator (He-normal for hidden layers, zero biases) and
 * identity normalisation.  n_in <= 1024, hidden sizes multiples of 64 and
 * <= 1024, n_out <= 16.  Synchronous. */
ff_status ff_mlp_create(int32_t n_in, int32_t h1, int32_t h2, int32_t h3, int32_t n_out,
                        uint64_t seed, ff_mlp** out);
void ff_mlp_destroy(ff_mlp* mlp);
int64_t ff_mlp_n_params(const ff_mlp* mlp);

/* Copy the FP32 parameter vector to/from host memory [ff_mlp_n_params]
 * (set also refreshes the BF16 copies and clears the Adam state).
 * Synchronous. */
ff_status ff_mlp_get_params(const ff_mlp* mlp, float* params_host);
ff_status ff_mlp_set_params(ff_mlp* mlp, const float* params_host);

/* Feature normalisation: host arrays [n_in] and the radiance floor.
 * Synchronous. */
ff_status ff_mlp_set_normalization(ff_mlp* mlp, const float* mean_host, const float* inv_std_host,
                                   float floor);
ff_status ff_mlp_get_normalization(const ff_mlp* mlp, float* mean_host, float* inv_std_host, float* floor);

/* Set the normalisation from P spectra radiance_dev [P][n_in] (per-band
 * mean and 1/s.d. of ln max(L, floor)).  Asynchronous on stream. */
ff_status ff_mlp_fit_normalization(ff_mlp* mlp, const float* radiance_dev, int64_t P, float floor,
                                   void* stream);

/* Warm start: z0_dev [P][n_out] = network(radiance_dev [P][n_in]).
 * Asynchronous on stream; internal activations are processed in chunks in
 * the network's one workspace (the handle is const but the workspace is
 * not): calls with one network must be ordered on one stream. */
ff_status ff_mlp_infer(const ff_mlp* mlp, const float* radiance_dev, int64_t P, float* z0_dev,
                       void* stream);

/* Warm start for listed rows (the front end's candidates, Sec. 2.1, in
 * front of the network of Sec. 2.5): for items i < n_listed of index_dev,
 * z0_dev row index_dev[i] = network(radiance_dev row index_dev[i]), the
 * same values ff_mlp_infer gives that row.  radiance_dev [P][n_in];
 * index_dev: n_listed int64 pixel numbers in device memory (for example the
 * first count entries from ff_hfdi_candidates; the caller reads that count
 * back); entries outside [0, P) are skipped; z0_dev [P][n_out], rows not
 * listed are left untouched.  Asynchronous on stream.  FF_EINVAL for NULL
 * buffers or negative sizes. */
ff_status ff_mlp_infer_listed(const ff_mlp* mlp, const float* radiance_dev, int64_t P, const int64_t* index_dev,
                              int64_t n_listed, float* z0_dev, void* stream);

/* Loss and gradient of one batch: loss_dev[0] = mean over the batch and
 * outputs of (z - target)^2, grads_dev [ff_mlp_n_params] (either may be
 * NULL).  target_dev [P][n_out].  P <= 65536.  Asynchronous on stream. */
ff_status ff_mlp_gradients(ff_mlp* mlp, const float* radiance_dev, const float* target_dev, int64_t P,
                           double* loss_dev, float* grads_dev, void* stream);

/* One Adam step on one batch (gradients as above, then the update with
 * learning rate lr).  loss_dev may be NULL.  Asynchronous on stream. */
ff_status ff_mlp_train_step(ff_mlp* mlp, const float* radiance_dev, const float* target_dev, int64_t P,
                            float lr, double* loss_dev, void* stream);

/* Training data: P spectra of the one-component model for the scene, with
 * states drawn from a Philox4x32-10 counter generator keyed by seed
 * (sample g = offset + p): f ~ logU[1e-4, 0.3], m ~ U[600, 1400] K,
 * s ~ U[50, 300] K, rho0 ~ U[0.05, 0.4], rho1 ~ U[-1e-4, 1e-4] /nm; a
 * fraction bg_fraction of samples has f = 0 (background, target m, s = x0).
 * Noise sigma = L / snr (snr <= 0: none) from Box-Muller pairs.  Writes
 * radiance_dev [P][n_bands], target_z_dev [P][5] (z of the state in prior's
 * box, clipped to [-1, 1]) and optionally state_dev [P][5] (physical).
 * Asynchronous on stream. */
ff_status ff_mlp_generate(const ff_scene* scene, const ff_prior* prior, uint64_t seed, uint64_t offset,
                          int64_t P, double snr, double bg_fraction, float* radiance_dev,
                          float* target_z_dev, float* state_dev, void* stream);

/* Train for `steps` Adam steps of `batch` fresh generated spectra each
 * (sample offset advances by batch per step); the learning rate decays by
 * cosine from lr to lr_final.  loss_history_dev [steps] or NULL.
 * Asynchronous on stream. */
ff_status ff_mlp_train(ff_mlp* mlp, const ff_scene* scene, const ff_prior* prior, int64_t steps,
                       int32_t batch, uint64_t seed, double snr, double bg_fraction, float lr,
                       float lr_final, double* loss_history_dev, void* stream);

/* Steps first_step .. first_step + n_steps - 1 of the same schedule of
 * total_steps steps (ff_mlp_train is the span 0 .. steps - 1): step i
 * trains on the samples offset i * batch of the seed's counter-based
 * stream (Philox4x32-10) at the cosine learning rate of step i, so a run
 * split into spans -- across a checkpoint written by ff_warmstart_save and
 * read by ff_warmstart_load -- takes exactly the uninterrupted run's
 * steps.  loss_history_dev [n_steps] or NULL.  Asynchronous on stream.
 * FF_EINVAL unless 0 <= first_step <= first_step + n_steps <= total_steps. */
ff_status ff_mlp_train_span(ff_mlp* mlp, const ff_scene* scene, const ff_prior* prior, int64_t total_steps,
                            int64_t first_step, int64_t n_steps, int32_t batch, uint64_t seed, double snr,
                            double bg_fraction, float lr, float lr_final, double* loss_history_dev,
                            void* stream);

/* Schedule steps the network has taken in ff_mlp_train / ff_mlp_train_span
 * (restored by ff_warmstart_load): the first_step of a resumed span. */
int64_t ff_mlp_steps_done(const ff_mlp* mlp);

/* The layer sizes (n_in, h1, h2, h3, n_out) into sizes_host[5]. */
ff_status ff_mlp_sizes(const ff_mlp* mlp, int32_t* sizes_host);

/* Checkpoints of a warm-start network (the learned start of the LM,
 * trained by the update of Sec. 2.5 eq. adam): ff_warmstart_save writes the
 * layer sizes, the FP32 master weights, the normalisation, the Adam first
 * and second moments, the Adam step count and the schedule steps taken to
 * path (a host file; synchronizes the network's device first);
 * ff_warmstart_load creates a network on the current device from such a
 * file (caller destroys it with ff_mlp_destroy).  A run resumed from a
 * checkpoint with ff_mlp_train_span continues bitwise as the uninterrupted
 * run.  FF_EINVAL for a missing, foreign, truncated or inconsistent file. */
ff_status ff_warmstart_save(const ff_mlp* mlp, const char* path);
ff_status ff_warmstart_load(const char* path, ff_mlp** out);

/* ------------------------------------------------------------------------
 * Graph-captured pipeline.  The launch sequence of one batch shape --
 * network inference of z0 for every scene that has a network (mlps: NULL,
 * or n_scenes entries, each NULL for the default start), then the retrieval
 * with fallback -- recorded once into a HIP graph and replayed by one graph
 * launch.  The graph binds every pointer given here (radiance,
 * outputs, evals counter, scene tables, network weights): rewrite the
 * radiance buffers in place between launches; results land in outs.  z0
 * lives in a buffer the pipeline owns (ff_pipeline_z0).
 * Create waits for stream, runs the sequence once eagerly (results
 * written, evals incremented) so that every workspace reaches its size
 * outside capture, then records it (thread-local capture) on a stream the
 * pipeline owns -- so its scratch is never shared or regrown -- and
 * instantiates the graph.  Synchronous.  The network's workspace stays
 * valid for the graph while the pipeline exists (a larger eager use keeps
 * the old buffers alive instead of freeing them); destroy pipelines before
 * their networks.  Launch: asynchronous on stream (may be NULL).  Replays of
 * one pipeline must not overlap each other or run concurrently with other
 * uses of the same network (they share buffers).
 * ------------------------------------------------------------------------ */
typedef struct ff_pipeline ff_pipeline;
ff_status ff_pipeline_create(const ff_scene* const* scenes, const float* const* radiance_dev,
                             const int64_t* P, int32_t n_scenes, const ff_prior* prior, const ff_mlp* const* mlps,
                             const ff_options* opts, const ff_outputs* outs, unsigned long long* evals_dev,
                             void* stream, ff_pipeline** out);
/* The same with the warm start routed by the front end (Keely et al.
 * Sec. 2.1): for each scene with a network the graph runs ff_hfdi_candidates
 * at hfdi_threshold (the paper: -0.1) into buffers the pipeline owns, marks
 * every z0 row "no start" (first entry NaN), and runs the network on the
 * candidates only, their count read on the device (inference is launched
 * for all P rows, chunks past the count doing nothing); the retrieval then
 * solves candidates from the network's start and every other pixel from x0
 * (ff_options: rows without a start).  The outputs equal those of
 * ff_hfdi_candidates + ff_mlp_infer_listed + ff_retrieve_batch run eagerly
 * on the same inputs.  FF_EINVAL for a NaN threshold, else as above. */
ff_status ff_pipeline_create_routed(const ff_scene* const* scenes, const float* const* radiance_dev,
                                    const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                    const ff_mlp* const* mlps, double hfdi_threshold, const ff_options* opts,
                                    const ff_outputs* outs, unsigned long long* evals_dev, void* stream,
                                    ff_pipeline** out);
ff_status ff_pipeline_launch(ff_pipeline* pipeline, void* stream);
const float* ff_pipeline_z0(const ff_pipeline* pipeline);   /* [sum P][n], scene after scene */
void ff_pipeline_destroy(ff_pipeline* pipeline);

/* Vector-ALU calibration of the current device: sustained lane-operations
 * per second, in rates_host[0..5], of a 32-bit FMA, the 32-bit base-2
 * exponential, the 32-bit reciprocal, a 64-bit FMA, a float <-> double
 * conversion, and one quadrature node of the Planck sums (x = a u,
 * 1/(2^x - 1), three accumulations: 7 VALU + 2 transcendentals), each over
 * eight independent chains per lane on a grid that fills every SIMD.  They
 * weigh the instructions of the retrieval's issue-slot roofline.
 * Synchronous (allocates and frees two small buffers); n_rates >= 6. */
ff_status ff_valu_rates(double* rates_host, int32_t n_rates, void* stream);

/* Retrieval launches use a library-owned scratch buffer per (device,
 * stream) that only grows (so that repeated calls allocate nothing and can
 * be captured); this frees them all after synchronizing each device that
 * holds one, except the buffers of live pipelines' private streams (their
 * graphs bind them; ff_pipeline_destroy frees them).  Call only when no library work is in flight.  Destroy a
 * stream only after its retrieval work has completed: a new stream that
 * receives the same handle reuses the buffer. */
ff_status ff_release_scratch(void);

#ifdef __cplusplus
}
#endif
#endif /* FIREFIT_H */
