// C-ABI entry points of firefit: argument validation, defaults, errors.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "ff_internal.hpp"

namespace ff {

static thread_local std::string g_last_error;

ff_status set_error(ff_status code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

ff_status clear_error()
{
    g_last_error.clear();
    return FF_OK;
}

ff_status hip_error(hipError_t e, const char* what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return FF_ENOMEM;
    return FF_EDEVICE;
}

int n_state(int model)
{
    switch (model) {
    case FF_MODEL_LOGNORMAL_1: return 5;
    case FF_MODEL_LOGNORMAL_2: return 8;
    case FF_MODEL_GAUSS_GRID_2: return 8;
    case FF_MODEL_ENDMEMBER_1: return 8;
    case FF_MODEL_FULL: return 11;
    default: return -1;
    }
}

static ff_status check_prior(const ff_prior* prior)
{
    if (!prior) return set_error(FF_EINVAL, "prior is NULL");
    const int n = n_state(prior->model);
    if (n < 0) return set_error(FF_EINVAL, "unknown model");
    for (int j = 0; j < n; ++j) {
        if (!std::isfinite(prior->lo[j]) || !std::isfinite(prior->hi[j]) || !(prior->hi[j] > prior->lo[j]))
            return set_error(FF_EINVAL, "prior box needs finite lo < hi for every state variable");
        if (!std::isfinite(prior->x0[j])) return set_error(FF_EINVAL, "prior x0 is not finite");
    }
    // the temperature means and spreads must stay positive over the whole box
    const int pos[5][4] = {{1, 2, -1, -1}, {2, 3, 4, 5}, {2, 3, 4, 5}, {1, 2, -1, -1}, {2, 3, 4, 5}};
    for (int k = 0; k < 4; ++k) {
        const int j = pos[prior->model - 1][k];
        if (j >= 0 && !(prior->lo[j] > 0.0))
            return set_error(FF_EINVAL, "temperature mean and spread bounds must be positive");
    }
    // the simplex step works on x = (z + 1)/2: surface fractions need the box [0, 1]
    const int sf = prior->model == FF_MODEL_ENDMEMBER_1 ? 3 : (prior->model == FF_MODEL_FULL ? 6 : -1);
    if (sf >= 0)
        for (int j = sf; j < sf + FF_N_ENDMEMBERS; ++j)
            if (prior->lo[j] != 0.0 || prior->hi[j] != 1.0)
                return set_error(FF_EINVAL, "surface fractions need the box [0, 1]");
    return FF_OK;
}

// The endmember model reads the scene's library.
static ff_status check_library(int model, const ff_scene* sc, const char* who)
{
    if ((model == FF_MODEL_ENDMEMBER_1 || model == FF_MODEL_FULL) && sc && !sc->has_endmembers)
        return set_error(FF_EINVAL, (std::string(who) + ": the endmember model needs ff_scene_set_endmembers").c_str());
    return FF_OK;
}

static ff_status check_options(const ff_options* o)
{
    if (!o) return set_error(FF_EINVAL, "options is NULL");
    if (o->max_iter < 0 || o->max_iter > 100000) return set_error(FF_EINVAL, "max_iter out of range");
    if (o->warm_max_iter < 0 || o->warm_max_iter > 100000) return set_error(FF_EINVAL, "warm_max_iter out of range");
    if (o->precision != FF_PRECISION_FP32 && o->precision != FF_PRECISION_FP64)
        return set_error(FF_EINVAL, "unknown precision");
    if (o->schedule != FF_SCHEDULE_PERSISTENT && o->schedule != FF_SCHEDULE_STATIC)
        return set_error(FF_EINVAL, "unknown schedule");
    if (o->block_size != 0 && (o->block_size < 64 || o->block_size > 256 || o->block_size % 64 != 0))
        return set_error(FF_EINVAL, "block_size must be 64, 128, 192 or 256");
    if (o->blocks_per_cu < 0) return set_error(FF_EINVAL, "blocks_per_cu < 0");
    if (o->lanes_per_pixel < 0 || o->lanes_per_pixel > 64 || (o->lanes_per_pixel & (o->lanes_per_pixel - 1)) != 0)
        return set_error(FF_EINVAL, "lanes_per_pixel must be 0 or a power of two <= 64");
    if (o->accumulate != FF_ACCUMULATE_FP32 && o->accumulate != FF_ACCUMULATE_FP64)
        return set_error(FF_EINVAL, "unknown accumulate mode");
    if (!(o->xtol >= 0) || !(o->ftol >= 0) || !(o->gtol >= 0) || !(o->kappa >= 0) || !(o->tau > 0) ||
        !(o->ftol_undetected >= 0) || !(o->f_detect >= 0))
        return set_error(FF_EINVAL, "tolerances must be >= 0 and tau > 0");
    return FF_OK;
}

static ff_status check_adam_options(const ff_adam_options* o, int n)
{
    if (!o) return set_error(FF_EINVAL, "adam options is NULL");
    if (o->n_stages < 0 || o->n_stages > FF_MAX_ADAM_STAGES) return set_error(FF_EINVAL, "n_stages out of range");
    if (o->precision != FF_PRECISION_FP32 && o->precision != FF_PRECISION_FP64)
        return set_error(FF_EINVAL, "unknown precision");
    if (o->accumulate != FF_ACCUMULATE_FP32 && o->accumulate != FF_ACCUMULATE_FP64)
        return set_error(FF_EINVAL, "unknown accumulate mode");
    if (o->block_size != 0 && (o->block_size < 64 || o->block_size > 256 || o->block_size % 64 != 0))
        return set_error(FF_EINVAL, "block_size must be 64, 128, 192 or 256");
    if (o->lanes_per_pixel < 0 || o->lanes_per_pixel > 64 || (o->lanes_per_pixel & (o->lanes_per_pixel - 1)) != 0)
        return set_error(FF_EINVAL, "lanes_per_pixel must be 0 or a power of two <= 64");
    if (!(o->beta1 >= 0.0 && o->beta1 < 1.0) || !(o->beta2 >= 0.0 && o->beta2 < 1.0) ||
        !(o->eps > 0.0) || !std::isfinite(o->eps))
        return set_error(FF_EINVAL, "Adam needs 0 <= beta1, beta2 < 1 and a finite eps > 0");
    for (int k = 0; k < o->n_stages; ++k) {
        const ff_adam_stage& s = o->stage[k];
        if (s.steps < 0 || s.steps > 100000) return set_error(FF_EINVAL, "stage steps out of range");
        if (!(s.lr > 0.0) || !std::isfinite(s.lr)) return set_error(FF_EINVAL, "stage lr must be finite and > 0");
        if (std::isnan(s.clip_norm) || std::isinf(s.clip_norm)) return set_error(FF_EINVAL, "stage clip_norm must be finite");
        if (s.free_mask >> n) return set_error(FF_EINVAL, "stage free_mask names a variable the model does not have");
        for (int j = 0; j < n; ++j) {
            if (((s.free_mask >> j) & 1u) &&
                (!std::isfinite(s.window_lo_nm[j]) || !std::isfinite(s.window_hi_nm[j]) ||
                 !(s.window_lo_nm[j] <= s.window_hi_nm[j])))
                return set_error(FF_EINVAL, "a free variable needs a finite window with lo <= hi");
            if (std::isinf(s.z_start[j])) return set_error(FF_EINVAL, "stage z_start must be NaN or finite");
        }
    }
    return FF_OK;
}

}  // namespace ff

using namespace ff;

extern "C" const char* ff_version(void) { return "firefit 0.1 (gfx950)"; }

extern "C" const char* ff_status_string(ff_status s)
{
    switch (s) {
    case FF_OK: return "ok";
    case FF_EINVAL: return "invalid argument";
    case FF_EDEVICE: return "device error";
    case FF_ENOMEM: return "out of memory";
    case FF_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

extern "C" const char* ff_last_error(void) { return g_last_error.c_str(); }

extern "C" void ff_options_default(ff_options* o)
{
    if (!o) return;
    o->max_iter = 50;
    o->precision = FF_PRECISION_FP32;
    o->n_quad = 32;
    o->schedule = FF_SCHEDULE_PERSISTENT;
    o->block_size = 256;
    o->blocks_per_cu = 0;
    o->lanes_per_pixel = 1;
    o->warm_max_iter = 0;
    o->fallback = 1;
    o->accumulate = FF_ACCUMULATE_FP32;
    o->xtol = 1e-6;
    o->ftol = 1e-8;
    o->gtol = 1e-10;
    o->kappa = 1e-5;
    o->tau = 1e-6;
    o->ftol_undetected = 1e-6;
    o->f_detect = 1e-4;
}

extern "C" ff_status ff_prior_default(int32_t model, ff_prior* p)
{
    if (!p) return set_error(FF_EINVAL, "ff_prior_default: NULL prior");
    for (int j = 0; j < FF_MAX_STATE; ++j) { p->lo[j] = 0.0; p->hi[j] = 1.0; p->x0[j] = 0.5; }
    p->model = model;
    if (model == FF_MODEL_LOGNORMAL_1) {
        const double lo[5] = {0.0, 350.0, 1.0, -0.2, -5e-4};
        const double hi[5] = {0.5, 2200.0, 500.0, 1.0, 5e-4};
        const double x0[5] = {0.01, 1000.0, 150.0, 0.2, 0.0};
        for (int j = 0; j < 5; ++j) { p->lo[j] = lo[j]; p->hi[j] = hi[j]; p->x0[j] = x0[j]; }
    } else if (model == FF_MODEL_LOGNORMAL_2) {
        const double lo[8] = {0.0, 0.0, 350.0, 1.0, 900.0, 1.0, -0.2, -5e-4};
        const double hi[8] = {0.5, 1.0, 900.0, 500.0, 2200.0, 500.0, 1.0, 5e-4};
        const double x0[8] = {0.01, 0.5, 650.0, 150.0, 1200.0, 150.0, 0.2, 0.0};
        for (int j = 0; j < 8; ++j) { p->lo[j] = lo[j]; p->hi[j] = hi[j]; p->x0[j] = x0[j]; }
    } else if (model == FF_MODEL_GAUSS_GRID_2) {
        const double lo[8] = {0.0, 0.0, 350.0, 10.0, 900.0, 10.0, -0.2, -5e-4};
        const double hi[8] = {0.5, 1.0, 900.0, 500.0, 2200.0, 500.0, 1.0, 5e-4};
        const double x0[8] = {0.01, 0.5, 650.0, 150.0, 1200.0, 150.0, 0.2, 0.0};
        for (int j = 0; j < 8; ++j) { p->lo[j] = lo[j]; p->hi[j] = hi[j]; p->x0[j] = x0[j]; }
    } else if (model == FF_MODEL_ENDMEMBER_1) {
        const double lo[8] = {0.0, 350.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const double hi[8] = {0.5, 2200.0, 500.0, 1.0, 1.0, 1.0, 1.0, 1.0};
        const double x0[8] = {0.01, 1000.0, 150.0, 0.2, 0.2, 0.2, 0.2, 0.2};
        for (int j = 0; j < 8; ++j) { p->lo[j] = lo[j]; p->hi[j] = hi[j]; p->x0[j] = x0[j]; }
    } else if (model == FF_MODEL_FULL) {
        const double lo[11] = {0.0, 0.0, 350.0, 10.0, 900.0, 10.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const double hi[11] = {0.5, 1.0, 900.0, 500.0, 2200.0, 500.0, 1.0, 1.0, 1.0, 1.0, 1.0};
        const double x0[11] = {0.01, 0.5, 650.0, 150.0, 1200.0, 150.0, 0.2, 0.2, 0.2, 0.2, 0.2};
        for (int j = 0; j < 11; ++j) { p->lo[j] = lo[j]; p->hi[j] = hi[j]; p->x0[j] = x0[j]; }
    } else {
        return set_error(FF_EINVAL, "ff_prior_default: unknown model");
    }
    return clear_error();
}

extern "C" ff_status ff_gauss_hermite(int32_t q, double* x, double* w)
{
    if (!x || !w) return set_error(FF_EINVAL, "ff_gauss_hermite: NULL output");
    if (q < 1 || q > 64) return set_error(FF_EINVAL, "ff_gauss_hermite: q must be in [1, 64]");
    if (!gauss_hermite(q, x, w)) return set_error(FF_EDEVICE, "ff_gauss_hermite: root bracketing failed");
    return clear_error();
}

extern "C" ff_status ff_forward(const ff_scene* scene, int32_t model, int32_t precision, int32_t n_quad,
                                const void* state_dev, int64_t P, void* radiance_dev, void* jac_dev,
                                void* stream)
{
    if (!scene) return set_error(FF_EINVAL, "ff_forward: scene is NULL");
    if (n_state(model) < 0) return set_error(FF_EINVAL, "ff_forward: unknown model");
    if (precision != FF_PRECISION_FP32 && precision != FF_PRECISION_FP64)
        return set_error(FF_EINVAL, "ff_forward: unknown precision");
    if (P < 0) return set_error(FF_EINVAL, "ff_forward: P < 0");
    if (P == 0) return clear_error();
    if (!state_dev || !radiance_dev) return set_error(FF_EINVAL, "ff_forward: NULL state or radiance");
    if (check_library(model, scene, "ff_forward") != FF_OK) return FF_EINVAL;
    return dispatch_forward(precision, model, n_quad, scene, state_dev, P, radiance_dev, jac_dev,
                            (hipStream_t)stream);
}

static ff_status retrieve_batch(const char* who, const ff_scene* const* scenes, const float* const* radiance_dev,
                                const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                const float* const* z0_dev, const ff_options* opts, const ff_outputs* outs,
                                unsigned long long* evals_dev, void* stream, bool noalloc)
{
    const std::string w(who);
    if (n_scenes < 0) return set_error(FF_EINVAL, w + ": n_scenes < 0");
    if (noalloc && n_scenes > FF_NOALLOC_MAX_SCENES)
        return set_error(FF_EINVAL, w + ": at most FF_NOALLOC_MAX_SCENES (" + std::to_string(FF_NOALLOC_MAX_SCENES) +
                                        ") scenes per call, got " + std::to_string(n_scenes));
    if (n_scenes == 0) return clear_error();
    if (!scenes || !radiance_dev || !P || !outs) return set_error(FF_EINVAL, w + ": NULL array");
    ff_status s = check_prior(prior);
    if (s != FF_OK) return s;
    s = check_options(opts);
    if (s != FF_OK) return s;
    int B = -1;
    for (int i = 0; i < n_scenes; ++i) {
        if (!scenes[i]) return set_error(FF_EINVAL, w + ": NULL scene");
        if (P[i] < 0) return set_error(FF_EINVAL, w + ": P < 0");
        if (B < 0) B = scenes[i]->n_bands;
        if (scenes[i]->n_bands != B) return set_error(FF_EINVAL, w + ": scenes differ in band count");
        if (P[i] > 0 && !radiance_dev[i]) return set_error(FF_EINVAL, w + ": NULL radiance");
        if (check_library(prior->model, scenes[i], who) != FF_OK) return FF_EINVAL;
    }
    BatchSpec bs{scenes, radiance_dev, P, n_scenes, prior, z0_dev, opts, outs, evals_dev, (hipStream_t)stream};
    if (noalloc) {
        s = noalloc_scratch(&bs.fixed_scratch, &bs.fixed_bytes);
        if (s != FF_OK) return s;
    }
    return dispatch_lm(opts->precision, prior->model, opts->n_quad, bs);
}

extern "C" ff_status ff_retrieve_batch(const ff_scene* const* scenes, const float* const* radiance_dev,
                                       const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                       const float* const* z0_dev, const ff_options* opts,
                                       const ff_outputs* outs, unsigned long long* evals_dev,
                                       void* stream)
{
    return retrieve_batch("ff_retrieve_batch", scenes, radiance_dev, P, n_scenes, prior, z0_dev, opts, outs,
                          evals_dev, stream, false);
}

extern "C" ff_status ff_retrieve_batch_noalloc(const ff_scene* const* scenes, const float* const* radiance_dev,
                                               const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                               const float* const* z0_dev, const ff_options* opts,
                                               const ff_outputs* outs, unsigned long long* evals_dev,
                                               void* stream)
{
    return retrieve_batch("ff_retrieve_batch_noalloc", scenes, radiance_dev, P, n_scenes, prior, z0_dev, opts,
                          outs, evals_dev, stream, true);
}

extern "C" ff_status ff_retrieve_listed(const ff_scene* scene, const float* radiance_dev, int64_t P,
                                        const int64_t* index_dev, const int64_t* count_dev, const ff_prior* prior,
                                        const float* z0_dev, const ff_options* opts, const ff_outputs* out,
                                        unsigned long long* evals_dev, void* stream)
{
    if (!scene || !out) return set_error(FF_EINVAL, "ff_retrieve_listed: NULL scene or outputs");
    if (P < 0) return set_error(FF_EINVAL, "ff_retrieve_listed: P < 0");
    if (P == 0) return clear_error();
    if (!radiance_dev || !index_dev || !count_dev)
        return set_error(FF_EINVAL, "ff_retrieve_listed: NULL radiance, index or count");
    ff_status s = check_prior(prior);
    if (s != FF_OK) return s;
    s = check_options(opts);
    if (s != FF_OK) return s;
    if (check_library(prior->model, scene, "ff_retrieve_listed") != FF_OK) return FF_EINVAL;
    const float* const rads[1] = {radiance_dev};
    const float* const z0s[1] = {z0_dev};
    const ff_scene* const scs[1] = {scene};
    const int64_t Ps[1] = {P};
    BatchSpec bs{scs, rads, Ps, 1, prior, z0_dev ? z0s : nullptr, opts, out, evals_dev, (hipStream_t)stream};
    bs.index = index_dev;
    bs.count_dev = count_dev;
    return dispatch_lm(opts->precision, prior->model, opts->n_quad, bs);
}

extern "C" ff_status ff_retrieve_atm_indexed(const ff_scene* const* atmospheres, int32_t n_atm,
                                             const int32_t* atm_index_dev, const float* radiance_dev, int64_t P,
                                             const ff_prior* prior, const float* z0_dev, const ff_options* opts,
                                             const ff_outputs* out, unsigned long long* evals_dev, void* stream)
{
    if (!atmospheres || !out) return set_error(FF_EINVAL, "ff_retrieve_atm_indexed: NULL atmospheres or outputs");
    if (n_atm < 1 || n_atm > FF_MAX_ATMOSPHERES)
        return set_error(FF_EINVAL, "ff_retrieve_atm_indexed: n_atm must be in [1, FF_MAX_ATMOSPHERES]");
    for (int a = 0; a < n_atm; ++a) {
        if (!atmospheres[a]) return set_error(FF_EINVAL, "ff_retrieve_atm_indexed: NULL atmosphere");
        if (atmospheres[a]->n_bands != atmospheres[0]->n_bands)
            return set_error(FF_EINVAL, "ff_retrieve_atm_indexed: atmospheres differ in band count");
    }
    if (P < 0) return set_error(FF_EINVAL, "ff_retrieve_atm_indexed: P < 0");
    if (P == 0) return clear_error();
    if (!radiance_dev || !atm_index_dev) return set_error(FF_EINVAL, "ff_retrieve_atm_indexed: NULL radiance or index");
    ff_status s = check_prior(prior);
    if (s != FF_OK) return s;
    s = check_options(opts);
    if (s != FF_OK) return s;
    for (int a = 0; a < n_atm; ++a)
        if (check_library(prior->model, atmospheres[a], "ff_retrieve_atm_indexed") != FF_OK) return FF_EINVAL;
    const float* const rads[1] = {radiance_dev};
    const float* const z0s[1] = {z0_dev};
    const ff_scene* const scs[1] = {atmospheres[0]};
    const int64_t Ps[1] = {P};
    BatchSpec bs{scs, rads, Ps, 1, prior, z0_dev ? z0s : nullptr, opts, out, evals_dev, (hipStream_t)stream};
    bs.atms = atmospheres;
    bs.n_atm = n_atm;
    bs.atm_index = atm_index_dev;
    return dispatch_lm(opts->precision, prior->model, opts->n_quad, bs);
}

extern "C" ff_status ff_retrieve_scene(const ff_scene* scene, const float* radiance_dev, int64_t P,
                                       const ff_prior* prior, const float* z0_dev, const ff_options* opts,
                                       const ff_outputs* out, unsigned long long* evals_dev, void* stream)
{
    if (!scene || !out) return set_error(FF_EINVAL, "ff_retrieve_scene: NULL scene or outputs");
    const float* const rads[1] = {radiance_dev};
    const float* const z0s[1] = {z0_dev};
    const ff_scene* const scs[1] = {scene};
    const int64_t Ps[1] = {P};
    return ff_retrieve_batch(scs, rads, Ps, 1, prior, z0s, opts, out, evals_dev, stream);
}

extern "C" ff_status ff_retrieve(const float* radiance_dev, int64_t P, const ff_srf* srf,
                                 const ff_atmosphere* atm, const ff_prior* prior, const float* z0_dev,
                                 const ff_options* opts, const ff_outputs* out, void* stream)
{
    if (srf == nullptr || atm == nullptr) return set_error(FF_EINVAL, "ff_retrieve: NULL srf/atmosphere");
    ff_scene* sc = nullptr;
    ff_status s = ff_scene_create(srf, atm, &sc);
    if (s != FF_OK) return s;
    s = ff_retrieve_scene(sc, radiance_dev, P, prior, z0_dev, opts, out, nullptr, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    ff_scene_destroy(sc);
    if (s != FF_OK) return s;
    if (e != hipSuccess) return hip_error(e, "ff_retrieve: stream synchronize");
    return clear_error();
}

extern "C" ff_status ff_adam_options_default(const ff_prior* prior, ff_adam_options* o)
{
    if (!o) return set_error(FF_EINVAL, "ff_adam_options_default: NULL options");
    ff_status s = check_prior(prior);
    if (s != FF_OK) return s;
    *o = ff_adam_options{};
    o->precision = FF_PRECISION_FP32;
    o->accumulate = FF_ACCUMULATE_FP32;
    o->n_quad = 32;
    o->block_size = 256;
    o->lanes_per_pixel = 1;
    o->beta1 = 0.9;
    o->beta2 = 0.999;
    o->eps = 1e-8;
    o->n_stages = 2;
    const double nan = std::nan("");
    auto zdef = [&](int j) { return 2.0 * (prior->x0[j] - prior->lo[j]) / (prior->hi[j] - prior->lo[j]) - 1.0; };
    auto set = [&](ff_adam_stage& st, int j, double lo, double hi) {
        st.free_mask |= 1u << j;
        st.window_lo_nm[j] = lo;
        st.window_hi_nm[j] = hi;
    };
    for (int k = 0; k < FF_MAX_ADAM_STAGES; ++k)
        for (int j = 0; j < FF_MAX_STATE; ++j) o->stage[k].z_start[j] = nan;
    ff_adam_stage& s1 = o->stage[0];
    ff_adam_stage& s2 = o->stage[1];
    s1.steps = 30;
    s1.lr = 0.03;
    s1.clip_norm = 1.0;
    s2.steps = 100;
    s2.lr = 0.015;
    s2.clip_norm = 1.0;
    // stage 1: one temperature (spread at its lower bound), f and the
    // reflectance over the whole range; stage 2: f and the temperature
    // distribution over the SWIR windows, reflectance held
    const double w1lo = 350.0, w1hi = 2500.0;          // Omega_1
    const double hot_lo = 900.0, hot_hi = 1800.0;      // Omega_2 flaming
    const double smol_lo = 1500.0, smol_hi = 2500.0;   // Omega_2 smouldering
    if (prior->model == FF_MODEL_LOGNORMAL_1 || prior->model == FF_MODEL_ENDMEMBER_1) {
        // the endmember surface: its fractions take the reflectance's place
        // in stage 1 (the paper's x_1 = {x_surf, alpha_1, T_1})
        if (prior->model == FF_MODEL_LOGNORMAL_1) {
            for (int j : {0, 1, 3, 4}) set(s1, j, w1lo, w1hi);
        } else {
            for (int j : {0, 1, 3, 4, 5, 6, 7}) set(s1, j, w1lo, w1hi);
        }
        s1.z_start[2] = -1.0;
        for (int j : {0, 1, 2}) set(s2, j, hot_lo, smol_hi);
        s2.z_start[2] = zdef(2);
    } else {
        // two components; with the endmember surface (the paper's full
        // model) stage 1 frees exactly x_1 = {x_surf, alpha_1, T_1}
        if (prior->model == FF_MODEL_FULL) {
            for (int j : {0, 4, 6, 7, 8, 9, 10}) set(s1, j, w1lo, w1hi);
        } else {
            for (int j : {0, 4, 6, 7}) set(s1, j, w1lo, w1hi);
        }
        s1.z_start[1] = 1.0;     // all weight on the flaming component
        s1.z_start[5] = -1.0;
        set(s2, 0, hot_lo, smol_hi);
        set(s2, 1, hot_lo, smol_hi);
        set(s2, 2, smol_lo, smol_hi);
        set(s2, 3, smol_lo, smol_hi);
        set(s2, 4, hot_lo, hot_hi);
        set(s2, 5, hot_lo, hot_hi);
        s2.z_start[1] = zdef(1);
        s2.z_start[3] = zdef(3);
        s2.z_start[5] = zdef(5);
    }
    return clear_error();
}

extern "C" ff_status ff_adam_retrieve_batch(const ff_scene* const* scenes, const float* const* radiance_dev,
                                            const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                            const float* const* z0_dev, const ff_adam_options* opts,
                                            const ff_outputs* outs, unsigned long long* evals_dev,
                                            void* stream)
{
    if (n_scenes < 0) return set_error(FF_EINVAL, "ff_adam_retrieve_batch: n_scenes < 0");
    if (n_scenes == 0) return clear_error();
    if (!scenes || !radiance_dev || !P || !outs) return set_error(FF_EINVAL, "ff_adam_retrieve_batch: NULL array");
    ff_status s = check_prior(prior);
    if (s != FF_OK) return s;
    s = check_adam_options(opts, n_state(prior->model));
    if (s != FF_OK) return s;
    int B = -1;
    for (int i = 0; i < n_scenes; ++i) {
        if (!scenes[i]) return set_error(FF_EINVAL, "ff_adam_retrieve_batch: NULL scene");
        if (P[i] < 0) return set_error(FF_EINVAL, "ff_adam_retrieve_batch: P < 0");
        if (B < 0) B = scenes[i]->n_bands;
        if (scenes[i]->n_bands != B) return set_error(FF_EINVAL, "ff_adam_retrieve_batch: scenes differ in band count");
        if (P[i] > 0 && !radiance_dev[i]) return set_error(FF_EINVAL, "ff_adam_retrieve_batch: NULL radiance");
        if (check_library(prior->model, scenes[i], "ff_adam_retrieve_batch") != FF_OK) return FF_EINVAL;
    }
    AdamSpec as{scenes, radiance_dev, P, n_scenes, prior, z0_dev, opts, outs, evals_dev, (hipStream_t)stream};
    return dispatch_adam(as);
}
