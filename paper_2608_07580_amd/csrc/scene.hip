// Scene setup: Gaussian spectral-response resampling of the high-resolution
// atmosphere onto the instrument bands and the per-band constants of the
// forward model (eq. solar, eq. thermal).  One workgroup per band, FP64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ff_internal.hpp"

namespace ff {
namespace {

constexpr int kSetupThreads = 256;

// Per band b: weights w_j = exp(-(l_j - lambda_b)^2 / (2 sig_b^2)) on the
// high-resolution samples within +-4 sig_b, normalised to sum 1; the
// resampled value of a spectrum X is sum_j w_j X_j.
__global__ void __launch_bounds__(kSetupThreads)
srf_band_tables(int B, int H, const double* __restrict__ lam_b, const double* __restrict__ fwhm_b,
                const double* __restrict__ hr_lam, const double* __restrict__ e_sol,
                const double* __restrict__ t_dn, const double* __restrict__ t_up,
                const double* __restrict__ r_atm, const double* __restrict__ s_sph,
                const float* __restrict__ sat, double cos_sza,
                double* __restrict__ tab64, float* __restrict__ tab32, int* __restrict__ bad)
{
    const int b = blockIdx.x;
    if (b >= B) return;
    const double lc = lam_b[b];
    const double sig = fwhm_b[b] / (2.0 * sqrt(2.0 * log(2.0)));
    double acc[6] = {0, 0, 0, 0, 0, 0};  // sum w, w E, w t_dn, w t_up, w rho_atm, w S
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const double d = hr_lam[j] - lc;
        if (fabs(d) > 4.0 * sig) continue;
        const double w = exp(-0.5 * (d / sig) * (d / sig));
        acc[0] += w;
        acc[1] += w * e_sol[j];
        acc[2] += w * t_dn[j];
        acc[3] += w * t_up[j];
        acc[4] += w * r_atm[j];
        acc[5] += w * s_sph[j];
    }
    __shared__ double red[6][kSetupThreads];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int stride = kSetupThreads / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + stride];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sw = red[0][0];
    if (!(sw > 0.0)) { bad[0] = 1; return; }
    const double E = red[1][0] / sw, tdn = red[2][0] / sw, tup = red[3][0] / sw;
    const double ratm = red[4][0] / sw, S = red[5][0] / sw;
    const double c1 = 2.0 * kPlanck * kLight * kLight;   // W m^2 sr^-1
    const double c2 = kPlanck * kLight / kBoltzmann;     // m K
    const double lam_m = lc * 1e-9;
    double row[FF_TABLE_COLS];
    row[COL_LAMBDA] = lc;
    row[COL_K] = E * cos_sza / M_PI;
    row[COL_TAU2] = tdn * tup;
    row[COL_TUP] = tup;
    row[COL_RATM] = ratm;
    row[COL_S] = S;
    row[COL_LSAT] = sat ? (double)sat[b] : INFINITY;
    row[COL_A2] = c2 / lam_m * M_LOG2E;
    row[COL_CB] = c1 / (lam_m * lam_m * lam_m * lam_m * lam_m) * 1e-9;
    row[COL_CJ] = row[COL_CB] * M_LN2;
    row[COL_DLAM] = lc - kLambdaRefNm;
    row[COL_PAD] = 0.0;
    for (int c = 0; c < FF_TABLE_COLS; ++c) {
        tab64[b * FF_TABLE_COLS + c] = row[c];
        tab32[b * FF_TABLE_COLS + c] = (float)row[c];
    }
}

// Band resampling of the endmember library with the same Gaussian
// responses as srf_band_tables: one workgroup per band, FP64 sums, rows
// written to the endmember section of both tables.
__global__ void __launch_bounds__(kSetupThreads)
srf_endmembers(int B, int H, const double* __restrict__ lam_b, const double* __restrict__ fwhm_b,
               const double* __restrict__ hr_lam, const double* __restrict__ refl,
               double* __restrict__ endm64, float* __restrict__ endm32, int* __restrict__ bad)
{
    const int b = blockIdx.x;
    if (b >= B) return;
    const double lc = lam_b[b];
    const double sig = fwhm_b[b] / (2.0 * sqrt(2.0 * log(2.0)));
    constexpr int NE = FF_N_ENDMEMBERS;
    double acc[NE + 1] = {};
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const double d = hr_lam[j] - lc;
        if (fabs(d) > 4.0 * sig) continue;
        const double w = exp(-0.5 * (d / sig) * (d / sig));
        acc[0] += w;
#pragma unroll
        for (int k = 0; k < NE; ++k) acc[k + 1] += w * refl[(size_t)k * H + j];
    }
    __shared__ double red[NE + 1][kSetupThreads];
    for (int c = 0; c <= NE; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int stride = kSetupThreads / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
            for (int c = 0; c <= NE; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + stride];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sw = red[0][0];
    if (!(sw > 0.0)) { bad[0] = 1; return; }
    for (int c = 0; c < kEndmCols; ++c) {
        const double v = c < NE ? red[c + 1][0] / sw : 0.0;
        endm64[(size_t)b * kEndmCols + c] = v;
        endm32[(size_t)b * kEndmCols + c] = (float)v;
    }
}

}  // namespace
}  // namespace ff

namespace ff {
namespace {

struct GridInv {
    float t[kGridNodes];   // 1/T_k of the grid nodes, as the kernels hold them
};

// Grid Planck ratios of the Gaussian-grid thermal model, one row per band:
// q_k = 1/(2^(a2 * (1/T_k)) - 1), by the FP32 operations the band loop uses.
__global__ void grid_planck(int B, const float* __restrict__ tab32, GridInv inv, float* __restrict__ out)
{
    const int b = blockIdx.x, k = threadIdx.x;
    if (b >= B || k >= kGridNodes) return;
    const float a2 = tab32[(size_t)b * FF_TABLE_COLS + COL_A2];
    const float x = a2 * inv.t[k];
    out[(size_t)b * kGridNodes + k] = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(x) - 1.0f);
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" ff_status ff_scene_create(const ff_srf* srf, const ff_atmosphere* atm, ff_scene** out)
{
    if (!out) return set_error(FF_EINVAL, "ff_scene_create: out is NULL");
    *out = nullptr;
    if (!srf || !atm) return set_error(FF_EINVAL, "ff_scene_create: srf/atm is NULL");
    if (srf->n_bands <= 0 || !srf->wavelength_nm || !srf->fwhm_nm)
        return set_error(FF_EINVAL, "ff_scene_create: bad band description");
    if (atm->n_hr <= 0 || !atm->lambda_nm || !atm->e_solar || !atm->tau_down || !atm->tau_up ||
        !atm->rho_atm || !atm->s_sph)
        return set_error(FF_EINVAL, "ff_scene_create: bad atmosphere description");
    const int B = srf->n_bands, H = atm->n_hr;
    for (int b = 0; b < B; ++b) {
        if (!(srf->fwhm_nm[b] > 0.0) || !std::isfinite(srf->wavelength_nm[b]) ||
            !(srf->wavelength_nm[b] > 0.0))
            return set_error(FF_EINVAL, "ff_scene_create: non-positive FWHM or wavelength");
    }
    if (!std::isfinite(atm->cos_sza)) return set_error(FF_EINVAL, "ff_scene_create: cos_sza");

    ff_scene* sc = new ff_scene();
    sc->n_bands = B;
    sc->lambda.assign(srf->wavelength_nm, srf->wavelength_nm + B);
    sc->fwhm.assign(srf->fwhm_nm, srf->fwhm_nm + B);
    // every resampled S_b is then exactly 0 (a weighted mean of zeros)
    sc->s_zero = std::all_of(atm->s_sph, atm->s_sph + H, [](double v) { return v == 0.0; });
    if (atm->sat_level) sc->lsat.assign(atm->sat_level, atm->sat_level + B);
    else sc->lsat.assign(B, INFINITY);
    hipError_t e = hipGetDevice(&sc->device);
    // staging: [lam_b, fwhm_b, hr_lam, E, tdn, tup, ratm, S] doubles + sat floats + bad flag
    const size_t nd = 2 * (size_t)B + 6 * (size_t)H;
    double* stage = nullptr;
    float* sat_d = nullptr;
    int* bad_d = nullptr;
    if (e == hipSuccess) e = hipMalloc(&stage, nd * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&sat_d, (size_t)B * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&bad_d, sizeof(int));
    const size_t n_tab = (size_t)B * (FF_TABLE_COLS + kEndmCols);
    const size_t n_tab32 = n_tab + (size_t)B * kGridNodes;   // + the grid Planck ratios
    if (e == hipSuccess) e = hipMalloc(&sc->table_f64, n_tab * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&sc->table_f32, n_tab32 * sizeof(float));
    if (e == hipSuccess) e = hipMemset(sc->table_f64, 0, n_tab * sizeof(double));
    if (e == hipSuccess) e = hipMemset(sc->table_f32, 0, n_tab32 * sizeof(float));
    if (e == hipSuccess) {
        std::vector<double> host(nd);
        std::memcpy(&host[0], srf->wavelength_nm, B * sizeof(double));
        std::memcpy(&host[B], srf->fwhm_nm, B * sizeof(double));
        const double* src[6] = {atm->lambda_nm, atm->e_solar, atm->tau_down, atm->tau_up,
                                atm->rho_atm, atm->s_sph};
        for (int i = 0; i < 6; ++i) std::memcpy(&host[2 * B + (size_t)i * H], src[i], H * sizeof(double));
        e = hipMemcpy(stage, host.data(), nd * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && atm->sat_level)
        e = hipMemcpy(sat_d, atm->sat_level, (size_t)B * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(bad_d, 0, sizeof(int));
    if (e == hipSuccess) {
        const double* s = stage;
        hipLaunchKernelGGL(srf_band_tables, dim3(B), dim3(kSetupThreads), 0, 0, B, H, s, s + B,
                           s + 2 * B, s + 2 * B + H, s + 2 * B + 2 * (size_t)H, s + 2 * B + 3 * (size_t)H,
                           s + 2 * B + 4 * (size_t)H, s + 2 * B + 5 * (size_t)H,
                           atm->sat_level ? sat_d : nullptr, atm->cos_sza, sc->table_f64,
                           sc->table_f32, bad_d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        GridInv inv;
        for (int k = 0; k < kGridNodes; ++k) inv.t[k] = (float)(1.0 / grid_node<kGridNodes>(k));
        hipLaunchKernelGGL(grid_planck, dim3(B), dim3(kGridNodes), 0, 0, B, sc->table_f32, inv, sc->table_f32 + n_tab);
        e = hipGetLastError();
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpy(&bad, bad_d, sizeof(int), hipMemcpyDeviceToHost);
    hipFree(stage);
    hipFree(sat_d);
    hipFree(bad_d);
    if (e != hipSuccess) {
        ff_scene_destroy(sc);
        return hip_error(e, "ff_scene_create");
    }
    if (bad) {
        ff_scene_destroy(sc);
        return set_error(FF_EINVAL, "ff_scene_create: a band's response window holds no high-resolution sample");
    }
    *out = sc;
    return clear_error();
}

extern "C" void ff_scene_destroy(ff_scene* sc)
{
    if (!sc) return;
    if (sc->table_f32) hipFree(sc->table_f32);
    if (sc->table_f64) hipFree(sc->table_f64);
    delete sc;
}

extern "C" int32_t ff_scene_n_bands(const ff_scene* sc) { return sc ? sc->n_bands : 0; }

extern "C" ff_status ff_scene_band_tables(const ff_scene* sc, double* out_host)
{
    if (!sc || !out_host) return set_error(FF_EINVAL, "ff_scene_band_tables: NULL argument");
    FF_HIP_TRY(hipMemcpy(out_host, sc->table_f64, (size_t)sc->n_bands * FF_TABLE_COLS * sizeof(double),
                         hipMemcpyDeviceToHost));
    return clear_error();
}

extern "C" ff_status ff_scene_set_endmembers(ff_scene* sc, int32_t n_hr, const double* lambda_nm,
                                             const double* reflectance_host)
{
    if (!sc || !lambda_nm || !reflectance_host) return set_error(FF_EINVAL, "ff_scene_set_endmembers: NULL argument");
    if (n_hr < 1) return set_error(FF_EINVAL, "ff_scene_set_endmembers: n_hr < 1");
    const int B = sc->n_bands, H = n_hr;
    if ((int)sc->fwhm.size() != B || (int)sc->lambda.size() != B)
        return set_error(FF_EINVAL, "ff_scene_set_endmembers: scene without band responses");
    for (int j = 0; j < H; ++j)
        if (!std::isfinite(lambda_nm[j])) return set_error(FF_EINVAL, "ff_scene_set_endmembers: non-finite wavelength");
    for (size_t i = 0; i < (size_t)FF_N_ENDMEMBERS * H; ++i)
        if (!std::isfinite(reflectance_host[i]))
            return set_error(FF_EINVAL, "ff_scene_set_endmembers: non-finite reflectance");
    int cur = 0;
    FF_HIP_TRY(hipGetDevice(&cur));
    if (cur != sc->device) FF_HIP_TRY(hipSetDevice(sc->device));
    const size_t nd = 2 * (size_t)B + (size_t)H * (1 + FF_N_ENDMEMBERS);
    double* stage = nullptr;
    int* bad_d = nullptr;
    hipError_t e = hipMalloc(&stage, nd * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&bad_d, sizeof(int));
    if (e == hipSuccess) {
        std::vector<double> host(nd);
        std::memcpy(&host[0], sc->lambda.data(), B * sizeof(double));
        std::memcpy(&host[B], sc->fwhm.data(), B * sizeof(double));
        std::memcpy(&host[2 * (size_t)B], lambda_nm, H * sizeof(double));
        std::memcpy(&host[2 * (size_t)B + H], reflectance_host, (size_t)FF_N_ENDMEMBERS * H * sizeof(double));
        e = hipMemcpy(stage, host.data(), nd * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(bad_d, 0, sizeof(int));
    if (e == hipSuccess) {
        const size_t off = (size_t)B * FF_TABLE_COLS;
        hipLaunchKernelGGL(srf_endmembers, dim3(B), dim3(kSetupThreads), 0, 0, B, H, stage, stage + B,
                           stage + 2 * B, stage + 2 * (size_t)B + H, sc->table_f64 + off, sc->table_f32 + off, bad_d);
        e = hipGetLastError();
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpy(&bad, bad_d, sizeof(int), hipMemcpyDeviceToHost);
    hipFree(stage);
    hipFree(bad_d);
    if (cur != sc->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_error(e, "ff_scene_set_endmembers");
    if (bad) {
        sc->has_endmembers = false;
        return set_error(FF_EINVAL, "ff_scene_set_endmembers: a band's response window holds no sample");
    }
    sc->has_endmembers = true;
    return clear_error();
}

extern "C" ff_status ff_scene_endmembers(const ff_scene* sc, double* out_host)
{
    if (!sc || !out_host) return set_error(FF_EINVAL, "ff_scene_endmembers: NULL argument");
    if (!sc->has_endmembers) return set_error(FF_EINVAL, "ff_scene_endmembers: no library set");
    const int B = sc->n_bands;
    std::vector<double> rows((size_t)B * kEndmCols);
    FF_HIP_TRY(hipMemcpy(rows.data(), sc->table_f64 + (size_t)B * FF_TABLE_COLS, rows.size() * sizeof(double),
                         hipMemcpyDeviceToHost));
    for (int k = 0; k < FF_N_ENDMEMBERS; ++k)
        for (int b = 0; b < B; ++b) out_host[(size_t)k * B + b] = rows[(size_t)b * kEndmCols + k];
    return clear_error();
}
