// Internal declarations of the firefit HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "firefit.h"

namespace ff {

// ---- errors ---------------------------------------------------------------
ff_status set_error(ff_status code, const std::string& msg);
ff_status clear_error();
ff_status hip_error(hipError_t e, const char* what);

#define FF_HIP_TRY(expr)                                   \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return ff::hip_error(_e, #expr); \
    } while (0)

// ---- physical constants (exact SI values) ----------------------------------
constexpr double kPlanck = 6.62607015e-34;
constexpr double kLight = 299792458.0;
constexpr double kBoltzmann = 1.380649e-23;
constexpr double kLambdaRefNm = 1440.0;   // reference wavelength of the reflectance slope

// ---- per-band table layout: row of FF_TABLE_COLS values per band -----------
// 0..6 are documented in firefit.h; 7..10 are derived constants of the
// range-scaled Planck evaluation:
//   a2 = c2 / lambda * log2(e)  [K]  so that exp(-c2/(lambda T)) = 2^(-a2 / T)
//   cb = c1 / lambda^5 per nm    [W m^-2 sr^-1 nm^-1]
//   cj = cb * ln 2               (T dB/dT = cj * x2 e / (1 - e)^2 with x2 = a2 / T)
//   dl = lambda - 1440 nm
enum TableCol : int {
    COL_LAMBDA = 0, COL_K = 1, COL_TAU2 = 2, COL_TUP = 3, COL_RATM = 4, COL_S = 5, COL_LSAT = 6,
    COL_A2 = 7, COL_CB = 8, COL_CJ = 9, COL_DLAM = 10, COL_PAD = 11
};
static_assert(FF_TABLE_COLS == 12, "table layout");

// The endmember library follows the band rows in the same allocation: row b
// of that section (kEndmCols values, FF_N_ENDMEMBERS used, the rest zero)
// starts at table + B * FF_TABLE_COLS + b * kEndmCols.
constexpr int kEndmCols = 8;
static_assert(FF_N_ENDMEMBERS <= kEndmCols, "endmember row");

// The FP32 table then holds the Planck ratios of the Gaussian-grid thermal
// model on its kGridNodes-node temperature grid, which do not depend on the
// pixel: row b, q_k = 1/(2^(a2_b / T_k) - 1), starts at
// table + B * (FF_TABLE_COLS + kEndmCols) + b * kGridNodes (FP32 table only).
constexpr int kGridNodes = 32;

// Node i of the Q-node temperature grid of the Gaussian-mixture model, K.
template <int Q>
__host__ __device__ constexpr double grid_node(int i) { return 350.0 + (2200.0 - 350.0) * i / (Q - 1); }

}  // namespace ff

// Scene handle: per-band tables in device memory, FP32 and FP64 copies, and
// the band centres on the host.
struct ff_scene {
    int32_t n_bands = 0;
    int device = 0;
    float* table_f32 = nullptr;   // [B][12] band rows, then [B][8] endmember rows
    double* table_f64 = nullptr;  // the same in FP64
    std::vector<double> lambda;   // [B] band centres, nm
    std::vector<double> fwhm;     // [B] band FWHM, nm
    std::vector<float> lsat;      // [B] saturation levels (+inf: none)
    bool has_endmembers = false;  // the endmember section holds a library
    bool s_zero = false;          // spherical albedo 0 on every band: 1 - S rho is exactly 1
};

namespace ff {

// Gauss-Hermite rule computed on the host (nodes by bracketing + Newton on
// the orthonormal Hermite recurrence, weights 1 / (q p_{q-1}(x)^2)).
bool gauss_hermite(int q, double* x, double* w);

// Quadrature weights used by the kernels for the lognormal temperature
// integral: w_hat = w / sqrt(pi), s = sqrt(2) x, v_hat = s * w_hat.
template <typename R, int Q>
struct Quad {
    R w[Q];
    R v[Q];
    R s[Q];
};
bool make_quad_f32(int q, float* w, float* v, float* s);
bool make_quad_f64(int q, double* w, double* v, double* s);

int n_state(int model);

// One retrieval launch sequence over a ragged batch of scenes.
struct BatchSpec {
    const ff_scene* const* scenes;
    const float* const* radiance;
    const int64_t* P;
    int n_scenes;
    const ff_prior* prior;
    const float* const* z0;
    const ff_options* opts;
    const ff_outputs* outs;
    unsigned long long* evals;
    hipStream_t stream;
    const int64_t* index = nullptr;     // one scene only: pixel rows to solve, or null for all
    const int64_t* count_dev = nullptr; // with index: number of listed pixels, read on the device
    const ff_scene* const* atms = nullptr;  // one scene only: per-pixel atmospheres ...
    int n_atm = 0;
    const int32_t* atm_index = nullptr;     // ... chosen by this [P] index
    void* fixed_scratch = nullptr;          // if set: queue counters and descriptors go here ...
    size_t fixed_bytes = 0;                 // ... (its size), instead of the stream's buffer
};

ff_status dispatch_lm(int precision, int model, int q, const BatchSpec& bs);

// The fixed device array of the allocation-free retrieval on the current
// device (its address looked up once per device) and its size in bytes.
ff_status noalloc_scratch(void** ptr, size_t* bytes);

// One staged-Adam launch sequence over a ragged batch of scenes.
struct AdamSpec {
    const ff_scene* const* scenes;
    const float* const* radiance;
    const int64_t* P;
    int n_scenes;
    const ff_prior* prior;
    const float* const* z0;
    const ff_adam_options* opts;
    const ff_outputs* outs;
    unsigned long long* evals;
    hipStream_t stream;
};

ff_status dispatch_adam(const AdamSpec& as);

// Library-owned, grow-only scratch per (device, stream); growth is refused
// while the stream is being captured into a graph.
ff_status stream_scratch(hipStream_t stream, size_t bytes, void** out);
bool stream_capturing(hipStream_t stream);
void release_stream_scratch(hipStream_t stream);
void pin_stream_scratch(hipStream_t stream);

// Input and output widths of a warm-start network; pin/unpin its activation
// workspace (while pinned, a grown workspace keeps the old buffers alive for
// the graphs that bind them).
void mlp_dims(const ff_mlp* m, int* n_in, int* n_out);
void mlp_pin(const ff_mlp* m, int delta);
ff_status mlp_infer_listed_dev(const ff_mlp* m, const float* rad, int64_t P, const int64_t* index,
                               const int64_t* count_dev, float* z0, hipStream_t s);
ff_status mark_no_start(float* z0, int64_t P, int n, hipStream_t s);
ff_status dispatch_forward(int precision, int model, int q, const ff_scene* sc, const void* state,
                           int64_t P, void* L, void* J, hipStream_t stream);

}  // namespace ff
