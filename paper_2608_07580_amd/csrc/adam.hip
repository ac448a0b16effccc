// Staged-Adam retrieval kernel: the paper's own solver (Keely et al.
// Sec. 2.5, eq. adam; Kingma & Ba 2015) on the windowed loss of eq. (loss) in
// the z coordinate of eq. (affine).
//
// Work mapping: one aligned group of L lanes owns one pixel (static grid,
// one pixel per group).  Every pixel takes the same number of steps, so the
// lanes of a wave stay in lock-step through the whole solve and no queue is
// needed.  A step is one model evaluation that accumulates only the
// windowed gradient (no J^T J): each band carries a bit per state variable
// saying whether the band lies in that variable's window, prepared per scene
// and stage by a small kernel from the FP64 band centres, and bands outside
// every free variable's window are skipped.  The Adam moments, bias
// corrections, clip and z update are per-lane FP64.  After the last stage one
// full evaluation over all unsaturated bands gives J^T J and the loss for the
// shared output epilogue (Gauss-Newton covariance, moments, residual).
#include <algorithm>
#include <cmath>

#include "solve.hpp"

namespace ff {

template <typename R, int Q>
struct AdamDesc {
    SceneDev sc[kMaxScenesPerLaunch];
    const double* tab64[kMaxScenesPerLaunch];  // FP64 table of each scene (band centres)
    uint16_t* bits;                // [scene][stage][B] window bits (bit j: variable j)
    int n_scenes;
    int B;
    int64_t total;
    int lpp;                       // lanes per pixel (power of two, <= 64)
    int n;                         // state variables of the model
    unsigned long long* evals;     // += model evaluations (may be null)
    int n_stages;
    int steps[FF_MAX_ADAM_STAGES];
    uint32_t free_mask[FF_MAX_ADAM_STAGES];
    double lr[FF_MAX_ADAM_STAGES];
    double clip[FF_MAX_ADAM_STAGES];
    double wlo[FF_MAX_ADAM_STAGES][FF_MAX_STATE];
    double whi[FF_MAX_ADAM_STAGES][FF_MAX_STATE];
    double zset[FF_MAX_ADAM_STAGES][FF_MAX_STATE];
    double beta1, beta2, eps;
    double lo[FF_MAX_STATE], hi[FF_MAX_STATE], zdef[FF_MAX_STATE];
};

namespace {

// Window bits of every (scene, stage, band): bit j is set when variable j is
// free in the stage and lo_j <= lambda_b <= hi_j (FP64 band centre).
template <typename Desc>
__global__ void window_bits(const Desc* __restrict__ D)
{
    const int B = D->B, K = D->n_stages;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)D->n_scenes * K * B) return;
    const int b = (int)(i % B);
    const int k = (int)((i / B) % K);
    const int s = (int)(i / ((int64_t)B * K));
    const double lam = D->tab64[s][(size_t)b * FF_TABLE_COLS + COL_LAMBDA];
    unsigned bits = 0;
    for (int j = 0; j < D->n; ++j)
        if (((D->free_mask[k] >> j) & 1u) && lam >= D->wlo[k][j] && lam <= D->whi[k][j]) bits |= 1u << j;
    D->bits[i] = (uint16_t)bits;
}

// Windowed loss gradient in z at physical state x:
//   G_j = -2 (hi_j - lo_j)/2 sum_{b in window_j, unsaturated} r_b dL_b/dx_j,
// with dL/dx_j = c1_j u[s1_j] + c2_j u[s2_j] in the model's basis; the sums
// of u r run per variable over its own bands.  The L lanes of a group take
// bands sub, sub + L, ... and combine their sums across the group.
template <typename R, typename ACC, int MODEL, int Q, typename Desc>
__device__ __forceinline__ void windowed_gradient(const Desc* descp, const float* __restrict__ rad,
                                                  const R* __restrict__ tab, const uint16_t* __restrict__ bits,
                                                  const double (&x)[ModelDims<MODEL>::N],
                                                  double (&G)[ModelDims<MODEL>::N], int sub, int L)
{
    using PM = PixelModel<R, MODEL, Q>;
    constexpr int N = PM::N;
    const int B = launder(descp)->B;
    PM pm;
    pm.setup(x, sub, L);
    ACC h1[N], h2[N];
#pragma unroll
    for (int j = 0; j < N; ++j) h1[j] = h2[j] = (ACC)0;

    for (int b0 = sub; b0 < B; b0 += 4 * L) {
        // radiance and window bits of four bands per load group
        float l0 = rad[b0];
        float l1 = b0 + L < B ? rad[b0 + L] : 0.f;
        float l2 = b0 + 2 * L < B ? rad[b0 + 2 * L] : 0.f;
        float l3 = b0 + 3 * L < B ? rad[b0 + 3 * L] : 0.f;
        unsigned k0 = bits[b0];
        unsigned k1 = b0 + L < B ? bits[b0 + L] : 0u;
        unsigned k2 = b0 + 2 * L < B ? bits[b0 + 2 * L] : 0u;
        unsigned k3 = b0 + 3 * L < B ? bits[b0 + 3 * L] : 0u;
#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + j * L;
            if (b >= B) break;
            const float lob = l0;
            const unsigned kb = k0;
            l0 = l1;
            l1 = l2;
            l2 = l3;
            k0 = k1;
            k1 = k2;
            k2 = k3;
            if (kb == 0u) continue;
            const int o = opaque_zero();
            const BandRow<R> row = load_row(tab + (size_t)b * FF_TABLE_COLS);
            R ub[N];
            const R lm = band_of<MODEL>(pm, tab, B, b, o, row, ub);
            const bool msk = (R)lob < row.lsat;
            const ACC r = msk ? (ACC)((R)lob - lm) : (ACC)0;
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const ACC rv = ((kb >> v) & 1u) ? r : (ACC)0;
                h1[v] += (ACC)ub[PM::s1[v]] * rv;
                if (PM::s2[v] >= 0) h2[v] += (ACC)ub[PM::s2[v] < 0 ? 0 : PM::s2[v]] * rv;
            }
        }
    }
    if (L > 1) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            h1[j] = group_sum(h1[j], L);
            if (PM::s2[j] >= 0) h2[j] = group_sum(h2[j], L);
        }
    }
    const Desc* D = launder(descp);
    double c1[N], c2[N];
    PM::coefficients(x, c1, c2);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double dl = c1[j] * (double)h1[j];
        if (PM::s2[j] >= 0) dl += c2[j] * (double)h2[j];
        G[j] = -2.0 * (0.5 * (D->hi[j] - D->lo[j])) * dl;
    }
}

// Second launch bound (waves per SIMD), FP32 kernels: the one-component
// model runs three waves per SIMD in at most 168 VGPRs, the others two in
// 256 (some per-pixel state outside the band loop goes to scratch); FP64
// keeps the compiler's choice.
template <typename R, typename ACC, int MODEL, int Q>
__global__ void __launch_bounds__(256, sizeof(R) != 4 ? 1 : (MODEL == FF_MODEL_LOGNORMAL_1 ? 3 : 2))
adam_kernel(const AdamDesc<R, Q>* __restrict__ descp)
{
    using PM = PixelModel<R, MODEL, Q>;
    constexpr int N = PM::N;
    constexpr int NT = N * (N + 1) / 2;
    using Desc = AdamDesc<R, Q>;
    const int L = launder(descp)->lpp;
    const int sub = (threadIdx.x & 63) & (L - 1);
    const bool head = sub == 0;
    const int64_t item = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
    unsigned long long nevals = 0;

    if (item < launder(descp)->total) {
        const Desc* D = launder(descp);
        const int sidx = scene_of(D, item);
        const SceneDev& sd = D->sc[sidx];
        const int64_t pix = item - sd.offset;
        const int B = D->B;
        const float* rad = sd.radiance + pix * B;
        const R* tab = reinterpret_cast<const R*>(sd.table);
        const double* tab64 = sd.table64;
        const OutPtrs o = out_ptrs(sd);
        int nonfin = 0, nvalid = 0;
        double lnorm2 = 0.0;
        scan_pixel<R>(rad, tab, B, sub, L, nonfin, nvalid, lnorm2);
        if (nonfin != 0 || nvalid <= N) {
            if (head) {
                write_nan<N>(o, pix);
                if (o.rrr) o.rrr[pix] = __builtin_nanf("");
                if (o.iters) o.iters[pix] = 0;
                if (o.status) o.status[pix] = nonfin != 0 ? FF_ST_NONFINITE_INPUT : FF_ST_NO_DOF;
            }
        } else {
            const bool warm = sd.z0 != nullptr;
            unsigned st = warm ? FF_ST_WARM_START : 0u;
            double z[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                double zz = warm ? (double)sd.z0[pix * N + j] : D->zdef[j];
                zz = isfinite(zz) ? zz : D->zdef[j];
                z[j] = fmin(1.0, fmax(-1.0, zz));
            }
            project_block<MODEL>(z);
            int steps = 0;
            bool bad = false;
            const int K = D->n_stages;
            for (int k = 0; k < K && !bad; ++k) {
                const Desc* Dk = launder(descp);
                double m[N], v[N];
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    m[j] = v[j] = 0.0;
                    const double zs = Dk->zset[k][j];
                    if (!__builtin_isnan(zs)) z[j] = fmin(1.0, fmax(-1.0, zs));
                }
                project_block<MODEL>(z);
                const uint16_t* bits = Dk->bits + ((size_t)sidx * K + k) * B;
                const int T = Dk->steps[k];
                double p1 = 1.0, p2 = 1.0;    // beta1^t, beta2^t
                for (int t = 1; t <= T; ++t) {
                    double x[N], G[N];
                    {
                        const Desc* Dx = launder(descp);
#pragma unroll
                        for (int j = 0; j < N; ++j) x[j] = Dx->lo[j] + 0.5 * (Dx->hi[j] - Dx->lo[j]) * (z[j] + 1.0);
                    }
                    windowed_gradient<R, ACC, MODEL, Q>(descp, rad, tab, bits, x, G, sub, L);
                    nevals += head ? 1 : 0;
                    const Desc* Ds = launder(descp);
                    double norm2 = 0.0;
                    bool fin = true;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        fin = fin && isfinite(G[j]);
                        norm2 += G[j] * G[j];
                    }
                    if (!fin) {
                        bad = true;
                        break;
                    }
                    const double norm = sqrt(norm2);
                    const double c = Ds->clip[k];
                    if (c > 0.0 && norm > c) {
                        const double sc = c / norm;
#pragma unroll
                        for (int j = 0; j < N; ++j) G[j] *= sc;
                    }
                    const double b1 = Ds->beta1, b2 = Ds->beta2, eps = Ds->eps, lr = Ds->lr[k];
                    const uint32_t fm = Ds->free_mask[k];
                    p1 *= b1;
                    p2 *= b2;
                    const double bc1 = 1.0 - p1, bc2 = 1.0 - p2;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        if ((fm >> j) & 1u) {
                            m[j] = b1 * m[j] + (1.0 - b1) * G[j];
                            v[j] = b2 * v[j] + (1.0 - b2) * G[j] * G[j];
                            const double mhat = m[j] / bc1, vhat = v[j] / bc2;
                            z[j] = fmin(1.0, fmax(-1.0, z[j] - lr * mhat / (sqrt(vhat) + eps)));
                        }
                    }
                    project_block<MODEL>(z);   // surface mixture back onto the simplex (Sec. 2.5)
                    ++steps;
                }
            }
            // outputs at the final point, over all unsaturated bands
            double x[N];
            bool bound = false;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                x[j] = D->lo[j] + 0.5 * (D->hi[j] - D->lo[j]) * (z[j] + 1.0);
                bound = bound || z[j] <= -1.0 || z[j] >= 1.0;
            }
            double A[NT], g[N];
            double F = __builtin_nan("");
            if (!bad) {
                F = evaluate<R, ACC, MODEL, Q>(descp, rad, tab, tab64, x, A, g, sub, L);
                nevals += head ? 1 : 0;
            }
            const Desc* De = launder(descp);
            if (bad || !isfinite(F)) {
                st |= FF_ST_NONFINITE_INPUT;
                if (head) {
                    write_nan<N>(o, pix);
                    if (o.rrr) o.rrr[pix] = __builtin_nanf("");
                    if (o.iters) o.iters[pix] = bad ? 0 : steps;
                    if (o.status) o.status[pix] = st;
                }
            } else if (head) {
                if (bound) st |= FF_ST_AT_BOUND;
                st |= write_solution<R, MODEL, Q>(De, o, pix, x, A, F, nvalid);
                if (o.rrr) o.rrr[pix] = lnorm2 > 0.0 ? (float)sqrt(F / lnorm2) : __builtin_nanf("");
                if (o.iters) o.iters[pix] = steps;
                if (o.status) o.status[pix] = st;
            }
        }
    }
    unsigned long long* evals = launder(descp)->evals;
    if (evals) wave_add(evals, nevals);
}

}  // namespace

template <typename R, typename ACC, int MODEL, int Q>
static ff_status launch_adam(const AdamSpec& as)
{
    const ff_adam_options& o = *as.opts;
    const int block = o.block_size > 0 ? o.block_size : 256;
    const int lpp = o.lanes_per_pixel > 0 ? o.lanes_per_pixel : 1;
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    if (!ensure_tables<R, MODEL, Q>(dev)) return set_error(FF_EDEVICE, "quadrature rule could not be placed on the device");
    int64_t total = 0;
    for (int s = 0; s < as.n_scenes; ++s) total += as.P[s];
    if (total == 0) return clear_error();

    // the stream's scratch: per chunk one descriptor and its window bits
    using Desc = AdamDesc<R, Q>;
    const int n_chunks = (as.n_scenes + kMaxScenesPerLaunch - 1) / kMaxScenesPerLaunch;
    const int K = std::max(o.n_stages, 1);
    const int B = as.scenes[0]->n_bands;
    const size_t desc_bytes = (sizeof(Desc) + 255) / 256 * 256;
    const size_t bits_bytes = ((size_t)kMaxScenesPerLaunch * K * B * sizeof(uint16_t) + 255) / 256 * 256;
    const size_t chunk_bytes = desc_bytes + bits_bytes;
    char* scratch = nullptr;
    {
        const ff_status st = stream_scratch(as.stream, (size_t)n_chunks * chunk_bytes, reinterpret_cast<void**>(&scratch));
        if (st != FF_OK) return st;
    }
    hipError_t e = hipSuccess;
    const int n = ModelDims<MODEL>::N;
    for (int c = 0; c < n_chunks && e == hipSuccess; ++c) {
        Desc prm{};
        int64_t off = 0;
        int ns = 0;
        for (int s = c * kMaxScenesPerLaunch; s < std::min(as.n_scenes, (c + 1) * kMaxScenesPerLaunch); ++s, ++ns) {
            SceneDev& d = prm.sc[ns];
            const ff_outputs& out = as.outs[s];
            d.radiance = as.radiance[s];
            d.table = sizeof(R) == 4 ? (const void*)as.scenes[s]->table_f32 : (const void*)as.scenes[s]->table_f64;
            d.table64 = as.scenes[s]->table_f64;
            d.P = as.P[s];
            d.offset = off;
            d.z0 = as.z0 ? as.z0[s] : nullptr;
            d.state = out.state;
            d.cov = out.cov_packed;
            d.moments = out.moments;
            d.rrr = out.rrr;
            d.iters = out.iters;
            d.status = out.status;
            d.state64 = out.state_f64;
            prm.tab64[ns] = as.scenes[s]->table_f64;
            off += as.P[s];
        }
        for (int s = ns; s < kMaxScenesPerLaunch; ++s) prm.sc[s].offset = INT64_MAX;
        if (off == 0) continue;
        char* base = scratch + (size_t)c * chunk_bytes;
        Desc* dptr = reinterpret_cast<Desc*>(base);
        prm.bits = reinterpret_cast<uint16_t*>(base + desc_bytes);
        prm.n_scenes = ns;
        prm.B = B;
        prm.total = off;
        prm.lpp = lpp;
        prm.n = n;
        prm.evals = as.evals;
        prm.n_stages = o.n_stages;
        for (int k = 0; k < o.n_stages; ++k) {
            const ff_adam_stage& sg = o.stage[k];
            prm.steps[k] = sg.steps;
            prm.free_mask[k] = sg.free_mask;
            prm.lr[k] = sg.lr;
            prm.clip[k] = sg.clip_norm;
            for (int j = 0; j < FF_MAX_STATE; ++j) {
                prm.wlo[k][j] = sg.window_lo_nm[j];
                prm.whi[k][j] = sg.window_hi_nm[j];
                prm.zset[k][j] = sg.z_start[j];
            }
        }
        prm.beta1 = o.beta1;
        prm.beta2 = o.beta2;
        prm.eps = o.eps;
        for (int j = 0; j < FF_MAX_STATE; ++j) {
            prm.lo[j] = j < n ? as.prior->lo[j] : 0.0;
            prm.hi[j] = j < n ? as.prior->hi[j] : 1.0;
            prm.zdef[j] = j < n ? 2.0 * (as.prior->x0[j] - as.prior->lo[j]) / (as.prior->hi[j] - as.prior->lo[j]) - 1.0 : 0.0;
        }
        const int64_t grid = (off * lpp + block - 1) / block;
        if (grid > 0x7fffffff) {
            e = hipErrorInvalidValue;
            break;
        }
        hipLaunchKernelGGL(fill_struct<Desc>, dim3(1), dim3(64), 0, as.stream, prm, dptr);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        const int64_t n_bits = (int64_t)ns * o.n_stages * B;
        if (n_bits > 0) {
            hipLaunchKernelGGL(window_bits<Desc>, dim3((unsigned)((n_bits + 255) / 256)), dim3(256), 0, as.stream,
                               (const Desc*)dptr);
            e = hipGetLastError();
            if (e != hipSuccess) break;
        }
        hipLaunchKernelGGL((adam_kernel<R, ACC, MODEL, Q>), dim3((unsigned)grid), dim3(block), 0, as.stream,
                           (const Desc*)dptr);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_error(e, "adam_kernel launch");
    return clear_error();
}

#define FF_DISPATCH_ADAM_Q(q, ...)                                       \
    switch (q) {                                                    \
    case 16: return launch_adam<__VA_ARGS__, 16>(as);               \
    case 24: return launch_adam<__VA_ARGS__, 24>(as);               \
    case 32: return launch_adam<__VA_ARGS__, 32>(as);               \
    default: return set_error(FF_EUNSUPPORTED, "unsupported quadrature order for FP32 (16, 24, 32)"); \
    }

ff_status dispatch_adam(const AdamSpec& as)
{
    const ff_adam_options& o = *as.opts;
    const int model = as.prior->model;
    const bool acc64 = o.accumulate == FF_ACCUMULATE_FP64;
    if (o.precision == FF_PRECISION_FP32) {
        if (model == FF_MODEL_LOGNORMAL_1) {
            if (acc64) { FF_DISPATCH_ADAM_Q(o.n_quad, float, double, FF_MODEL_LOGNORMAL_1) }
            FF_DISPATCH_ADAM_Q(o.n_quad, float, float, FF_MODEL_LOGNORMAL_1)
        }
        if (model == FF_MODEL_GAUSS_GRID_2) {
            if (acc64) { FF_DISPATCH_ADAM_Q(o.n_quad, float, double, FF_MODEL_GAUSS_GRID_2) }
            FF_DISPATCH_ADAM_Q(o.n_quad, float, float, FF_MODEL_GAUSS_GRID_2)
        }
        if (model == FF_MODEL_ENDMEMBER_1) {
            if (acc64) { FF_DISPATCH_ADAM_Q(o.n_quad, float, double, FF_MODEL_ENDMEMBER_1) }
            FF_DISPATCH_ADAM_Q(o.n_quad, float, float, FF_MODEL_ENDMEMBER_1)
        }
        if (model == FF_MODEL_FULL) {
            if (acc64) { FF_DISPATCH_ADAM_Q(o.n_quad, float, double, FF_MODEL_FULL) }
            FF_DISPATCH_ADAM_Q(o.n_quad, float, float, FF_MODEL_FULL)
        }
        if (acc64) { FF_DISPATCH_ADAM_Q(o.n_quad, float, double, FF_MODEL_LOGNORMAL_2) }
        FF_DISPATCH_ADAM_Q(o.n_quad, float, float, FF_MODEL_LOGNORMAL_2)
    }
    if (o.n_quad != 32) return set_error(FF_EUNSUPPORTED, "FP64 supports quadrature order 32 only");
    if (model == FF_MODEL_LOGNORMAL_1) return launch_adam<double, double, FF_MODEL_LOGNORMAL_1, 32>(as);
    if (model == FF_MODEL_GAUSS_GRID_2) return launch_adam<double, double, FF_MODEL_GAUSS_GRID_2, 32>(as);
    if (model == FF_MODEL_ENDMEMBER_1) return launch_adam<double, double, FF_MODEL_ENDMEMBER_1, 32>(as);
    if (model == FF_MODEL_FULL) return launch_adam<double, double, FF_MODEL_FULL, 32>(as);
    return launch_adam<double, double, FF_MODEL_LOGNORMAL_2, 32>(as);
}

}  // namespace ff
