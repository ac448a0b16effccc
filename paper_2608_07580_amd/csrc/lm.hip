// Per-pixel Levenberg-Marquardt retrieval kernel and forward-model kernel.
//
// Work mapping: one lane owns one pixel for its whole solve.  Every round
// of the kernel's loop each lane runs one model evaluation (the initial
// point of a fresh pixel or the trial point of its current LM step), so the
// dominant work -- B x Q Planck evaluations per lane -- is executed by all
// lanes in lock-step with no cross-lane traffic; the damped step, tests and
// epilogue are per-lane FP64 scalar code.  In the persistent schedule a
// lane whose pixel has finished pulls the next pixel from a device queue
// (one wave-aggregated atomic per refill), so uneven convergence does not
// leave lanes idle until the queue drains.  A pixel whose solve from a
// per-pixel start fails is re-solved from the default start by the same
// lane at once, so the fallback overlaps the rest of the queue instead of
// forming a second, sparsely occupied launch.
//
// Loss, coordinates and solver (Keely et al. Sec. 2.5): r = m (L_obs - L(x(z))),
// F = r.r (eq. loss), z = 2 (x - lo)/(hi - lo) - 1 clipped to [-1, 1]
// (eq. affine).  The damped Gauss-Newton (Levenberg-Marquardt) iteration
// replaces the paper's Adam: (A + mu diag(d)) delta = -g on the free
// variables (a variable at a bound whose gradient points out of the box is
// held), z_t = clip(z + delta), gain-ratio acceptance and damping update.
// With an endmember surface the fractions' sum is kept by the step, a
// fraction at zero is held by the sign of its reduced gradient (or when the
// step would push it negative), and the step is shortened so that no
// fraction goes below zero.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "solve.hpp"

namespace ff {

constexpr int kMaxSolveTries = 64;

// Launch descriptor, kept in device memory (written by a one-thread fill
// kernel on the launch stream).  The kernel reads its fields through a
// laundered pointer where they are used, so loop-invariant values are
// re-fetched by scalar loads instead of occupying registers for the whole
// persistent loop.
template <typename R, int Q>
struct LmDesc {
    SceneDev sc[kMaxScenesPerLaunch];
    int n_scenes;
    int B;
    int64_t total;
    const int64_t* total_dev;      // if set: min(total, *total_dev) items (a device-side count)
    unsigned long long* queue;     // queue head
    int lpp;                       // lanes per pixel (power of two, <= 64)
    unsigned long long* evals;     // += model evaluations (may be null)
    int schedule;
    int max_iter;
    int warm_max_iter;             // cap of a solve from z0 (0: max_iter)
    int fallback;
    double xtol, ftol, gtol, kappa, tau;
    double ftol_undetected, f_detect;   // decrease test while the fire fraction is below f_detect
    double lo[FF_MAX_STATE], hi[FF_MAX_STATE], zdef[FF_MAX_STATE];
    int n_atm;                     // per-pixel atmospheres (with SceneDev::atm)
    const void* atm_tables[FF_MAX_ATMOSPHERES];
    const double* atm_tables64[FF_MAX_ATMOSPHERES];   // their FP64 tables
};

namespace {

// Projected-gradient test: max over free j of |g_j| / sqrt(A_jj F) <= gtol.
template <int N>
__device__ __forceinline__ bool gradient_small(const double (&z)[N], const double (&A)[N * (N + 1) / 2],
                                               const double (&g)[N], double F, double gtol)
{
    if (!(F > 0.0)) return true;
    bool small = true;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double gj = (double)g[j], ajj = (double)A[tri(j, j)];
        const bool act = ((double)z[j] <= -1.0 && gj > 0.0) || ((double)z[j] >= 1.0 && gj < 0.0);
        if (!act && ajj > 0.0 && fabs(gj) > gtol * sqrt(ajj * F)) small = false;
    }
    return small;
}

// Fractions of a simplex block held at zero (Karush-Kuhn-Tucker sign):
// fraction k at zero is held when its gradient exceeds the mean gradient of
// the fractions above zero, so moving weight onto it would raise the loss.
template <int N, int SF>
__device__ __forceinline__ void simplex_hold(const double (&z)[N], const double (&g)[N], bool (&act)[N])
{
    double gs = 0.0;
    int m = 0;
#pragma unroll
    for (int k = SF; k < SF + FF_N_ENDMEMBERS; ++k)
        if ((double)z[k] > -1.0) { gs += (double)g[k]; ++m; }
    const double gbar = m > 0 ? gs / m : 0.0;
#pragma unroll
    for (int k = SF; k < SF + FF_N_ENDMEMBERS; ++k) act[k] = (double)z[k] <= -1.0 && (double)g[k] - gbar > 0.0;
}

// The projected-gradient test with a simplex block: the free fractions'
// gradient less its mean over them.
template <int N, int SF>
__device__ __forceinline__ bool gradient_small_simplex(const double (&z)[N], const double (&A)[N * (N + 1) / 2],
                                                       const double (&g)[N], double F, double gtol)
{
    if (!(F > 0.0)) return true;
    bool act[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double gj = (double)g[j], zj = (double)z[j];
        act[j] = (zj <= -1.0 && gj > 0.0) || (zj >= 1.0 && gj < 0.0);
    }
    simplex_hold<N, SF>(z, g, act);
    double gs = 0.0;
    int m = 0;
#pragma unroll
    for (int k = SF; k < SF + FF_N_ENDMEMBERS; ++k)
        if (!act[k]) { gs += (double)g[k]; ++m; }
    const double gm = m > 0 ? gs / m : 0.0;
    bool small = true;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double gr = (j >= SF && j < SF + FF_N_ENDMEMBERS) ? (double)g[j] - gm : (double)g[j];
        const double ajj = (double)A[tri(j, j)];
        if (!act[j] && ajj > 0.0 && fabs(gr) > gtol * sqrt(ajj * F)) small = false;
    }
    return small;
}

template <int MODEL, int N>
__device__ __forceinline__ bool converged_gradient(const double (&z)[N], const double (&A)[N * (N + 1) / 2], const double (&g)[N],
                                                   double F, double gtol)
{
    if constexpr (simplex_first_v<MODEL> >= 0) return gradient_small_simplex<N, simplex_first_v<MODEL>>(z, A, g, F, gtol);
    else return gradient_small<N>(z, A, g, F, gtol);
}

// Occupancy target (second launch bound, waves per SIMD), FP32 kernels: the
// one-component model runs three waves per SIMD (at most 168 VGPRs) and the
// two-lognormal, endmember and Gaussian-grid models two (256 registers); the
// band loop stays free of spills and some per-pixel state outside it goes to
// scratch.  The full model (grid thermal term over the endmember surface) is
// faster at the compiler's one wave (measured: two waves spill its band
// loop), and so is FP64.
template <typename R, typename ACC, int MODEL, int Q>
__global__ void __launch_bounds__(256, sizeof(R) != 4 ? 1
                                       : MODEL == FF_MODEL_LOGNORMAL_1 ? 3
                                       : (MODEL == FF_MODEL_LOGNORMAL_2 || MODEL == FF_MODEL_ENDMEMBER_1
                                          || MODEL == FF_MODEL_GAUSS_GRID_2) ? 2 : 1)
lm_kernel(const LmDesc<R, Q>* __restrict__ descp)
{
    using PM = PixelModel<R, MODEL, Q>;
    constexpr int N = PM::N;
    constexpr int NT = N * (N + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int L = launder(descp)->lpp;        // lanes per pixel
    const int sub = lane & (L - 1);           // this lane's index in its group
    const bool head = sub == 0;               // the group's writer

    // ---- per-lane pixel state (identical on the L lanes of a group) ----
    bool has = false, exhausted = false, warm = false, static_taken = false;
    bool szero = false;         // the pixel's table has S = 0 on every band
    bool fbmode = false;        // re-solving a failed warm start from the default start
    int it_prev = 0;            // iterations of the failed warm-started solve
    float rrr_prev = 0.f;       // its relative residual
    int64_t item = -1, pix = 0;
    int sidx = 0;
    const float* rad = nullptr;
    const R* tab = nullptr;
    const double* tab64 = nullptr;
    double lnorm2 = 0.0, amax = 1.0;
    int nvalid = 0;
    constexpr int SF = simplex_first_v<MODEL>;
    // z and the trial point in FP64 in every kernel: near a bound an FP32 z
    // resolves f only to ~1.5e-8 (z spacing 6e-8 near -1), coarser than the
    // steps of a solve creeping along the f -> 0 valley of a background pixel
    double z[N], zt[N];
    double A[NT], g[N], d[N];
    bool cut = false;           // the last step was shortened by the simplex (no convergence test on it)
    double F = 0.0;
    double mu = 0.0, nu = 2.0, pred = 0.0;
    int it = 0, phase = 0;
    unsigned st = 0;
    unsigned long long nevals = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) { z[j] = zt[j] = g[j] = d[j] = 0.0; }
#pragma unroll
    for (int j = 0; j < NT; ++j) A[j] = (R)0;

    int64_t total = launder(descp)->total;
    if (const int64_t* td = launder(descp)->total_dev) total = min(total, *td);
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;

    for (;;) {
        // ------------------------------------------------------------ refill
        for (;;) {
            const LmDesc<R, Q>* D = launder(descp);
            const bool is_static = D->schedule == FF_SCHEDULE_STATIC;
            const bool need = !has && !exhausted;
            int64_t my = -1;
            if (is_static) {
                if (need) {
                    if (!static_taken) { my = gtid / L; static_taken = true; }
                    else exhausted = true;
                }
            } else {
                // one queue slot per group that needs a pixel: the group heads
                // take consecutive slots with one atomic per wave, then each
                // head hands its slot to the rest of its group
                if (__ballot(need) == 0ull) break;
                const unsigned long long mask = __ballot(need && head);
                const int cnt = __popcll(mask);
                const int leader = __ffsll((long long)mask) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(D->queue, (unsigned long long)cnt);
                const unsigned lo32 = __builtin_amdgcn_readlane((unsigned)(base & 0xffffffffull), leader);
                const unsigned hi32 = __builtin_amdgcn_readlane((unsigned)(base >> 32), leader);
                base = ((unsigned long long)hi32 << 32) | lo32;
                const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
                const unsigned long long mine = base + below;
                const int src = lane - sub;
                const unsigned mlo = (unsigned)__shfl((int)(unsigned)(mine & 0xffffffffull), src);
                const unsigned mhi = (unsigned)__shfl((int)(unsigned)(mine >> 32), src);
                if (need) my = (int64_t)(((unsigned long long)mhi << 32) | mlo);
            }
            if (need && my >= 0) {
                if (my >= total) {
                    exhausted = true;
                } else {
                    item = my;
                    sidx = scene_of(D, item);
                    const SceneDev& sd = D->sc[sidx];
                    pix = item - sd.offset;
                    if (sd.index) pix = sd.index[pix];
                }
                if (need && my >= 0 && my < total && pix >= 0 && pix < D->sc[sidx].P) {
                    const SceneDev& sd = D->sc[sidx];
                    const int B = D->B;
                    rad = sd.radiance + pix * B;
                    tab = reinterpret_cast<const R*>(sd.table);
                    tab64 = sd.table64;
                    szero = sd.s_zero != 0 && !sd.atm;
                    bool atm_ok = true;
                    if (sd.atm) {
                        const int a = sd.atm[pix];
                        atm_ok = a >= 0 && a < D->n_atm;
                        tab = atm_ok ? reinterpret_cast<const R*>(D->atm_tables[a]) : nullptr;
                        tab64 = atm_ok ? D->atm_tables64[a] : nullptr;
                    }
                    int nonfin = 0;
                    nvalid = 0;
                    lnorm2 = 0.0;
                    if (atm_ok) scan_pixel<R>(rad, tab, B, sub, L, nonfin, nvalid, lnorm2);
                    const bool fin = nonfin == 0;
                    it = 0;
                    phase = 0;
                    st = 0;
                    warm = false;
                    fbmode = false;
                    if (!atm_ok || !fin || nvalid <= N) {
                        if (head) {
                            const OutPtrs o = out_ptrs(sd);
                            write_nan<N>(o, pix);
                            if (o.rrr) o.rrr[pix] = __builtin_nanf("");
                            if (o.iters) o.iters[pix] = 0;
                            if (o.status)
                                o.status[pix] = !atm_ok ? FF_ST_BAD_ATMOSPHERE
                                                        : (!fin ? FF_ST_NONFINITE_INPUT : FF_ST_NO_DOF);
                        }
                    } else {
                        const float* z0 = sd.z0;
                        // a start row whose first entry is NaN carries no start:
                        // the pixel is solved from x0 as without z0
                        warm = z0 != nullptr && !isnan(z0[pix * N]);
#pragma unroll
                        for (int j = 0; j < N; ++j) {
                            double zz = warm ? (double)z0[pix * N + j] : D->zdef[j];
                            zz = isfinite(zz) ? zz : D->zdef[j];
                            z[j] = fmin(1.0, fmax(-1.0, zz));
                        }
                        project_block<MODEL>(z);
                        if (warm) st |= FF_ST_WARM_START;
                        has = true;
                    }
                }
            }
            if (is_static) break;
        }
        if (__ballot(has) == 0ull) break;
        if (has) {
            // ---------------------------------------------- one evaluation
            double xe[N];
            {
                const LmDesc<R, Q>* D = launder(descp);
#pragma unroll
                for (int j = 0; j < N; ++j)
                    xe[j] = D->lo[j] + 0.5 * (D->hi[j] - D->lo[j]) * ((double)(phase == 0 ? z[j] : zt[j]) + 1.0);
            }
            double At[NT], gt[N];
            // FP32 kernels drop the saturation mask when no pixel of the wave
            // has a saturated band, and the one-component kernel the
            // 1/(1 - S rho) factor when every pixel's table has S = 0 (the
            // common cases; the sums are the same either way)
            double Fe;
            if constexpr (sizeof(R) == 4) {
                const bool masked = __ballot(nvalid < launder(descp)->B) != 0ull;
                bool s0 = false;
                if constexpr (MODEL == FF_MODEL_LOGNORMAL_1) s0 = !masked && __ballot(!szero) == 0ull;
                if constexpr (MODEL == FF_MODEL_LOGNORMAL_1) {
                    if (s0) Fe = evaluate<R, ACC, MODEL, Q, false, true>(descp, rad, tab, tab64, xe, At, gt, sub, L);
                    else if (masked) Fe = evaluate<R, ACC, MODEL, Q, true>(descp, rad, tab, tab64, xe, At, gt, sub, L);
                    else Fe = evaluate<R, ACC, MODEL, Q, false>(descp, rad, tab, tab64, xe, At, gt, sub, L);
                } else {
                    Fe = masked ? evaluate<R, ACC, MODEL, Q, true>(descp, rad, tab, tab64, xe, At, gt, sub, L)
                                : evaluate<R, ACC, MODEL, Q, false>(descp, rad, tab, tab64, xe, At, gt, sub, L);
                }
            } else {
                Fe = evaluate<R, ACC, MODEL, Q>(descp, rad, tab, tab64, xe, At, gt, sub, L);
            }
            nevals += head ? 1 : 0;

            // -------------------------------------------- LM bookkeeping
            const LmDesc<R, Q>* D = launder(descp);
            bool done = false, need_step = false;
            if (phase == 0) {
                F = Fe;
#pragma unroll
                for (int j = 0; j < NT; ++j) A[j] = At[j];
#pragma unroll
                for (int j = 0; j < N; ++j) g[j] = gt[j];
                if (!isfinite(Fe)) {
                    st |= FF_ST_NONFINITE_INPUT;
                    done = true;
                } else if (converged_gradient<MODEL>(z, A, g, F, D->gtol)) {
                    st |= FF_ST_CONVERGED_GTOL;
                    done = true;
                } else {
                    amax = 0.0;
#pragma unroll
                    for (int j = 0; j < N; ++j) amax = fmax(amax, (double)A[tri(j, j)]);
                    if (!(amax > 0.0)) amax = 1.0;
#pragma unroll
                    for (int j = 0; j < N; ++j) d[j] = fmax(A[tri(j, j)], 1e-12 * amax);
                    mu = D->tau * amax;
                    nu = 2.0;
                    phase = 1;
                    need_step = true;
                }
            } else {
                ++it;
                const double rho = (F - Fe) / pred;
                if (isfinite(Fe) && (rho > 0.0 || pred <= D->kappa * F)) {
                    const double fold = F;
#pragma unroll
                    for (int j = 0; j < N; ++j) { z[j] = zt[j]; g[j] = gt[j]; }
#pragma unroll
                    for (int j = 0; j < NT; ++j) A[j] = At[j];
                    F = Fe;
                    const double rc = fmin(fmax(rho, 0.0), 1.0);
                    const double t = 2.0 * rc - 1.0;
                    mu *= fmax(1.0 / 3.0, 1.0 - t * t * t);
                    nu = 2.0;
#pragma unroll
                    for (int j = 0; j < N; ++j) d[j] = fmax(d[j], A[tri(j, j)]);
                    // the decrease test; below the detection level of the fire
                    // fraction the thermal variables are not identified and the
                    // loss is a noise valley: the tolerance is the FP32 cost's
                    const double xf = D->lo[0] + 0.5 * (D->hi[0] - D->lo[0]) * (z[0] + 1.0);
                    const double ft = xf < D->f_detect ? D->ftol_undetected : D->ftol;
                    if (pred <= ft * fold && (SF < 0 || !cut)) {
                        st |= FF_ST_CONVERGED_FTOL;
                        done = true;
                    } else if (converged_gradient<MODEL>(z, A, g, F, D->gtol)) {
                        st |= FF_ST_CONVERGED_GTOL;
                        done = true;
                    }
                } else {
                    mu *= nu;
                    nu *= 2.0;
                }
                need_step = !done;
            }

            // ------------------------------------------- next damped step
            if (need_step) {
                const int cap = (warm && D->warm_max_iter > 0) ? D->warm_max_iter : D->max_iter;
                if (it >= cap) {
                    st |= FF_ST_MAX_ITER;
                    done = true;
                } else {
                    const double xtol = D->xtol;
                    int tries = 0;
                    for (;;) {
                        // keep the FP64 widening of the stored state inside the retry
                        // loop (hoisting it would hold ~2x the state in registers)
#pragma unroll
                        for (int j = 0; j < NT; ++j) asm volatile("" : "+v"(A[j]));
#pragma unroll
                        for (int j = 0; j < N; ++j) asm volatile("" : "+v"(g[j]), "+v"(z[j]), "+v"(d[j]));
                        if (++tries > kMaxSolveTries || mu > 1e30 * amax) {
                            st |= FF_ST_DAMPING_OVERFLOW;
                            done = true;
                            break;
                        }
                        bool act[N];
                        double m[NT], rhs[N], delta[N];
                        double hstep[N], hmax = 0.0;
                        if constexpr (SF < 0) {
#pragma unroll
                        for (int j = 0; j < N; ++j) {
                            const double gj = (double)g[j], zj = (double)z[j];
                            act[j] = (zj <= -1.0 && gj > 0.0) || (zj >= 1.0 && gj < 0.0);
                            rhs[j] = act[j] ? 0.0 : -gj;
                        }
#pragma unroll
                        for (int i = 0; i < N; ++i) {
#pragma unroll
                            for (int k = 0; k < i; ++k)
                                m[tri(i, k)] = (act[i] || act[k]) ? 0.0 : (double)A[tri(i, k)];
                            m[tri(i, i)] = act[i] ? 1.0 : (double)A[tri(i, i)] + mu * (double)d[i];
                        }
                        if (!cholesky_packed<N>(m)) {
                            mu *= nu;
                            nu *= 2.0;
                            continue;
                        }
                        cholesky_solve<N>(m, rhs, delta);
#pragma unroll
                        for (int j = 0; j < N; ++j) {
                            const double zz = fmin(1.0, fmax(-1.0, (double)z[j] + delta[j]));
                            zt[j] = zz;
                            hstep[j] = (double)zz - (double)z[j];
                            hmax = fmax(hmax, fabs(hstep[j]));
                        }
                        if (hmax <= xtol) {
                            st |= FF_ST_CONVERGED_XTOL;
                            done = true;
                            break;
                        }
                        } else {
                        // Simplex block: the damped step on the free variables
                        // keeps the free fractions' sum (delta -= nu' M^-1 c, c
                        // the free fractions' indicator, nu' = c.delta / c.M^-1
                        // c); a fraction at zero the step would push below
                        // zero is held and the step solved again; the step is
                        // then shortened (ratio test) so no fraction goes
                        // negative, the stopping fraction set to exactly zero
                        // (no projection: shifting every fraction by the
                        // rounding of the sum would lift zeros off zero).
#pragma unroll
                        for (int j = 0; j < N; ++j) {
                            const double gj = (double)g[j], zj = (double)z[j];
                            act[j] = (zj <= -1.0 && gj > 0.0) || (zj >= 1.0 && gj < 0.0);
                        }
                        simplex_hold<N, SF>(z, g, act);
                        bool factored = true;
#pragma unroll 1
                        for (int pass = 0; pass <= FF_N_ENDMEMBERS; ++pass) {
#pragma unroll
                            for (int j = 0; j < N; ++j) rhs[j] = act[j] ? 0.0 : -(double)g[j];
#pragma unroll
                            for (int i = 0; i < N; ++i) {
#pragma unroll
                                for (int k = 0; k < i; ++k)
                                    m[tri(i, k)] = (act[i] || act[k]) ? 0.0 : (double)A[tri(i, k)];
                                m[tri(i, i)] = act[i] ? 1.0 : (double)A[tri(i, i)] + mu * (double)d[i];
                            }
                            if (!cholesky_packed<N>(m)) {
                                factored = false;
                                break;
                            }
                            cholesky_solve<N>(m, rhs, delta);
                            double c[N], y[N], cd = 0.0, cy = 0.0;
#pragma unroll
                            for (int j = 0; j < N; ++j) c[j] = (j >= SF && j < SF + FF_N_ENDMEMBERS && !act[j]) ? 1.0 : 0.0;
                            cholesky_solve<N>(m, c, y);
#pragma unroll
                            for (int j = 0; j < N; ++j) {
                                cd += c[j] * delta[j];
                                cy += c[j] * y[j];
                            }
                            if (cy > 0.0) {
#pragma unroll
                                for (int j = 0; j < N; ++j) delta[j] -= cd / cy * y[j];
                            }
                            bool more = false;
#pragma unroll
                            for (int k = SF; k < SF + FF_N_ENDMEMBERS; ++k)
                                if (!act[k] && (double)z[k] <= -1.0 && delta[k] < 0.0) {
                                    act[k] = true;
                                    more = true;
                                }
                            if (!more) break;
                        }
                        if (!factored) {
                            mu *= nu;
                            nu *= 2.0;
                            continue;
                        }
                        double a = 1.0;
                        int stop = -1;
#pragma unroll
                        for (int k = SF; k < SF + FF_N_ENDMEMBERS; ++k) {
                            const double x = 0.5 * ((double)z[k] + 1.0), dx = 0.5 * delta[k];
                            if (dx < 0.0 && x + dx < 0.0 && x / -dx < a) {
                                a = x / -dx;
                                stop = k;
                            }
                        }
#pragma unroll
                        for (int j = 0; j < N; ++j) zt[j] = fmin(1.0, fmax(-1.0, (double)z[j] + a * delta[j]));
#pragma unroll
                        for (int k = SF; k < SF + FF_N_ENDMEMBERS; ++k)
                            if (k == stop) zt[k] = -1.0;
                        cut = stop >= 0;
#pragma unroll
                        for (int j = 0; j < N; ++j) {
                            hstep[j] = (double)zt[j] - (double)z[j];
                            hmax = fmax(hmax, fabs(hstep[j]));
                        }
                        if (hmax <= xtol && !cut) {
                            st |= FF_ST_CONVERGED_XTOL;
                            done = true;
                            break;
                        }
                        }
                        double hg = 0.0, hah = 0.0;
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            hg += hstep[i] * (double)g[i];
                            double row = 0.0;
#pragma unroll
                            for (int k = 0; k < N; ++k) row += (double)A[tri(i, k)] * hstep[k];
                            hah += hstep[i] * row;
                        }
                        pred = -(2.0 * hg + hah);
                        if (pred > 0.0) break;
                        mu *= nu;
                        nu *= 2.0;
                    }
                }
            }

            if (done) {
                // --------------------------------------------------- epilogue
                has = false;
                const OutPtrs o = out_ptrs(D->sc[sidx]);
                const bool valid = !(st & FF_ST_NONFINITE_INPUT);
                double x[N];
                bool bound = false;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    x[j] = D->lo[j] + 0.5 * (D->hi[j] - D->lo[j]) * ((double)z[j] + 1.0);
                    bound = bound || (double)z[j] <= -1.0 || (double)z[j] >= 1.0;
                }
                if (valid && bound) st |= FF_ST_AT_BOUND;
                const double rrr_new = valid && lnorm2 > 0.0 ? sqrt(F / lnorm2) : __builtin_nan("");
                int it_out = it;
                bool write = true, restart = false;
                if (fbmode) {
                    // fallback from the default start: kept if it converged or fits better
                    write = (st & FF_ST_CONVERGED) != 0 || !(rrr_new >= (double)rrr_prev);
                    it_out = it_prev + 1 + it;
                    if (write) st |= FF_ST_USED_FALLBACK | FF_ST_WARM_START;
                    else if (o.iters && head) o.iters[pix] = it_out;
                } else if (warm && D->fallback && !(st & FF_ST_CONVERGED)) {
                    // the warm-started result is written now and the same lane
                    // re-solves the pixel from the default start right away
                    restart = true;
                }
                if (write) {
                    // the group's lanes share the covariance's column solves
                    if (valid) st |= write_solution<R, MODEL, Q>(D, o, pix, x, A, F, nvalid, sub, L);
                    else if (head) write_nan<N>(o, pix);
                    if (head) {
                        if (o.rrr) o.rrr[pix] = (float)rrr_new;
                        if (o.iters) o.iters[pix] = it_out;
                        if (o.status) o.status[pix] = st;
                    }
                }
                if (restart) {
                    has = true;
                    fbmode = true;
                    warm = false;
                    it_prev = it;
                    rrr_prev = (float)rrr_new;
                    it = 0;
                    phase = 0;
                    st = 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) z[j] = fmin(1.0, fmax(-1.0, D->zdef[j]));
                    project_block<MODEL>(z);
                }
            }
        }
    }

    // one atomic per wave for the evaluation count
    unsigned long long* evals = launder(descp)->evals;
    if (evals) wave_add(evals, nevals);
}

// Forward model and dL/dx at P states, one lane per pixel.
template <typename R, int MODEL, int Q>
__global__ void __launch_bounds__(256)
forward_kernel(const R* __restrict__ tab, int B, const R* __restrict__ state, int64_t P,
               R* __restrict__ L, R* __restrict__ J)
{
    using PM = PixelModel<R, MODEL, Q>;
    constexpr int N = PM::N;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = (double)state[p * N + j];
    PM pm;
    pm.setup(x);
    double c1[N], c2[N];
    PM::coefficients(x, c1, c2);
    for (int b = 0; b < B; ++b) {
        const BandRow<R> row = load_row(tab + (size_t)b * FF_TABLE_COLS);
        R ub[N];
        const R lm = band_of<MODEL>(pm, tab, B, b, opaque_zero(), row, ub);
        L[p * B + b] = lm;
        if (J) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double v = c1[i] * (double)ub[PM::s1[i]];
                if (PM::s2[i] >= 0) v += c2[i] * (double)ub[PM::s2[i]];
                J[(p * B + b) * N + i] = (R)v;
            }
        }
    }
}

}  // namespace


template <typename R, typename ACC, int MODEL, int Q>
static ff_status launch_lm(const BatchSpec& bs)
{
    const ff_options& o = *bs.opts;
    const int block = o.block_size > 0 ? o.block_size : 256;
    const int lpp = o.lanes_per_pixel > 0 ? o.lanes_per_pixel : 1;
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    if (!ensure_tables<R, MODEL, Q>(dev)) return set_error(FF_EDEVICE, "quadrature rule could not be placed on the device");
    int n_cu = 0;
    FF_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    int occ = 0;
    FF_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, lm_kernel<R, ACC, MODEL, Q>, block, 0));
    if (occ < 1) occ = 1;
    const int per_cu = o.blocks_per_cu > 0 ? std::min(o.blocks_per_cu, occ) : occ;

    const int n_chunks = (bs.n_scenes + kMaxScenesPerLaunch - 1) / kMaxScenesPerLaunch;
    int64_t total = 0;
    bool any_warm = false;
    for (int s = 0; s < bs.n_scenes; ++s) {
        total += bs.P[s];
        if (bs.z0 && bs.z0[s] && bs.P[s] > 0) any_warm = true;
    }
    if (total == 0) return clear_error();
    const bool fallback = any_warm && o.fallback != 0;

    // the stream's scratch: per chunk one queue counter and one descriptor
    using Desc = LmDesc<R, Q>;
    const size_t desc_bytes = (sizeof(Desc) + 255) / 256 * 256;
    const size_t n_ctr = (size_t)n_chunks;
    const size_t ctr_bytes = (n_ctr * sizeof(unsigned long long) + 255) / 256 * 256;
    const size_t bytes = ctr_bytes + (size_t)n_chunks * desc_bytes;
    char* buf = nullptr;
    if (bs.fixed_scratch) {
        if (bytes > bs.fixed_bytes)
            return set_error(FF_EINVAL, "retrieval needs " + std::to_string(bytes) + " bytes of scratch, the fixed array holds " +
                                            std::to_string(bs.fixed_bytes));
        buf = static_cast<char*>(bs.fixed_scratch);
    } else {
        const ff_status st = stream_scratch(bs.stream, bytes, reinterpret_cast<void**>(&buf));
        if (st != FF_OK) return st;
    }
    auto* ctr = reinterpret_cast<unsigned long long*>(buf);
    char* descs = buf + ctr_bytes;
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)((n_ctr + 255) / 256)), dim3(256), 0, bs.stream, ctr, (int)n_ctr);
    hipError_t e = hipGetLastError();

    for (int c = 0; c < n_chunks && e == hipSuccess; ++c) {
        Desc prm{};
        int64_t off = 0;
        int ns = 0;
        for (int s = c * kMaxScenesPerLaunch; s < std::min(bs.n_scenes, (c + 1) * kMaxScenesPerLaunch); ++s, ++ns) {
            SceneDev& d = prm.sc[ns];
            const ff_outputs& out = bs.outs[s];
            d.radiance = bs.radiance[s];
            d.table = sizeof(R) == 4 ? (const void*)bs.scenes[s]->table_f32 : (const void*)bs.scenes[s]->table_f64;
            d.table64 = bs.scenes[s]->table_f64;
            d.P = bs.P[s];
            d.offset = off;
            d.index = bs.index;
            d.atm = bs.atm_index;
            d.z0 = bs.z0 ? bs.z0[s] : nullptr;
            d.state = out.state;
            d.cov = out.cov_packed;
            d.moments = out.moments;
            d.rrr = out.rrr;
            d.iters = out.iters;
            d.status = out.status;
            d.state64 = out.state_f64;
            d.s_zero = bs.scenes[s]->s_zero ? 1 : 0;
            off += bs.P[s];
        }
        for (int s = ns; s < kMaxScenesPerLaunch; ++s) prm.sc[s].offset = INT64_MAX;
        if (off == 0) continue;
        prm.n_scenes = ns;
        prm.B = bs.scenes[0]->n_bands;
        prm.total = off;
        prm.total_dev = bs.count_dev;
        prm.n_atm = bs.atm_index ? bs.n_atm : 0;
        for (int a = 0; a < prm.n_atm; ++a) {
            prm.atm_tables[a] = sizeof(R) == 4 ? (const void*)bs.atms[a]->table_f32 : (const void*)bs.atms[a]->table_f64;
            prm.atm_tables64[a] = bs.atms[a]->table_f64;
        }
        prm.evals = bs.evals;
        prm.max_iter = o.max_iter;
        prm.warm_max_iter = o.warm_max_iter;
        prm.fallback = fallback ? 1 : 0;
        prm.xtol = o.xtol;
        prm.ftol = o.ftol;
        prm.gtol = o.gtol;
        prm.kappa = o.kappa;
        prm.tau = o.tau;
        prm.ftol_undetected = o.ftol_undetected;
        prm.f_detect = o.f_detect;
        const int n = ModelDims<MODEL>::N;
        for (int j = 0; j < FF_MAX_STATE; ++j) {
            prm.lo[j] = j < n ? bs.prior->lo[j] : 0.0;
            prm.hi[j] = j < n ? bs.prior->hi[j] : 1.0;
            prm.zdef[j] = j < n ? 2.0 * (bs.prior->x0[j] - bs.prior->lo[j]) / (bs.prior->hi[j] - bs.prior->lo[j]) - 1.0 : 0.0;
        }
        const int64_t grid_static = (off * lpp + block - 1) / block;
        const int64_t grid_pers = std::min<int64_t>((int64_t)n_cu * per_cu, grid_static);
        prm.queue = ctr + c;
        prm.lpp = lpp;
        prm.schedule = o.schedule;
        const int64_t grid = o.schedule == FF_SCHEDULE_STATIC ? grid_static : grid_pers;
        if (grid > 0x7fffffff) {
            e = hipErrorInvalidValue;
            break;
        }
        Desc* dptr = reinterpret_cast<Desc*>(descs + (size_t)c * desc_bytes);
        hipLaunchKernelGGL(fill_struct<Desc>, dim3(1), dim3(64), 0, bs.stream, prm, dptr);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL((lm_kernel<R, ACC, MODEL, Q>), dim3((unsigned)grid), dim3(block), 0, bs.stream,
                           (const Desc*)dptr);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_error(e, "lm_kernel launch");
    return clear_error();
}

template <typename R, int MODEL, int Q>
static ff_status launch_forward(const ff_scene* sc, const void* state, int64_t P, void* L, void* J,
                                hipStream_t stream)
{
    if (P == 0) return clear_error();
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    if (!ensure_tables<R, MODEL, Q>(dev)) return set_error(FF_EDEVICE, "quadrature rule could not be placed on the device");
    const int block = 256;
    const int64_t grid = (P + block - 1) / block;
    if (grid > 0x7fffffff) return set_error(FF_EINVAL, "ff_forward: P too large");
    const R* tab = sizeof(R) == 4 ? (const R*)(const void*)sc->table_f32 : (const R*)(const void*)sc->table_f64;
    hipLaunchKernelGGL((forward_kernel<R, MODEL, Q>), dim3((unsigned)grid), dim3(block), 0, stream, tab,
                       sc->n_bands, (const R*)state, P, (R*)L, (R*)J);
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

// ------------------------------------------------ allocation-free scratch
// The queue counters and launch descriptors of ff_retrieve_batch_noalloc
// live in this fixed array (each device holds its own copy for the life of
// the process): one 256-byte block of counters, then one descriptor per
// launch of at most kMaxScenesPerLaunch scenes.  Host code never passes the
// array's name to a kernel: it looks the device address up once per device.
constexpr size_t kNoAllocScratchBytes = 16384;
static_assert(FF_NOALLOC_MAX_SCENES % kMaxScenesPerLaunch == 0, "whole launches");
static_assert(256 + (FF_NOALLOC_MAX_SCENES / kMaxScenesPerLaunch) * ((sizeof(LmDesc<double, 32>) + 255) / 256 * 256) <=
                  kNoAllocScratchBytes, "fixed scratch holds the descriptors of FF_NOALLOC_MAX_SCENES scenes");
static_assert(sizeof(LmDesc<double, 32>) == sizeof(LmDesc<float, 16>), "descriptor size independent of type and order");
static_assert((FF_NOALLOC_MAX_SCENES / kMaxScenesPerLaunch) * sizeof(unsigned long long) <= 256, "counters block");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

ff_status noalloc_scratch(void** ptr, size_t* bytes)
{
    static std::mutex mtx;
    static void* addr[64] = {};
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(FF_EUNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(mtx);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(FF_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoAllocScratchBytes;
    return FF_OK;
}

// ---------------------------------------------------------------- dispatch
#define FF_DISPATCH_Q(FN, q, ...)                                       \
    switch (q) {                                                    \
    case 16: return FN<__VA_ARGS__, 16>(bs);                        \
    case 24: return FN<__VA_ARGS__, 24>(bs);                        \
    case 32: return FN<__VA_ARGS__, 32>(bs);                        \
    default: return set_error(FF_EUNSUPPORTED, "unsupported quadrature order for FP32 (16, 24, 32)"); \
    }

ff_status dispatch_lm(int precision, int model, int q, const BatchSpec& bs)
{
    const bool acc64 = bs.opts->accumulate == FF_ACCUMULATE_FP64;
    if (precision == FF_PRECISION_FP32) {
        if (model == FF_MODEL_LOGNORMAL_1) {
            if (acc64) { FF_DISPATCH_Q(launch_lm, q, float, double, FF_MODEL_LOGNORMAL_1) }
            FF_DISPATCH_Q(launch_lm, q, float, float, FF_MODEL_LOGNORMAL_1)
        }
        if (model == FF_MODEL_GAUSS_GRID_2) {
            if (acc64) { FF_DISPATCH_Q(launch_lm, q, float, double, FF_MODEL_GAUSS_GRID_2) }
            FF_DISPATCH_Q(launch_lm, q, float, float, FF_MODEL_GAUSS_GRID_2)
        }
        if (model == FF_MODEL_ENDMEMBER_1) {
            if (acc64) { FF_DISPATCH_Q(launch_lm, q, float, double, FF_MODEL_ENDMEMBER_1) }
            FF_DISPATCH_Q(launch_lm, q, float, float, FF_MODEL_ENDMEMBER_1)
        }
        if (model == FF_MODEL_FULL) {
            if (acc64) { FF_DISPATCH_Q(launch_lm, q, float, double, FF_MODEL_FULL) }
            FF_DISPATCH_Q(launch_lm, q, float, float, FF_MODEL_FULL)
        }
        if (acc64) { FF_DISPATCH_Q(launch_lm, q, float, double, FF_MODEL_LOGNORMAL_2) }
        FF_DISPATCH_Q(launch_lm, q, float, float, FF_MODEL_LOGNORMAL_2)
    }
    if (q != 32) return set_error(FF_EUNSUPPORTED, "FP64 supports quadrature order 32 only");
    if (model == FF_MODEL_LOGNORMAL_1) return launch_lm<double, double, FF_MODEL_LOGNORMAL_1, 32>(bs);
    if (model == FF_MODEL_GAUSS_GRID_2) return launch_lm<double, double, FF_MODEL_GAUSS_GRID_2, 32>(bs);
    if (model == FF_MODEL_ENDMEMBER_1) return launch_lm<double, double, FF_MODEL_ENDMEMBER_1, 32>(bs);
    if (model == FF_MODEL_FULL) return launch_lm<double, double, FF_MODEL_FULL, 32>(bs);
    return launch_lm<double, double, FF_MODEL_LOGNORMAL_2, 32>(bs);
}

#define FF_DISPATCH_FWD(q, ...)                                      \
    switch (q) {                                                    \
    case 16: return launch_forward<__VA_ARGS__, 16>(sc, state, P, L, J, stream); \
    case 24: return launch_forward<__VA_ARGS__, 24>(sc, state, P, L, J, stream); \
    case 32: return launch_forward<__VA_ARGS__, 32>(sc, state, P, L, J, stream); \
    default: return set_error(FF_EUNSUPPORTED, "unsupported quadrature order for FP32 (16, 24, 32)"); \
    }

ff_status dispatch_forward(int precision, int model, int q, const ff_scene* sc, const void* state, int64_t P,
                           void* L, void* J, hipStream_t stream)
{
    if (precision == FF_PRECISION_FP32) {
        if (model == FF_MODEL_LOGNORMAL_1) { FF_DISPATCH_FWD(q, float, FF_MODEL_LOGNORMAL_1) }
        if (model == FF_MODEL_GAUSS_GRID_2) { FF_DISPATCH_FWD(q, float, FF_MODEL_GAUSS_GRID_2) }
        if (model == FF_MODEL_ENDMEMBER_1) { FF_DISPATCH_FWD(q, float, FF_MODEL_ENDMEMBER_1) }
        if (model == FF_MODEL_FULL) { FF_DISPATCH_FWD(q, float, FF_MODEL_FULL) }
        FF_DISPATCH_FWD(q, float, FF_MODEL_LOGNORMAL_2)
    }
    if (q != 32) return set_error(FF_EUNSUPPORTED, "FP64 supports quadrature order 32 only");
    if (model == FF_MODEL_LOGNORMAL_1) return launch_forward<double, FF_MODEL_LOGNORMAL_1, 32>(sc, state, P, L, J, stream);
    if (model == FF_MODEL_GAUSS_GRID_2) return launch_forward<double, FF_MODEL_GAUSS_GRID_2, 32>(sc, state, P, L, J, stream);
    if (model == FF_MODEL_ENDMEMBER_1) return launch_forward<double, FF_MODEL_ENDMEMBER_1, 32>(sc, state, P, L, J, stream);
    if (model == FF_MODEL_FULL) return launch_forward<double, FF_MODEL_FULL, 32>(sc, state, P, L, J, stream);
    return launch_forward<double, FF_MODEL_LOGNORMAL_2, 32>(sc, state, P, L, J, stream);
}

}  // namespace ff
