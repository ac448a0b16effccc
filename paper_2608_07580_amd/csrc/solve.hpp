// Per-pixel pieces shared by the retrieval kernels (Levenberg-Marquardt and
// staged Adam): launch-descriptor scene slots, group reductions over the
// lanes of a pixel, the model evaluation with the normal equations in z,
// FP64 Cholesky, the projection of surface fractions onto the unit simplex,
// and the output epilogue (Gauss-Newton covariance, moments).
//
// Loss and coordinates (Keely et al. Sec. 2.5): r = m (L_obs - L(x(z))),
// F = r.r (eq. loss), z = 2 (x - lo)/(hi - lo) - 1 (eq. affine).
#pragma once

#include "physics.hpp"

namespace ff {

constexpr int kMaxScenesPerLaunch = 16;

// One scene of a launch: inputs, per-pixel start, outputs, and the offset of
// its first pixel in the launch's pixel numbering.  With a row list, item i
// of the scene solves radiance row index[i] (rows outside [0, P) are
// skipped) and writes that row's outputs.  With a per-pixel atmosphere
// index, row p uses the launch's atmosphere table atm[p].
struct SceneDev {
    const float* radiance;
    const void* table;
    const double* table64;      // the scene's FP64 table (solar term of the residual)
    int64_t P;
    int64_t offset;
    const int64_t* index;
    const int32_t* atm;
    const float* z0;
    float* state;
    float* cov;
    float* moments;
    float* rrr;
    int32_t* iters;
    uint32_t* status;
    double* state64;
    int32_t s_zero;             // S = 0 on every band of the table (one scene table, no per-pixel atmospheres)
};

// Hide a pointer's value from the optimiser: loads through the result are
// not hoisted across this point (the pointer stays in SGPRs, no code).
template <typename T>
__device__ __forceinline__ const T* launder(const T* p)
{
#ifdef FF_LAUNDER
    asm volatile("" : "+s"(p));
#endif
    return p;
}

namespace {

// upper-triangle row-major index of (i, j), i <= j: the output packing
__device__ __forceinline__ int upper(int n, int i, int j) { return i * n - i * (i - 1) / 2 + (j - i); }

// scene slot of a launch-wide pixel number (slots past n_scenes have offset INT64_MAX)
template <typename Desc>
__device__ __forceinline__ int scene_of(const Desc* p, int64_t item)
{
    int s = 0;
    const int ns = p->n_scenes;
    for (int i = 1; i < ns; ++i)
        if (item >= p->sc[i].offset) s = i;
    return s;
}

// In-place Cholesky M = C C^T of a packed lower-triangular SPD matrix; the
// diagonal is stored as 1 / C_jj so the triangular solves only multiply.
// Returns false if a pivot is not strictly positive.
template <int N>
__device__ __forceinline__ bool cholesky_packed(double (&m)[N * (N + 1) / 2])
{
    bool ok = true;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double dj = m[tri(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= m[tri(j, k)] * m[tri(j, k)];
        ok = ok && dj > 0.0;
        const double dd = dj > 0.0 ? dj : 1.0;
        double inv = __builtin_amdgcn_rsq(dd);
        inv = inv * (1.5 - 0.5 * dd * inv * inv);   // one Newton step: full FP64 accuracy
        m[tri(j, j)] = inv;
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            double v = m[tri(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= m[tri(i, k)] * m[tri(j, k)];
            m[tri(i, j)] = v * inv;
        }
    }
    return ok;
}

// Solve C C^T x = rhs with the factor of cholesky_packed.
template <int N>
__device__ __forceinline__ void cholesky_solve(const double (&c)[N * (N + 1) / 2], const double (&rhs)[N],
                                               double (&x)[N])
{
    double y[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double v = rhs[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= c[tri(i, k)] * y[k];
        y[i] = v * c[tri(i, i)];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double v = y[i];
#pragma unroll
        for (int k = i + 1; k < N; ++k) v -= c[tri(k, i)] * x[k];
        x[i] = v * c[tri(i, i)];
    }
}

// Euclidean projection of v onto the unit simplex {x >= 0, sum x = 1}
// (sort-based, Duchi, Shalev-Shwartz, Singer & Chandra 2008): sort
// descending (a 9-comparator network, all indices fixed so v stays in
// registers), theta = (sum of the largest j values - 1)/j for the largest j
// with u_j > theta, x = max(v - theta, 0).
__device__ __forceinline__ void project_simplex5(double (&v)[5])
{
    double u[5] = {v[0], v[1], v[2], v[3], v[4]};
    auto cx = [&](int a, int b) {
        const double hi = fmax(u[a], u[b]), lo = fmin(u[a], u[b]);
        u[a] = hi;
        u[b] = lo;
    };
    cx(0, 1); cx(3, 4); cx(2, 4); cx(2, 3); cx(0, 3); cx(0, 2); cx(1, 4); cx(1, 3); cx(1, 2);
    double cum = 0.0, theta = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        cum += u[j];
        const double t = (cum - 1.0) / (double)(j + 1);
        if (u[j] - t > 0.0) theta = t;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) v[i] = v[i] - theta > 0.0 ? v[i] - theta : 0.0;
}

// The model's simplex block of z (fractions x = (z + 1)/2) projected onto
// the unit simplex (Sec. 2.5: the surface mixture after each step); no-op
// for models without one.
template <int MODEL, typename T, int N>
__device__ __forceinline__ void project_block(T (&z)[N])
{
    constexpr int SF = simplex_first_v<MODEL>;
    if constexpr (SF >= 0) {
        static_assert(FF_N_ENDMEMBERS == 5, "simplex block of five fractions");
        double x[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = 0.5 * ((double)z[SF + k] + 1.0);
        project_simplex5(x);
#pragma unroll
        for (int k = 0; k < 5; ++k) z[SF + k] = (T)(2.0 * x[k] - 1.0);
    }
}

// Sum over the L lanes of a pixel's group (aligned, L a power of two) by an
// xor butterfly: every lane of the group ends with the same bits, since each
// level adds the same two partial sums (a + b == b + a in IEEE arithmetic).
__device__ __forceinline__ float group_sum(float v, int L)
{
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double group_sum(double v, int L)
{
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ int group_sum(int v, int L)
{
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

// Radiance checks of a new pixel over the group's bands: count of
// non-finite values, count of unsaturated bands and their squared norm
// (identical on every lane of the group).
template <typename R>
__device__ __forceinline__ void scan_pixel(const float* __restrict__ rad, const R* __restrict__ tab, int B,
                                           int sub, int L, int& nonfin, int& nvalid, double& lnorm2)
{
    // Eight bands per lane per pass with all their loads issued first: a fresh
    // pixel's row is not in cache, and the wave (whose other lanes wait for
    // this scan) then waits for a few memory round trips instead of one per
    // band.  The sums keep the band order of a plain loop.
    constexpr int kBatch = 8;
    nonfin = 0;
    nvalid = 0;
    lnorm2 = 0.0;
    for (int b0 = sub; b0 < B; b0 += kBatch * L) {
        float v[kBatch];
        R ls[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int b = b0 + j * L;
            v[j] = b < B ? rad[b] : 0.f;
            ls[j] = b < B ? tab[(size_t)b * FF_TABLE_COLS + COL_LSAT] : (R)0;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            if (b0 + j * L >= B) break;
            nonfin += isfinite(v[j]) ? 0 : 1;
            if ((R)v[j] < ls[j]) {
                ++nvalid;
                lnorm2 += (double)v[j] * (double)v[j];
            }
        }
    }
    if (L > 1) {
        nonfin = group_sum(nonfin, L);
        nvalid = group_sum(nvalid, L);
        lnorm2 = group_sum(lnorm2, L);
    }
}

// One model evaluation at physical state x: basis Gram matrix G = sum_b u u^T,
// h = sum_b u r_b and F = sum_b r_b^2 over unmasked bands, then the normal
// equations in z: A = D M G M^T D, g = J^T r = -D M h (D = diag((hi-lo)/2)).
// The L lanes of a pixel's group take bands sub, sub + L, ... and their
// partial sums are combined across the group before the normal equations.
// Desc provides B and the box lo, hi.
//
// The residual r = L_obs - L_s - L_t and the loss F = sum r^2 are formed in
// FP64 in every kernel: the solar term L_s (eq. solar) from the FP64 table
// and the FP64 surface variables, the thermal term L_t = f tau_up I from the
// kernel's own (FP32 or FP64) quadrature sums.  In an FP32 kernel an FP32
// solar term would carry ~1e-7 L of rounding per band that changes from one
// evaluation to the next -- about 3e-5 of the noise sigma (L / 300) per
// residual and a few 1e-6 of F -- which the gain ratio and the stop tests
// cannot tell from progress on f = 0 background pixels.
//
// MASKED = false drops the saturation mask from the band loop; it is valid
// (and gives the same sums) only when every band of the pixel is below its
// saturation level, which the caller knows from scan_pixel (nvalid == B).
// S0 = true (one-component model) takes 1/(1 - S rho) as 1 without forming
// it; valid only for a table whose S is 0 on every band, where the general
// path's reciprocal is exactly 1 too, so the sums are the same.
template <typename R, typename ACC, int MODEL, int Q, bool MASKED = true, bool S0 = false, typename Desc>
__device__ __forceinline__ double evaluate(const Desc* descp, const float* __restrict__ rad,
                                      const R* __restrict__ tab, const double* __restrict__ tab64,
                                      const double (&x)[ModelDims<MODEL>::N],
                                      double (&A)[ModelDims<MODEL>::N * (ModelDims<MODEL>::N + 1) / 2],
                                      double (&g)[ModelDims<MODEL>::N], int sub, int L)
{
    using PM = PixelModel<R, MODEL, Q>;
    constexpr int N = PM::N;
    constexpr int NT = N * (N + 1) / 2;
    constexpr int NS = SurfaceDims<MODEL>::NS;
    const int B = launder(descp)->B;
    PM pm;
    pm.setup(x, sub, L);
    double sv[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) sv[k] = x[N - NS + k];
    ACC G[NT], h[N];
    double F = 0.0;
    // the FP64 solar term's 1/(1 - S rho) when S = 0: a 1 the compiler
    // cannot fold, so the term keeps the general path's FMA and rounding
    double one = 1.0;
    if constexpr (S0) asm volatile("" : "+v"(one));
#pragma unroll
    for (int i = 0; i < NT; ++i) G[i] = (ACC)0;
#pragma unroll
    for (int i = 0; i < N; ++i) h[i] = (ACC)0;

    for (int b0 = sub; b0 < B; b0 += 4 * L) {
        // four radiance values per lane per load group (bands b0 + jL): with
        // one lane per pixel they share a cache line, with L lanes the group
        // reads L consecutive values per load
        float l0 = rad[b0];
        float l1 = b0 + L < B ? rad[b0 + L] : 0.f;
        float l2 = b0 + 2 * L < B ? rad[b0 + 2 * L] : 0.f;
        float l3 = b0 + 3 * L < B ? rad[b0 + 3 * L] : 0.f;
#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + j * L;
            if (b >= B) break;
            const float lob = l0;
            l0 = l1;
            l1 = l2;
            l2 = l3;
            // quadrature weights are re-read (scalar loads) every band
            const int o = opaque_zero();
            const BandRow<R> row = load_row(tab + (size_t)b * FF_TABLE_COLS);
            R ub[N];
            const R lm = band_of<MODEL, S0>(pm, tab, B, b, o, row, ub);
            const bool msk = !MASKED || (R)lob < row.lsat;
            double r64;
            if constexpr (sizeof(R) == 8) {
                r64 = (double)lob - (double)lm;
                (void)tab64;
            } else {
                (void)lm;
                const R lt = pm.f * ub[0];
                r64 = ((double)lob - solar_fp64<MODEL, S0>(tab64, B, b, sv, one)) - (double)lt;
            }
            r64 = msk ? r64 : 0.0;
            const ACC r = (ACC)r64;
            ACC ua[N];
#pragma unroll
            for (int i = 0; i < N; ++i) ua[i] = msk ? (ACC)ub[i] : (ACC)0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                h[i] += ua[i] * r;
#pragma unroll
                for (int k = 0; k <= i; ++k) G[tri(i, k)] += ua[i] * ua[k];
            }
            F = fma(r64, r64, F);
        }
    }
    if (L > 1) {
#pragma unroll
        for (int i = 0; i < NT; ++i) G[i] = group_sum(G[i], L);
#pragma unroll
        for (int i = 0; i < N; ++i) h[i] = group_sum(h[i], L);
        F = group_sum(F, L);
    }

    const Desc* D = launder(descp);
    double c1[N], c2[N];
    PM::coefficients(x, c1, c2);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double dzi = 0.5 * (D->hi[i] - D->lo[i]);
        const int a1 = PM::s1[i], a2 = PM::s2[i];
        double gi = c1[i] * (double)h[a1];
        if (a2 >= 0) gi += c2[i] * (double)h[a2];
        g[i] = -dzi * gi;
#pragma unroll
        for (int k = 0; k <= i; ++k) {
            const double dzk = 0.5 * (D->hi[k] - D->lo[k]);
            const int b1 = PM::s1[k], b2 = PM::s2[k];
            double v = c1[i] * c1[k] * (double)G[tri(a1, b1)];
            if (b2 >= 0) v += c1[i] * c2[k] * (double)G[tri(a1, b2)];
            if (a2 >= 0) v += c2[i] * c1[k] * (double)G[tri(a2, b1)];
            if (a2 >= 0 && b2 >= 0) v += c2[i] * c2[k] * (double)G[tri(a2, b2)];
            A[tri(i, k)] = dzi * dzk * v;
        }
    }
    return F;
}

// Outputs of one pixel (all pointers may be null).
struct OutPtrs {
    float* state;
    float* cov;
    float* moments;
    float* rrr;
    int32_t* iters;
    uint32_t* status;
    double* state64;
};

__device__ __forceinline__ OutPtrs out_ptrs(const SceneDev& d)
{
    return OutPtrs{d.state, d.cov, d.moments, d.rrr, d.iters, d.status, d.state64};
}

template <int N>
__device__ inline void write_nan(const OutPtrs& o, int64_t pix)
{
    constexpr int NT = N * (N + 1) / 2;
    const float qn = __builtin_nanf("");
    if (o.state) for (int j = 0; j < N; ++j) o.state[pix * N + j] = qn;
    if (o.state64) for (int j = 0; j < N; ++j) o.state64[pix * N + j] = __builtin_nan("");
    if (o.cov) for (int j = 0; j < NT; ++j) o.cov[pix * NT + j] = qn;
    if (o.moments) { o.moments[2 * pix] = qn; o.moments[2 * pix + 1] = qn; }
}

// State, covariance and moments of a solved pixel at physical state x with
// J^T J = A (in z) and loss F over nvalid bands.  The Gauss-Newton
// covariance sigma^2 A^-1 (sigma^2 = F / (N_valid - n)) is formed in z and
// scaled to x; variables whose Jacobian column is identically zero are
// unidentified and get NaN rows/columns.  Returns FF_ST_COV_SINGULAR when
// some rows are NaN, else 0.  The L lanes of a pixel's group (sub = this
// lane, all holding the same x, A, F) share the covariance: a lane solves and
// writes columns sub, sub + L, ...; lane 0 writes state and moments.
template <typename R, int MODEL, int Q, typename Desc>
__device__ __forceinline__ unsigned write_solution(const Desc* D, const OutPtrs& o, int64_t pix,
                                                   const double (&x)[ModelDims<MODEL>::N],
                                                   const double (&A)[ModelDims<MODEL>::N * (ModelDims<MODEL>::N + 1) / 2],
                                                   double F, int nvalid, int sub = 0, int L = 1)
{
    using PM = PixelModel<R, MODEL, Q>;
    constexpr int N = PM::N;
    constexpr int NT = N * (N + 1) / 2;
    unsigned st = 0;
    bool keep[N];
    double cm[NT];
    bool any_drop = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        keep[i] = (double)A[tri(i, i)] > 0.0;
        any_drop = any_drop || !keep[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < i; ++k)
            cm[tri(i, k)] = (keep[i] && keep[k]) ? (double)A[tri(i, k)] : 0.0;
        cm[tri(i, i)] = keep[i] ? (double)A[tri(i, i)] : 1.0;
    }
    const bool ok = cholesky_packed<N>(cm);
    if (any_drop || !ok) st |= FF_ST_COV_SINGULAR;
    const double s2 = F / (double)(nvalid - N);
    if (o.cov) {
        for (int c = sub; c < N; c += L) {
            double e[N], col[N];
#pragma unroll
            for (int i = 0; i < N; ++i) { e[i] = i == c ? 1.0 : 0.0; col[i] = 0.0; }
            if (ok) cholesky_solve<N>(cm, e, col);
            bool keepc = false;
#pragma unroll
            for (int i = 0; i < N; ++i) keepc = keepc || (i == c && keep[i]);
            const double dc = D->hi[c] - D->lo[c];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if (i <= c) {
                    const double v = (ok && keep[i] && keepc)
                        ? s2 * col[i] * 0.25 * (D->hi[i] - D->lo[i]) * dc
                        : __builtin_nan("");
                    o.cov[pix * NT + upper(N, i, c)] = (float)v;
                }
            }
        }
    }
    if (sub == 0) {
        double et, sd;
        PM::moments(x, et, sd);
        if (o.moments) { o.moments[2 * pix] = (float)et; o.moments[2 * pix + 1] = (float)sd; }
        if (o.state) for (int j = 0; j < N; ++j) o.state[pix * N + j] = (float)x[j];
        if (o.state64) for (int j = 0; j < N; ++j) o.state64[pix * N + j] = x[j];
    }
    return st;
}

template <typename T>
__global__ void fill_struct(const T v, T* __restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = v;
}

__global__ void zero_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// one atomic per wave: the wave's sum of v added to *counter (lane 0 adds)
__device__ __forceinline__ void wave_add(unsigned long long* counter, unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffull), off);
        const unsigned hi = __shfl_xor((unsigned)(v >> 32), off);
        v += ((unsigned long long)hi << 32) | lo;
    }
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(counter, v);
}

}  // namespace
}  // namespace ff
