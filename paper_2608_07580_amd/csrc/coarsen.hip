// Resolution rescaling (Keely et al., the spatial resolution rescaling of the
// methods and its Results): coarse radiance by block means of fine pixels in
// radiance space, and the Quantile Error Curve between each coarse pixel's
// moment-matched Gaussian and the fine retrievals inside its footprint.
//
// block_mean_kernel (HBM-bound): one workgroup per coarse pixel.  With a
// band count divisible by 4 each thread owns a quad of bands (16-byte loads)
// and the workgroup's threads form G = 256 / (B / 4) groups that take every
// G-th fine pixel of the footprint, so G fine rows stream at once; the group
// sums meet in LDS.  Sums in FP64 (exact for up to 1,024 float32 values of
// similar size, so the order of the additions does not change them), one
// rounding to float32.  Other band counts: lanes over bands, one float each.
//
// qec_kernel: one wave per coarse pixel.  The wave gathers the selected fine
// pixels of the footprint into LDS (ballot compaction), ranks them by
// counting (n <= 1,024 values, each lane ranks its own), reads the
// empirical quantiles off the sorted values, and finds each mixture
// quantile by bisection on the equal-weight mixture CDF, the CDF terms
// spread over the lanes and summed by a butterfly.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ff_internal.hpp"

namespace ff {
namespace {

constexpr int kMaxBlock = 32;                  // footprint side
constexpr int kMaxFine = kMaxBlock * kMaxBlock;
constexpr int kMaxLevels = 16;

__global__ void __launch_bounds__(256) block_mean_kernel(const float* __restrict__ rad, int cols, int B, int block,
                                                         int C, float* __restrict__ out)
{
    const int k = blockIdx.x;       // coarse pixel
    const int r = k / C, c = k % C;
    const double inv = 1.0 / (double)(block * block);
    const int nq = B / 4;
    if ((B & 3) == 0 && nq <= 256) {
        __shared__ double part[256 * 4];
        const int G = 256 / nq;
        const int t = threadIdx.x, q = t % nq, g = t / nq;
        const int n = block * block;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (g < G) {
#pragma unroll 4
            for (int idx = g; idx < n; idx += G) {
                const int i = idx / block, j = idx - i * block;
                const int64_t px = (int64_t)(r * block + i) * cols + (int64_t)c * block + j;
                const float4 v = *reinterpret_cast<const float4*>(rad + px * B + 4 * q);
                s0 += (double)v.x;
                s1 += (double)v.y;
                s2 += (double)v.z;
                s3 += (double)v.w;
            }
            part[4 * t + 0] = s0;
            part[4 * t + 1] = s1;
            part[4 * t + 2] = s2;
            part[4 * t + 3] = s3;
        }
        __syncthreads();
        if (t < nq) {
            for (int h = 1; h < G; ++h) {
                const double* p = part + 4 * (h * nq + t);
                s0 += p[0];
                s1 += p[1];
                s2 += p[2];
                s3 += p[3];
            }
            const float4 m = {(float)(s0 * inv), (float)(s1 * inv), (float)(s2 * inv), (float)(s3 * inv)};
            *reinterpret_cast<float4*>(out + (int64_t)k * B + 4 * t) = m;
        }
        return;
    }
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < block; ++i) {
            const int64_t row = (int64_t)(r * block + i) * cols + (int64_t)c * block;
            for (int j = 0; j < block; ++j) s += (double)rad[(row + j) * B + b];
        }
        out[(int64_t)k * B + b] = (float)(s * inv);
    }
}

struct QecArgs {
    const float* fm;   const float* fs;   const uint32_t* fst;   // fine moments [P][2], state [P][n], status
    const float* cm;   const float* cs;   const uint32_t* cst;   // coarse
    const uint8_t* fmask;  const uint8_t* cmask;                 // optional selections (0: excluded)
    int n_state;
    int cols, block, C;
    double f_min;
    int min_fine;
    int n_levels;
    double level[kMaxLevels];
    double z[kMaxLevels];      // standard-normal quantiles of the levels
    float* emp;
    float* mix;
    int32_t* n_used;
};

__device__ __forceinline__ bool selected(const float* m, const float* s, const uint32_t* st, const uint8_t* mask,
                                         int n_state, int64_t p, double f_min)
{
    const float et = m[2 * p], sd = m[2 * p + 1];
    return (st[p] & FF_ST_CONVERGED) != 0 && (double)s[p * n_state] >= f_min && isfinite(et) && isfinite(sd) &&
           sd > 0.f && (!mask || mask[p] != 0);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ void __launch_bounds__(64) qec_kernel(QecArgs a)
{
    __shared__ float s_et[kMaxFine];
    __shared__ float s_sd[kMaxFine];
    __shared__ float s_sorted[kMaxFine];
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const int r = k / a.C, c = k % a.C;
    const int nb = a.block * a.block;
    // gather the selected fine pixels (footprint order)
    int n = 0;
    for (int base = 0; base < nb; base += 64) {
        const int i = base + lane;
        bool sel = false;
        int64_t p = 0;
        if (i < nb) {
            p = (int64_t)(r * a.block + i / a.block) * a.cols + (int64_t)c * a.block + i % a.block;
            sel = selected(a.fm, a.fs, a.fst, a.fmask, a.n_state, p, a.f_min);
        }
        const unsigned long long m = __ballot(sel);
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (sel) {
            s_et[n + below] = a.fm[2 * p];
            s_sd[n + below] = a.fm[2 * p + 1];
        }
        n += __popcll(m);
    }
    __syncthreads();
    if (lane == 0) a.n_used[k] = n;
    const bool ok = selected(a.cm, a.cs, a.cst, a.cmask, a.n_state, k, a.f_min) && n >= a.min_fine;
    if (!ok) {
        for (int j = lane; j < a.n_levels; j += 64) {
            a.emp[(int64_t)k * a.n_levels + j] = __builtin_nanf("");
            a.mix[(int64_t)k * a.n_levels + j] = __builtin_nanf("");
        }
        return;
    }
    // rank sort: value i goes to the number of values before it in (value, index) order
    for (int i = lane; i < n; i += 64) {
        const float v = s_et[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const float w = s_et[j];
            rank += (w < v || (w == v && j < i)) ? 1 : 0;
        }
        s_sorted[rank] = v;
    }
    __syncthreads();
    const double et_c = (double)a.cm[2 * k], sd_c = (double)a.cm[2 * k + 1];
    // bracket of every mixture quantile
    double lo = INFINITY, hi = -INFINITY;
    for (int i = lane; i < n; i += 64) {
        lo = fmin(lo, (double)s_et[i] - 12.0 * (double)s_sd[i]);
        hi = fmax(hi, (double)s_et[i] + 12.0 * (double)s_sd[i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    const double inv_n = 1.0 / (double)n;
    for (int j = 0; j < a.n_levels; ++j) {
        const double q = a.level[j];
        const double gauss = et_c + sd_c * a.z[j];
        // empirical: linear interpolation between order statistics
        const double h = (double)(n - 1) * q;
        const int i0 = (int)floor(h);
        const int i1 = min(i0 + 1, n - 1);
        const double t = h - (double)i0;
        const double x0 = (double)s_sorted[i0], x1 = (double)s_sorted[i1];
        const double qe = t >= 0.5 ? x1 - (x1 - x0) * (1.0 - t) : x0 + (x1 - x0) * t;
        // mixture: bisection on (1/n) sum_i Phi((x - mu_i)/sd_i) = q
        double a0 = lo, a1 = hi;
        for (int it = 0; it < 100 && a1 - a0 > 1e-9 * fmax(1.0, fabs(a0)); ++it) {
            const double x = 0.5 * (a0 + a1);
            double F = 0.0;
            for (int i = lane; i < n; i += 64)
                F += 0.5 * erfc(-(x - (double)s_et[i]) / ((double)s_sd[i] * 1.4142135623730951));
            F = wave_sum(F) * inv_n;
            if (F < q) a0 = x;
            else a1 = x;
        }
        if (lane == 0) {
            a.emp[(int64_t)k * a.n_levels + j] = (float)(gauss - qe);
            a.mix[(int64_t)k * a.n_levels + j] = (float)(gauss - 0.5 * (a0 + a1));
        }
    }
}

// Standard-normal quantile by bisection on erfc (host, FP64).
double normal_quantile(double q)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        const double x = 0.5 * (lo + hi);
        if (0.5 * std::erfc(-x / std::sqrt(2.0)) < q) lo = x;
        else hi = x;
    }
    return 0.5 * (lo + hi);
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" ff_status ff_block_mean(const float* radiance_dev, int32_t rows, int32_t cols, int32_t n_bands,
                                   int32_t block, float* out_dev, void* stream)
{
    if (rows < 0 || cols < 0 || n_bands < 1 || block < 1) return set_error(FF_EINVAL, "ff_block_mean: bad sizes");
    const int R = rows / block, C = cols / block;
    if ((int64_t)R * C == 0) return clear_error();
    if (block > kMaxBlock) return set_error(FF_EINVAL, "ff_block_mean: block larger than 32");
    if (!radiance_dev || !out_dev) return set_error(FF_EINVAL, "ff_block_mean: NULL buffer");
    hipLaunchKernelGGL(block_mean_kernel, dim3((unsigned)(R * C)), dim3(256), 0, (hipStream_t)stream, radiance_dev,
                       cols, n_bands, block, C, out_dev);
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

extern "C" ff_status ff_qec(const float* fine_moments_dev, const float* fine_state_dev, const uint32_t* fine_status_dev,
                            const uint8_t* fine_mask_dev, const float* coarse_moments_dev, const float* coarse_state_dev,
                            const uint32_t* coarse_status_dev, const uint8_t* coarse_mask_dev, int32_t n_state,
                            int32_t rows, int32_t cols,
                            int32_t block, double f_min, int32_t min_fine, int32_t n_levels,
                            const double* levels_host, float* qec_emp_dev, float* qec_mix_dev, int32_t* n_used_dev,
                            void* stream)
{
    if (rows < 0 || cols < 0 || block < 1 || block > kMaxBlock || n_state < 1 || n_state > FF_MAX_STATE)
        return set_error(FF_EINVAL, "ff_qec: bad sizes (block must be in [1, 32])");
    if (n_levels < 1 || n_levels > kMaxLevels || !levels_host)
        return set_error(FF_EINVAL, "ff_qec: 1 to 16 quantile levels");
    for (int j = 0; j < n_levels; ++j)
        if (!(levels_host[j] > 0.0 && levels_host[j] < 1.0)) return set_error(FF_EINVAL, "ff_qec: levels must lie in (0, 1)");
    if (min_fine < 1) return set_error(FF_EINVAL, "ff_qec: min_fine < 1");
    const int R = rows / block, C = cols / block;
    if ((int64_t)R * C == 0) return clear_error();
    if (!fine_moments_dev || !fine_state_dev || !fine_status_dev || !coarse_moments_dev || !coarse_state_dev ||
        !coarse_status_dev || !qec_emp_dev || !qec_mix_dev || !n_used_dev)
        return set_error(FF_EINVAL, "ff_qec: NULL buffer");
    QecArgs a{};
    a.fm = fine_moments_dev;
    a.fs = fine_state_dev;
    a.fst = fine_status_dev;
    a.cm = coarse_moments_dev;
    a.cs = coarse_state_dev;
    a.cst = coarse_status_dev;
    a.fmask = fine_mask_dev;
    a.cmask = coarse_mask_dev;
    a.n_state = n_state;
    a.cols = cols;
    a.block = block;
    a.C = C;
    a.f_min = f_min;
    a.min_fine = min_fine;
    a.n_levels = n_levels;
    for (int j = 0; j < n_levels; ++j) {
        a.level[j] = levels_host[j];
        a.z[j] = normal_quantile(levels_host[j]);
    }
    a.emp = qec_emp_dev;
    a.mix = qec_mix_dev;
    a.n_used = n_used_dev;
    hipLaunchKernelGGL(qec_kernel, dim3((unsigned)(R * C)), dim3(64), 0, (hipStream_t)stream, a);
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}
