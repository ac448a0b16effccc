// Fire-candidate pre-filter (Keely et al. Sec. 2.1): the hyperspectral fire
// detection index HFDI = (L(2430) - L(2061)) / (L(2430) + L(2061)) per pixel
// and the list of candidate pixels, in increasing order, built on the device.
//
// Three launches, no host round trip: (1) each workgroup takes a tile of
// kTile pixels, writes their index values, keeps each wave's candidate flags
// as one 64-bit ballot per step and counts its candidates; (2) one workgroup
// scans the tile counts into tile offsets and the total; (3) each workgroup
// reads its tile's ballots back and writes the candidates' pixel numbers at
// its offset, ordered by the ballot prefix and a prefix over the waves of
// the workgroup.  The list is therefore deterministic and sorted, and the
// total is left in device memory for the retrieval to read.
//
// Reads: two radiance values per pixel (separate cache lines of the row),
// once; the pass is HBM-latency bound and small next to any retrieval.
#include <algorithm>
#include <cmath>

#include "ff_internal.hpp"

namespace ff {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kThreads * kPerThread;

struct HfdiArgs {
    const float* rad;
    int64_t P;
    int B;
    int ia, ib;           // bands nearest 2430 and 2061 nm
    float sat_a, sat_b;   // their saturation levels (+inf when none)
    double threshold;
};

// Index value and candidate decision of pixel p: IEEE float32 arithmetic on
// the radiances; the threshold is compared in double; a saturated index band
// makes a candidate whatever the index.
__device__ __forceinline__ bool candidate(const HfdiArgs& a, int64_t p, float& h)
{
    const float la = a.rad[p * a.B + a.ia];
    const float lb = a.rad[p * a.B + a.ib];
    h = (la - lb) / (la + lb);   // correctly rounded (no fast-math division)
    return (double)h >= a.threshold || la >= a.sat_a || lb >= a.sat_b;
}

// Ballots of one tile: kPerThread steps x (kThreads / 64) waves.
constexpr int kTileMasks = kPerThread * (kThreads / 64);

__global__ void __launch_bounds__(kThreads) hfdi_count(HfdiArgs a, float* __restrict__ hfdi_out,
                                                       int64_t* __restrict__ tile_count,
                                                       unsigned long long* __restrict__ masks)
{
    __shared__ int wave_n[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int n = 0;
#pragma unroll 4
    for (int k = 0; k < kPerThread; ++k) {
        const int64_t p = base + (int64_t)k * kThreads + threadIdx.x;
        bool c = false;
        if (p < a.P) {
            float h;
            c = candidate(a, p, h);
            n += c ? 1 : 0;
            if (hfdi_out) hfdi_out[p] = h;
        }
        const unsigned long long m = __ballot(c);
        if (lane == 0) masks[(size_t)blockIdx.x * kTileMasks + k * (kThreads / 64) + wave] = m;
    }
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & 63) == 0) wave_n[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += wave_n[w];
        tile_count[blockIdx.x] = t;
    }
}

// Exclusive scan of the tile counts (one workgroup): each thread sums a
// contiguous run of tiles, the run sums are scanned in LDS, and each thread
// writes its run's offsets; the total goes to *count.
__global__ void __launch_bounds__(1024) scan_tiles(const int64_t* __restrict__ tile_count, int n_tiles,
                                                   int64_t* __restrict__ tile_off, int64_t* __restrict__ count)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (n_tiles + 1023) / 1024;
    const int lo = t * per, hi = min(n_tiles, lo + per);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += tile_count[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;   // exclusive prefix of this thread's run
    for (int i = lo; i < hi; ++i) {
        tile_off[i] = run;
        run += tile_count[i];
    }
    if (t == 1023) *count = part[1023];
}

__global__ void __launch_bounds__(kThreads) hfdi_write(const int64_t* __restrict__ tile_off,
                                                       const unsigned long long* __restrict__ masks,
                                                       int64_t* __restrict__ index_out)
{
    __shared__ int wave_n[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t off = tile_off[blockIdx.x];
    for (int k = 0; k < kPerThread; ++k) {
        const int64_t p = base + (int64_t)k * kThreads + threadIdx.x;
        // the count pass's ballot for this step and wave (pixels past P are 0)
        const unsigned long long m = masks[(size_t)blockIdx.x * kTileMasks + k * (kThreads / 64) + wave];
        const bool c = ((m >> lane) & 1ull) != 0;
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (lane == 0) wave_n[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            before += w < wave ? wave_n[w] : 0;
            total += wave_n[w];
        }
        if (c) index_out[off + before + below] = p;
        off += total;
        __syncthreads();
    }
}

int nearest(const std::vector<double>& lam, double target)
{
    int best = 0;
    for (int b = 1; b < (int)lam.size(); ++b)
        if (std::fabs(lam[b] - target) < std::fabs(lam[best] - target)) best = b;
    return best;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" ff_status ff_hfdi_candidates(const ff_scene* scene, const float* radiance_dev, int64_t P,
                                        double threshold, float* hfdi_dev, int64_t* index_dev,
                                        int64_t* count_dev, void* stream)
{
    if (!scene) return set_error(FF_EINVAL, "ff_hfdi_candidates: scene is NULL");
    if (P < 0) return set_error(FF_EINVAL, "ff_hfdi_candidates: P < 0");
    if (!count_dev || (P > 0 && (!radiance_dev || !index_dev)))
        return set_error(FF_EINVAL, "ff_hfdi_candidates: NULL radiance, index or count");
    if (std::isnan(threshold)) return set_error(FF_EINVAL, "ff_hfdi_candidates: threshold is NaN");
    if ((int)scene->lambda.size() != scene->n_bands || (int)scene->lsat.size() != scene->n_bands ||
        scene->n_bands < 1)
        return set_error(FF_EINVAL, "ff_hfdi_candidates: scene without band centres");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_tiles64 = (P + kTile - 1) / kTile;
    if (n_tiles64 > 0x7fffffff) return set_error(FF_EINVAL, "ff_hfdi_candidates: P too large");
    const int n_tiles = (int)std::max<int64_t>(n_tiles64, 1);
    int64_t* scratch = nullptr;
    {
        const size_t bytes = (size_t)2 * n_tiles * sizeof(int64_t) + (size_t)n_tiles * kTileMasks * sizeof(uint64_t);
        const ff_status st = stream_scratch(s, bytes, reinterpret_cast<void**>(&scratch));
        if (st != FF_OK) return st;
    }
    int64_t* tile_count = scratch;
    int64_t* tile_off = scratch + n_tiles;
    auto* masks = reinterpret_cast<unsigned long long*>(scratch + 2 * (size_t)n_tiles);

    HfdiArgs a;
    a.rad = radiance_dev;
    a.P = P;
    a.B = scene->n_bands;
    a.ia = nearest(scene->lambda, 2430.0);
    a.ib = nearest(scene->lambda, 2061.0);
    a.sat_a = scene->lsat[a.ia];
    a.sat_b = scene->lsat[a.ib];
    a.threshold = threshold;

    // with P = 0 the one tile counts nothing and the total becomes 0
    hipLaunchKernelGGL(hfdi_count, dim3(n_tiles), dim3(kThreads), 0, s, a, hfdi_dev, tile_count, masks);
    FF_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(1024), 0, s, tile_count, n_tiles, tile_off, count_dev);
    FF_HIP_TRY(hipGetLastError());
    if (P > 0) {
        hipLaunchKernelGGL(hfdi_write, dim3(n_tiles), dim3(kThreads), 0, s, tile_off, masks, index_dev);
        FF_HIP_TRY(hipGetLastError());
    }
    return clear_error();
}
