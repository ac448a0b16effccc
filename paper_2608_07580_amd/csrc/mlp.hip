// Learned warm start: a multilayer perceptron mapping a radiance spectrum to
// a starting state z0 of the Levenberg-Marquardt solve.
//
//  * bf16 matrix-core GEMM (v_mfma_f32_16x16x32_bf16, FP32 accumulation)
//    with LDS-staged 64x64x32 tiles, used for the forward pass, the
//    backward data pass and the weight gradients, with fused epilogues
//    (bias + GELU, GELU-derivative gating, FP32 store);
//  * feature, loss/output, column-sum and Adam kernels;
//  * a training-data generator: Philox4x32-10 counter-based draws (Salmon,
//    Moraes, Dror & Shaw 2011) of one-component states, the forward model of
//    physics.hpp and Box-Muller noise.
#include <algorithm>
#include <cmath>
#include <string>
#include <cstdio>
#include <cstring>
#include <vector>

#include "physics.hpp"

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

namespace ff {

// ---------------------------------------------------------------- Philox
struct U32x4 {
    uint32_t v[4];
};

// Philox4x32-10: 10 rounds of (hi, lo) = M * c multiplies with a Weyl key
// schedule.  Constants from the published definition.
__host__ __device__ inline U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0 = (uint64_t)M0 * c0;
        const uint64_t p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    return U32x4{{c0, c1, c2, c3}};
}

// uniform in (0, 1): the top 24 bits, centred in their cell
__host__ __device__ inline double u01(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;
constexpr int kGemmThreads = 256;

enum : int { EPI_FWD_GELU = 0, EPI_FWD_LINEAR = 1, EPI_BWD_GELU = 2, EPI_F32 = 3, EPI_FWD_GELU_NOH = 4 };

struct EpiArgs {
    const float* bias;
    float* outf;
    int ldof;
    __bf16* outb;
    int ldob;
    const float* hprev;
    int ldh;
    // rows read from device memory: only rows m < *mcount - mbase exist
    // (the rest of the launch's M rows are skipped); null: all M rows
    const int64_t* mcount = nullptr;
    int64_t mbase = 0;
};

// The rows of an M-row launch that exist (see EpiArgs::mcount).
__device__ __forceinline__ int live_rows(const EpiArgs& ep, int M)
{
    if (!ep.mcount) return M;
    const int64_t c = *ep.mcount - ep.mbase;
    return c <= 0 ? 0 : (c < (int64_t)M ? (int)c : M);
}

// GELU in its tanh form, evaluated as x * sigmoid(2u) (equal to
// 0.5 x (1 + tanh u) with u = sqrt(2/pi) (x + 0.044715 x^3)): one exp2 and one
// reciprocal; for large |u| the power saturates to 0 or +inf and the
// reciprocal to 1 or 0, the exact limits.  With r = sigmoid(2u):
// 1 + tanh u = 2 r and 1 - tanh^2 u = 4 r (1 - r).
__device__ __forceinline__ float gelu_r(float x, float& x2)
{
    const float c2 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;   // -2 sqrt(2/pi) log2 e
    x2 = x * x;
    const float u = x * __builtin_fmaf(0.044715f, x2, 1.0f);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(c2 * u));
}

__device__ __forceinline__ float gelu_t(float x, float& dgelu)
{
    float x2;
    const float r = gelu_r(x, x2);
    const float c = 0.7978845608028654f;   // sqrt(2 / pi)
    dgelu = r + 2.0f * x * r * (1.0f - r) * c * __builtin_fmaf(3.0f * 0.044715f, x2, 1.0f);
    return x * r;
}

__device__ __forceinline__ float gelu_only(float x)
{
    float x2;
    return x * gelu_r(x, x2);
}

// Store one accumulator element through the epilogue EPI.
template <int EPI>
__device__ __forceinline__ void epilogue_store(int m, int n, float v, const EpiArgs& ep)
{
    if (EPI == EPI_FWD_GELU || EPI == EPI_FWD_GELU_NOH) {
        const float h = v + ep.bias[n];
        const float g = gelu_only(h);
        if (EPI == EPI_FWD_GELU) ep.outf[(size_t)m * ep.ldof + n] = h;
        ep.outb[(size_t)m * ep.ldob + n] = (__bf16)g;
    } else if (EPI == EPI_FWD_LINEAR) {
        ep.outf[(size_t)m * ep.ldof + n] = v + ep.bias[n];
    } else if (EPI == EPI_BWD_GELU) {
        float dg;
        gelu_t(ep.hprev[(size_t)m * ep.ldh + n], dg);
        ep.outb[(size_t)m * ep.ldob + n] = (__bf16)(v * dg);
    } else {
        ep.outf[(size_t)m * ep.ldof + n] = v;
    }
}

// C[m][n] = sum_k Aop[m][k] Bop[k][n];  Aop = TA ? A[k][m] : A[m][k],
// Bop = TB ? B[n][k] : B[k][n] (lda/ldb = row strides of the stored arrays).
// Loads: m < Ml, n < Nl, k < K (8-element chunks along the contiguous
// dimension, whose extent must be a multiple of 8); stores: m < M, n < N.
// With gridDim.z = S > 1 (EPI_F32 only) workgroup z sums the z-th of S
// kBK-aligned slices of k and stores its partial at outf + z M ldof.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(kGemmThreads)
gemm_bf16(int M, int N, int Ml, int Nl, int K, const __bf16* __restrict__ A, int lda,
          const __bf16* __restrict__ B, int ldb, EpiArgs ep)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[kBM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kBN][kBK + kPad];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    M = live_rows(ep, M);
    if (m0 >= M) return;
    Ml = min(Ml, M);
    float4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    const bf16x8_t zero8 = {};
    int kbeg = 0, kend = K;
    if (gridDim.z > 1) {
        const int kc = ((K + (int)gridDim.z - 1) / (int)gridDim.z + kBK - 1) / kBK * kBK;
        kbeg = (int)blockIdx.z * kc;
        kend = min(K, kbeg + kc);
        ep.outf += (size_t)blockIdx.z * (size_t)M * ep.ldof;
    }

    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        // ---- A tile -> As[m][k]
        if (!TA) {
            const int r = t >> 2, kc = (t & 3) * 8;
            const int m = m0 + r, k = k0 + kc;
            bf16x8_t v = zero8;
            if (m < Ml && k < K) v = *reinterpret_cast<const bf16x8_t*>(A + (size_t)m * lda + k);
            *reinterpret_cast<bf16x8_t*>(&As[r][kc]) = v;
        } else {
            const int kr = t >> 3, mc = (t & 7) * 8;
            const int k = k0 + kr, m = m0 + mc;
            bf16x8_t v = zero8;
            if (k < K && m < Ml) v = *reinterpret_cast<const bf16x8_t*>(A + (size_t)k * lda + m);
#pragma unroll
            for (int e = 0; e < 8; ++e) As[mc + e][kr] = v[e];
        }
        // ---- B tile -> Bs[n][k]
        if (TB) {
            const int r = t >> 2, kc = (t & 3) * 8;
            const int n = n0 + r, k = k0 + kc;
            bf16x8_t v = zero8;
            if (n < Nl && k < K) v = *reinterpret_cast<const bf16x8_t*>(B + (size_t)n * ldb + k);
            *reinterpret_cast<bf16x8_t*>(&Bs[r][kc]) = v;
        } else {
            const int kr = t >> 3, nc = (t & 7) * 8;
            const int k = k0 + kr, n = n0 + nc;
            bf16x8_t v = zero8;
            if (k < K && n < Nl) v = *reinterpret_cast<const bf16x8_t*>(B + (size_t)k * ldb + n);
#pragma unroll
            for (int e = 0; e < 8; ++e) Bs[nc + e][kr] = v[e];
        }
        __syncthreads();
        bf16x8_t a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8_t*>(&As[wm * 32 + i * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn * 32 + j * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }

    // ---- epilogue: lane holds D[4*(lane/16) + e][lane % 16] of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 32 + j * 16 + (lane & 15);
            if (n >= N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                if (m < M) epilogue_store<EPI>(m, n, acc[i][j][e], ep);
            }
        }
    }
}

// Forward-pass GEMM C[m][n] = sum_k A[m][k] B[n][k] (both operands contiguous
// in k) for large row counts: 128x128 output tile per workgroup of four
// waves (64x64 each, 4x4 MFMA 16x16x32 accumulators), k advanced 32 at a
// time through double-buffered LDS with one barrier per step; the next k
// slice is fetched into registers while the current one feeds the matrix
// cores.  (A 64-wide k step measured slower: its LDS and registers halve
// the workgroups resident per CU.)  Requires N % 128 == 0 and K % 8 == 0;
// rows m >= Ml read as zero, rows m >= M are not stored.
constexpr int kFM = 128, kFN = 128;

template <int EPI>
__global__ void __launch_bounds__(kGemmThreads)
gemm_nt_128(int M, int N, int Ml, int K, const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B,
            int ldb, EpiArgs ep)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[2][kFM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][kFN][kBK + kPad];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * kFM, n0 = blockIdx.x * kFN;
    M = live_rows(ep, M);
    if (m0 >= M) return;
    Ml = min(Ml, M);
    const int lr = t >> 2, lk = (t & 3) * 8;     // this thread's load rows lr, lr + 64 and k chunk
    const bf16x8_t zero8 = {};
    float4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

    bf16x8_t ra[2], rb[2];
    auto fetch = [&](int k0) {
        const int k = k0 + lk;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = m0 + lr + 64 * h;
            const int n = n0 + lr + 64 * h;
            ra[h] = (m < Ml && k < K) ? *reinterpret_cast<const bf16x8_t*>(A + (size_t)m * lda + k) : zero8;
            rb[h] = (n < N && k < K) ? *reinterpret_cast<const bf16x8_t*>(B + (size_t)n * ldb + k) : zero8;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<bf16x8_t*>(&As[buf][lr + 64 * h][lk]) = ra[h];
            *reinterpret_cast<bf16x8_t*>(&Bs[buf][lr + 64 * h][lk]) = rb[h];
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += kBK) {
        const bool more = k0 + kBK < K;
        if (more) fetch(k0 + kBK);
        bf16x8_t a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const bf16x8_t*>(&As[cur][wm * 64 + i * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = *reinterpret_cast<const bf16x8_t*>(&Bs[cur][wn * 64 + j * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (more) stash(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + e;
                if (m < M) epilogue_store<EPI>(m, n, acc[i][j][e], ep);
            }
        }
    }
}

// Forward-pass GEMM with direct-to-LDS loads (global_load_lds_dwordx4):
// 128x128 tile, four waves of 64x64 each as 2x2 v_mfma_f32_32x32x16_bf16
// tiles (on gfx950 the 32x32x16 form sustains twice the rate of 16x16x32,
// measured 2.3 vs 1.3 PFLOP/s, and reads half the operand bytes per flop);
// each k slice
// (32 wide) is copied by the load unit straight into LDS without passing
// through registers, three slices in flight (ring of three LDS stages, one
// barrier per slice).  A wave's load writes 1 KB of LDS at M0 + 16 * lane,
// i.e. 16 rows of 64 B; lane L takes row L / 4 of its block and 16-byte
// chunk (L % 4) ^ ((row >> 1) & 3), so the chunks of a row are stored
// swizzled and the 16-byte operand reads of 8 consecutive rows hit disjoint
// banks.  Rows m >= Ml load row Ml - 1 (in bounds; their results are not
// stored).  Requires N % 128 == 0, K % 32 == 0, Ml >= 1.
// XCD-aware tile order: the grid is 1-D and the hardware hands consecutive
// workgroup ids to the 8 XCDs in turn, so id g works on tile
// (g % 8) * per_xcd + g / 8 -- each XCD takes a contiguous run of tiles
// (all column tiles of its row blocks), and an activation row block is
// fetched into one L2 instead of four.
typedef __attribute__((address_space(3))) void* lds_ptr_t;
constexpr int kLdsStages = 3;
constexpr int kXcds = 8;   // XCDs of an MI355X

template <int VM>
__device__ __forceinline__ void wait_vmcnt()
{
    // s_waitcnt with vmcnt = VM and the other counters at their maximum
    __builtin_amdgcn_s_waitcnt((VM & 0xF) | ((VM >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <int EPI>
__global__ void __launch_bounds__(kGemmThreads)
gemm_nt_lds(int M, int N, int Ml, int K, const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B,
            int ldb, EpiArgs ep)
{
    // one LDS object per stage, so the compiler can tell a stage being read
    // from the stages whose loads are still in flight
    __shared__ __attribute__((aligned(1024))) __bf16 A0[kFM * 32], A1[kFM * 32], A2[kFM * 32];
    __shared__ __attribute__((aligned(1024))) __bf16 B0[kFN * 32], B1[kFN * 32], B2[kFN * 32];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w >> 1, wn = w & 1;
    const int n_tiles_n = N / kFN;
    const int n_tiles = n_tiles_n * ((M + kFM - 1) / kFM);
    const int per_xcd = (n_tiles + kXcds - 1) / kXcds;
    const int tile = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    if (tile >= n_tiles) return;
    const int m0 = (tile / n_tiles_n) * kFM, n0 = (tile % n_tiles_n) * kFN;
    M = live_rows(ep, M);
    if (m0 >= M) return;
    Ml = min(Ml, M);
    const __bf16* ga[2];
    const __bf16* gb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = 32 * w + 16 * h + (lane >> 2);
        const int c = (lane & 3) ^ ((r >> 1) & 3);
        const int m = min(m0 + r, Ml - 1);
        ga[h] = A + (size_t)m * lda + 8 * c;
        gb[h] = B + (size_t)(n0 + r) * ldb + 8 * c;
    }
    auto issue = [&](__bf16* as, __bf16* bs, int k0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row0 = 32 * w + 16 * h;
            __builtin_amdgcn_global_load_lds((const void*)(ga[h] + k0), (lds_ptr_t)(as + row0 * 32), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(gb[h] + k0), (lds_ptr_t)(bs + row0 * 32), 16, 0, 0);
        }
    };
    // 32x32x16 operand layout: lane l holds row (A) / column (B) l % 32 and
    // k = 8 (l / 32) + 0..7 of a 16-wide k half; result element e of lane l
    // is D[8 (e / 4) + 4 (l / 32) + e % 4][l % 32].  The inference epilogue
    // (BF16 output only) swaps the operands, so a lane holds one output row
    // and runs of four consecutive columns, which it packs into 8-byte LDS
    // writes; the tile then leaves through LDS as 16-byte row-contiguous
    // stores.
    constexpr bool kRowsInLanes = EPI == EPI_FWD_GELU_NOH;
    f32x16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
    int ao[4], bo[4];   // element offsets of this lane's operand chunks inside a stage: [tile * 2 + k half]
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            const int ra = wm * 64 + ti * 32 + (lane & 31);
            const int rb = wn * 64 + ti * 32 + (lane & 31);
            const int c = 2 * kh + (lane >> 5);
            ao[ti * 2 + kh] = ra * 32 + ((c ^ ((ra >> 1) & 3)) * 8);
            bo[ti * 2 + kh] = rb * 32 + ((c ^ ((rb >> 1) & 3)) * 8);
        }
    }
    auto compute = [&](const __bf16* as, const __bf16* bs) {
        // The eight operand reads are issued (and waited for) in one asm
        // block: the slice they read is complete by the caller's vmcnt wait
        // and barrier, while the compiler, unable to tell LDS stages apart,
        // would otherwise wait for every load still in flight.
        typedef __attribute__((address_space(3))) const __bf16* lds_cptr_t;
        const unsigned la = (unsigned)(uintptr_t)(lds_cptr_t)as, lb = (unsigned)(uintptr_t)(lds_cptr_t)bs;
        bf16x8_t a[4], b[4];
        asm volatile(
            "ds_read_b128 %0, %8\n\t"
            "ds_read_b128 %1, %9\n\t"
            "ds_read_b128 %2, %10\n\t"
            "ds_read_b128 %3, %11\n\t"
            "ds_read_b128 %4, %12\n\t"
            "ds_read_b128 %5, %13\n\t"
            "ds_read_b128 %6, %14\n\t"
            "ds_read_b128 %7, %15\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=v"(a[0]), "=v"(a[1]), "=v"(a[2]), "=v"(a[3]), "=v"(b[0]), "=v"(b[1]), "=v"(b[2]), "=v"(b[3])
            : "v"(la + 2u * ao[0]), "v"(la + 2u * ao[1]), "v"(la + 2u * ao[2]), "v"(la + 2u * ao[3]),
              "v"(lb + 2u * bo[0]), "v"(lb + 2u * bo[1]), "v"(lb + 2u * bo[2]), "v"(lb + 2u * bo[3])
            : "memory");
#pragma unroll
        for (int kh = 0; kh < 2; ++kh)
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    if constexpr (kRowsInLanes)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[tj * 2 + kh], a[ti * 2 + kh],
                                                                               acc[ti][tj], 0, 0, 0);
                    else
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti * 2 + kh], b[tj * 2 + kh],
                                                                               acc[ti][tj], 0, 0, 0);
                }
    };
    // slice kt lives in stage kt % 3; at step kt: wait for slice kt, barrier
    // (everyone is done with slice kt - 1, whose stage slice kt + 2 reuses),
    // issue slice kt + 2, compute slice kt
    auto step = [&](int kt, int KT, __bf16* as, __bf16* bs, __bf16* an, __bf16* bn) {
        if (kt + 1 < KT) wait_vmcnt<4>();
        else wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        if (kt + 2 < KT) issue(an, bn, (kt + 2) * 32);
        compute(as, bs);
    };
    const int KT = K / 32;
    issue(A0, B0, 0);
    if (KT > 1) issue(A1, B1, 32);
    for (int kt = 0; kt < KT; kt += 3) {
        step(kt, KT, A0, B0, A2, B2);
        if (kt + 1 < KT) step(kt + 1, KT, A1, B1, A0, B0);
        if (kt + 2 < KT) step(kt + 2, KT, A2, B2, A1, B1);
    }
    if constexpr (kRowsInLanes) {
        // Every wave is past its last operand read (and every load has
        // landed) after this barrier; wave w then owns stage buffer w
        // (8 KB = its 64 x 64 BF16 sub-tile).  Rows of 128 B, 16-byte chunk
        // c of row r at chunk c ^ ((r >> 1) & 7) against bank conflicts.
        __builtin_amdgcn_s_barrier();
        __bf16* stage = w == 0 ? A0 : w == 1 ? A1 : w == 2 ? A2 : B0;
        const int r = lane & 31;
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int nl = tj * 32 + 8 * q + 4 * (lane >> 5);   // first of this lane's 4 columns
                const float* bias = ep.bias + n0 + wn * 64 + nl;
                const float b0 = bias[0], b1 = bias[1], b2 = bias[2], b3 = bias[3];
#pragma unroll
                for (int ti = 0; ti < 2; ++ti) {
                    const int rr = ti * 32 + r;
                    bf16x4_t v;
                    v[0] = (__bf16)gelu_only(acc[ti][tj][4 * q + 0] + b0);
                    v[1] = (__bf16)gelu_only(acc[ti][tj][4 * q + 1] + b1);
                    v[2] = (__bf16)gelu_only(acc[ti][tj][4 * q + 2] + b2);
                    v[3] = (__bf16)gelu_only(acc[ti][tj][4 * q + 3] + b3);
                    const int chunk = (nl >> 3) ^ ((rr >> 1) & 7);
                    *reinterpret_cast<bf16x4_t*>(stage + rr * 64 + chunk * 8 + (nl & 4)) = v;
                }
            }
        }
        __builtin_amdgcn_s_barrier();
        // 8 rows x 8 chunks per pass, 8 passes
#pragma unroll
        for (int pass = 0; pass < 8; ++pass) {
            const int rr = pass * 8 + (lane >> 3), c = lane & 7;
            const bf16x8_t v = *reinterpret_cast<const bf16x8_t*>(stage + rr * 64 + ((c ^ ((rr >> 1) & 7)) * 8));
            const int m = m0 + wm * 64 + rr;
            if (m < M)
                *reinterpret_cast<bf16x8_t*>(ep.outb + (size_t)m * ep.ldob + n0 + wn * 64 + 8 * c) = v;
        }
        return;
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            const int n = n0 + wn * 64 + tj * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int m = m0 + wm * 64 + ti * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                if (m < M) epilogue_store<EPI>(m, n, acc[ti][tj][e], ep);
            }
        }
    }
}

// u_b = (ln max(L_b, floor) - mean_b) * inv_std_b, zero-padded to kin columns
// (kin a multiple of 8).  One thread per 8 consecutive features of a row: two
// 16-byte radiance loads when the row's length is a multiple of 4 (rows
// 16-byte aligned), one 16-byte BF16 store.  ln from the hardware log2
// (v_log_f32, ~1 ulp): the feature is rounded to BF16 (8 significant bits).
__device__ __forceinline__ void features_chunk(const float* __restrict__ row, int n_in, int b0,
                                               const float* __restrict__ mean, const float* __restrict__ inv_std,
                                               float floor_v, __bf16* __restrict__ out)
{
    float v[8], mu[8], is[8];
    if ((n_in & 3) == 0) {
        // whole 16-byte quarters (row, mean and 1/s.d. alike), a quarter past
        // the row's end re-read from its last quarter and masked below: no
        // divergent element-wise tail (n_in >= 4 here)
        const int o0 = min(b0, n_in - 4), o1 = min(b0 + 4, n_in - 4);
        const float4 x0 = *reinterpret_cast<const float4*>(row + o0);
        const float4 x1 = *reinterpret_cast<const float4*>(row + o1);
        const float4 m0 = *reinterpret_cast<const float4*>(mean + o0);
        const float4 m1 = *reinterpret_cast<const float4*>(mean + o1);
        const float4 s0 = *reinterpret_cast<const float4*>(inv_std + o0);
        const float4 s1 = *reinterpret_cast<const float4*>(inv_std + o1);
        v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w; v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
        mu[0] = m0.x; mu[1] = m0.y; mu[2] = m0.z; mu[3] = m0.w; mu[4] = m1.x; mu[5] = m1.y; mu[6] = m1.z; mu[7] = m1.w;
        is[0] = s0.x; is[1] = s0.y; is[2] = s0.z; is[3] = s0.w; is[4] = s1.x; is[5] = s1.y; is[6] = s1.z; is[7] = s1.w;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool in = b0 + j < n_in;
            v[j] = in ? row[b0 + j] : 0.f;
            mu[j] = in ? mean[b0 + j] : 0.f;
            is[j] = in ? inv_std[b0 + j] : 0.f;
        }
    }
    bf16x8_t u;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        u[j] = (__bf16)(b0 + j < n_in
                            ? (__builtin_amdgcn_logf(fmaxf(v[j], floor_v)) * 0.6931471805599453f - mu[j]) * is[j]
                            : 0.f);
    *reinterpret_cast<bf16x8_t*>(out) = u;
}

__global__ void features_kernel(const float* __restrict__ L, int P, int n_in, int kin,
                                const float* __restrict__ mean, const float* __restrict__ inv_std,
                                float floor_v, __bf16* __restrict__ X)
{
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned cpr = (unsigned)kin / 8u;   // chunks per row
    if (i >= (unsigned)P * cpr) return;
    const unsigned p = i / cpr;
    const int b0 = 8 * (int)(i - p * cpr);
    features_chunk(L + (size_t)p * n_in, n_in, b0, mean, inv_std, floor_v, X + (size_t)p * kin + b0);
}

// features_kernel for listed rows: row r of X is radiance row index[r];
// entries outside [0, P) give a row of zeros (its output is not stored)
// count (may be null): only list entries base + r < *count exist
__global__ void features_listed_kernel(const float* __restrict__ L, const int64_t* __restrict__ index, int64_t P,
                                       int R, int n_in, int kin, const float* __restrict__ mean,
                                       const float* __restrict__ inv_std, float floor_v, __bf16* __restrict__ X,
                                       const int64_t* __restrict__ count, int64_t base)
{
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned cpr = (unsigned)kin / 8u;
    if (i >= (unsigned)R * cpr) return;
    const unsigned r = i / cpr;
    if (count && base + (int64_t)r >= *count) return;
    const int b0 = 8 * (int)(i - r * cpr);
    const int64_t p = index[r];
    __bf16* out = X + (size_t)r * kin + b0;
    if (p >= 0 && p < P)
        features_chunk(L + p * n_in, n_in, b0, mean, inv_std, floor_v, out);
    else
        *reinterpret_cast<bf16x8_t*>(out) = bf16x8_t{};
}

// z = tanh(y); loss += (z - t)^2; dY = d loss_mean / dy = scale (z - t)(1 - z^2)
// as bf16 (16 columns, zero beyond n_out)
__global__ void loss_kernel(const float* __restrict__ Y, const float* __restrict__ target, int64_t P,
                            int n_out, __bf16* __restrict__ dY, double* __restrict__ loss)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float part = 0.f;
    if (p < P) {
        const float scale = 2.0f / ((float)P * (float)n_out);
        for (int j = 0; j < 16; ++j) {
            float d = 0.f;
            if (j < n_out) {
                const float y = Y[p * 16 + j];
                const float z = tanhf(y);
                const float diff = z - target[p * n_out + j];
                part += diff * diff;
                d = scale * diff * (1.0f - z * z);
            }
            dY[p * 16 + j] = (__bf16)d;
        }
    }
    __shared__ float red[256];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) atomicAdd(loss, (double)red[0] / ((double)P * n_out));
}

__global__ void output_kernel(const float* __restrict__ Y, int64_t P, int n_out, float* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * n_out) return;
    const int64_t p = i / n_out;
    const int j = (int)(i - p * n_out);
    z[i] = tanhf(Y[p * 16 + j]);
}

// output_kernel for listed rows: row r goes to z row index[r] (skipped
// outside [0, P))
__global__ void output_listed_kernel(const float* __restrict__ Y, const int64_t* __restrict__ index, int64_t P,
                                     int64_t R, int n_out, float* __restrict__ z, const int64_t* __restrict__ count,
                                     int64_t base)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * n_out) return;
    const int64_t r = i / n_out;
    if (count && base + r >= *count) return;
    const int j = (int)(i - r * n_out);
    const int64_t p = index[r];
    if (p >= 0 && p < P) z[p * n_out + j] = tanhf(Y[r * 16 + j]);
}

// out[n] = sum_m D[m][n] for n < N (bias gradients)
// Column sums of D [M][N] (the bias gradients), in two deterministic passes
// that fill the chip: partial sums of 64-row chunks, one workgroup per
// (64 columns, chunk), then the chunks summed in order per column.
constexpr int kColChunk = 64;
constexpr int kWgradSplit = 8;
constexpr int64_t kGenPool = 32;     // training steps whose spectra one generator launch makes

// out[i] = sum over the S planes of part[z n + i], in plane order.
__global__ void __launch_bounds__(256) sum_planes_kernel(const float* __restrict__ part, int S, int64_t n,
                                                         float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = part[i];
    for (int z = 1; z < S; ++z) v += part[(size_t)z * n + i];
    out[i] = v;
}

__global__ void __launch_bounds__(256)
colsum_part_kernel(const __bf16* __restrict__ D, int64_t M, int N, int ld, float* __restrict__ part)
{
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int grp = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * kColChunk;
    float s = 0.f;
    if (col < N)
        for (int64_t m = r0 + grp; m < M && m < r0 + kColChunk; m += 4) s += (float)D[m * ld + col];
    __shared__ float red[4][64];
    red[grp][threadIdx.x & 63] = s;
    __syncthreads();
    if (grp == 0 && col < N)
        part[(int64_t)blockIdx.y * N + col] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void colsum_final_kernel(const float* __restrict__ part, int chunks, int N, float* __restrict__ out)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= N) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * N + col];
    out[col] = s;
}

struct LayerMap {
    int64_t off_w[4], off_b[4], off_wb[4];
    int in_dim[4], out_dim[4], in_pad[4];
};

// Adam (m, v moments, bias-corrected) on the FP32 master weights, then the
// BF16 copy of each weight into its padded matrix.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float bc1, float bc2, __bf16* __restrict__ wb, LayerMap map)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int64_t nw = (int64_t)map.out_dim[l] * map.in_dim[l];
        if (i >= map.off_w[l] && i < map.off_w[l] + nw) {
            const int64_t r = (i - map.off_w[l]) / map.in_dim[l];
            const int64_t c = (i - map.off_w[l]) - r * map.in_dim[l];
            wb[map.off_wb[l] + r * map.in_pad[l] + c] = (__bf16)pi;
        }
    }
}

__global__ void refresh_bf16_kernel(const float* __restrict__ p, int64_t n, __bf16* __restrict__ wb, LayerMap map)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int64_t nw = (int64_t)map.out_dim[l] * map.in_dim[l];
        if (i >= map.off_w[l] && i < map.off_w[l] + nw) {
            const int64_t r = (i - map.off_w[l]) / map.in_dim[l];
            const int64_t c = (i - map.off_w[l]) - r * map.in_dim[l];
            wb[map.off_wb[l] + r * map.in_pad[l] + c] = (__bf16)p[i];
        }
    }
}

// per band: mean and 1/s.d. of ln max(L, floor) over P spectra
__global__ void fit_norm_kernel(const float* __restrict__ L, int64_t P, int B, float floor_v,
                                float* __restrict__ mean, float* __restrict__ inv_std)
{
    const int b = blockIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        const double v = log((double)fmaxf(L[p * B + b], floor_v));
        s1 += v;
        s2 += v * v;
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = r1[0] / (double)P;
        const double var = fmax(r2[0] / (double)P - mu * mu, 1e-12);
        mean[b] = (float)mu;
        inv_std[b] = (float)(1.0 / sqrt(var));
    }
}

struct GenArgs {
    double lo[5], hi[5], x0[5];
    uint32_t k0, k1;
    uint64_t offset;
    double snr;
    double bg;
};

// Training spectra (one-component model, FP32 forward), eight bands per
// lane: the lanes of an aligned quad share one sample -- they draw the same
// state, compute a quarter of its node temperatures each and gather them
// with DPP -- so a batch of 2,048 samples is 73,728 lanes instead of 2,048.
constexpr int kGenBands = 8;

inline int gen_chunks(int B) { return (((B + kGenBands - 1) / kGenBands) + 3) / 4 * 4; }

template <int Q>
__global__ void __launch_bounds__(256)
generate_kernel(const float* __restrict__ tab, int B, int64_t P, int chunks, GenArgs ga, float* __restrict__ rad,
                float* __restrict__ target, float* __restrict__ state)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P * chunks) return;            // whole quads: P * chunks is a multiple of four
    const int64_t p = t / chunks;
    const int q = (int)(t - p * chunks);
    const uint64_t g = ga.offset + (uint64_t)p;
    const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);
    const U32x4 r0 = philox4x32_10(glo, ghi, 0u, 0u, ga.k0, ga.k1);
    const U32x4 r1 = philox4x32_10(glo, ghi, 1u, 0u, ga.k0, ga.k1);
    const double lf0 = log(1e-4), lf1 = log(0.3);
    double x[5];
    x[0] = exp(lf0 + (lf1 - lf0) * u01(r0.v[0]));
    x[1] = 600.0 + 800.0 * u01(r0.v[1]);
    x[2] = 50.0 + 250.0 * u01(r0.v[2]);
    x[3] = 0.05 + 0.35 * u01(r0.v[3]);
    x[4] = -1e-4 + 2e-4 * u01(r1.v[0]);
    if (u01(r1.v[1]) < ga.bg) {
        x[0] = 0.0;
        x[1] = ga.x0[1];
        x[2] = ga.x0[2];
    }
    if (q == 0) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const double z = 2.0 * (x[j] - ga.lo[j]) / (ga.hi[j] - ga.lo[j]) - 1.0;
            target[p * 5 + j] = (float)fmin(1.0, fmax(-1.0, z));
            if (state) state[p * 5 + j] = (float)x[j];
        }
    }
    PixelModel<float, FF_MODEL_LOGNORMAL_1, Q> pm;
    pm.setup(x, (int)(threadIdx.x & 63), 4);
    const bool noisy = ga.snr > 0.0;
    const float inv_snr = noisy ? (float)(1.0 / ga.snr) : 0.f;
    float nz[4] = {0.f, 0.f, 0.f, 0.f};
    const int b0 = q * kGenBands;
    for (int b = b0; b < b0 + kGenBands && b < B; ++b) {
        if (noisy && (b & 3) == 0) {
            // four normals per Philox block: Box-Muller on (x0, x1) and (x2, x3)
            const U32x4 rn = philox4x32_10(glo, ghi, 2u + (uint32_t)(b >> 2), 0u, ga.k0, ga.k1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float ua = (float)u01(rn.v[2 * h]), ub = (float)u01(rn.v[2 * h + 1]);
                const float rr = sqrtf(-2.0f * logf(ua));
                float sn, cs;
                sincosf(6.283185307179586f * ub, &sn, &cs);
                nz[2 * h] = rr * cs;
                nz[2 * h + 1] = rr * sn;
            }
        }
        const BandRow<float> row = load_row(tab + (size_t)b * FF_TABLE_COLS);
        float ub[5];
        const float lt = pm.band(row, opaque_zero(), ub);
        rad[p * B + b] = noisy ? lt * (1.0f + nz[b & 3] * inv_snr) : lt;
    }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__global__ void zero_f64(double* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0;
}

}  // namespace
}  // namespace ff

using namespace ff;

struct ff_mlp {
    int device = 0;
    int n_in = 0, h[3] = {0, 0, 0}, n_out = 0, kin = 0;
    int64_t n_params = 0, n_wb = 0;
    LayerMap map{};
    float* params = nullptr;
    float* grads = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    __bf16* wb = nullptr;
    float* mean = nullptr;
    float* inv_std = nullptr;
    float floor_v = 1e-6f;
    int64_t step = 0;                 // Adam updates taken (bias correction of eq. adam)
    int64_t train_steps = 0;          // schedule steps taken by ff_mlp_train / ff_mlp_train_span
    int64_t ws_rows = 0;
    __bf16* X = nullptr;
    float* H[3] = {nullptr, nullptr, nullptr};
    __bf16* A[3] = {nullptr, nullptr, nullptr};
    float* Y = nullptr;
    __bf16* dY = nullptr;
    __bf16* dH[3] = {nullptr, nullptr, nullptr};
    float* part = nullptr;            // column-sum partials [rows / 64][1024]
    float* wpart = nullptr;           // split-K weight-gradient partials [kWgradSplit][largest layer]
    int pins = 0;                     // graphs that bind the workspace (see ff_pipeline_create)
    std::vector<void*> retired;       // workspace buffers replaced while pinned, freed at destroy
};

namespace {

// Largest weight-gradient matrix (outputs x inputs) over the layers.
int64_t wgrad_max(const ff_mlp* m)
{
    int64_t mx = (int64_t)m->n_out * m->h[2];
    mx = std::max<int64_t>(mx, (int64_t)m->h[0] * m->n_in);
    mx = std::max<int64_t>(mx, (int64_t)m->h[1] * m->h[0]);
    mx = std::max<int64_t>(mx, (int64_t)m->h[2] * m->h[1]);
    return mx;
}

// Drop the activation workspace: freed, or -- while a captured graph binds
// it -- kept until the network is destroyed.
void free_ws(ff_mlp* m)
{
    void* bufs[14] = {m->X, m->H[0], m->H[1], m->H[2], m->A[0], m->A[1], m->A[2],
                      m->dH[0], m->dH[1], m->dH[2], m->Y, m->dY, m->part, m->wpart};
    for (void* b : bufs) {
        if (!b) continue;
        if (m->pins > 0) m->retired.push_back(b);
        else (void)hipFree(b);
    }
    m->X = nullptr; m->Y = nullptr; m->dY = nullptr; m->part = nullptr; m->wpart = nullptr;
    for (int i = 0; i < 3; ++i) { m->H[i] = nullptr; m->A[i] = nullptr; m->dH[i] = nullptr; }
    m->ws_rows = 0;
}

// Activation workspace for up to `rows` rows (grown on demand; the caller's
// stream is synchronised first so no launch still reads the old buffers).
ff_status ensure_ws(ff_mlp* m, int64_t rows, hipStream_t stream)
{
    if (rows <= m->ws_rows) return FF_OK;
    if (stream_capturing(stream))
        return set_error(FF_EINVAL, "network workspace must grow outside graph capture: run the same call "
                                    "once before capturing it");
    FF_HIP_TRY(hipStreamSynchronize(stream));
    free_ws(m);
    const int64_t R = cdiv(rows, 64) * 64;
    hipError_t e = hipMalloc(&m->X, (size_t)R * m->kin * sizeof(__bf16));
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        e = hipMalloc(&m->H[i], (size_t)R * m->h[i] * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&m->A[i], (size_t)R * m->h[i] * sizeof(__bf16));
        if (e == hipSuccess) e = hipMalloc(&m->dH[i], (size_t)R * m->h[i] * sizeof(__bf16));
    }
    if (e == hipSuccess) e = hipMalloc(&m->Y, (size_t)R * 16 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->dY, (size_t)R * 16 * sizeof(__bf16));
    if (e == hipSuccess) e = hipMalloc(&m->part, (size_t)(R / kColChunk) * 1024 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->wpart, (size_t)kWgradSplit * wgrad_max(m) * sizeof(float));
    if (e != hipSuccess) {
        free_ws(m);
        return hip_error(e, "mlp workspace");
    }
    m->ws_rows = R;
    return FF_OK;
}

template <bool TA, bool TB, int EPI>
void gemm(int M, int N, int Ml, int Nl, int K, const __bf16* A, int lda, const __bf16* B, int ldb,
          const EpiArgs& ep, hipStream_t s)
{
    dim3 grid((unsigned)cdiv(N, kBN), (unsigned)cdiv(M, kBM));
    hipLaunchKernelGGL((gemm_bf16<TA, TB, EPI>), grid, dim3(kGemmThreads), 0, s, M, N, Ml, Nl, K, A, lda, B, ldb, ep);
}

template <int EPI>
void gemm_fwd(int M, int N, int K, const __bf16* A, int lda, const __bf16* B, int ldb, const EpiArgs& ep,
              hipStream_t s)
{
    dim3 grid((unsigned)(N / kFN), (unsigned)cdiv(M, kFM));
    if (K % 32 == 0 && M >= 1) {
        const int64_t tiles = (int64_t)(N / kFN) * cdiv(M, kFM);
        const unsigned blocks = (unsigned)(cdiv(tiles, kXcds) * kXcds);
        hipLaunchKernelGGL((gemm_nt_lds<EPI>), dim3(blocks), dim3(kGemmThreads), 0, s, M, N, M, K, A, lda, B, ldb,
                           ep);
    } else
        hipLaunchKernelGGL((gemm_nt_128<EPI>), grid, dim3(kGemmThreads), 0, s, M, N, M, K, A, lda, B, ldb, ep);
}

// forward pass of R rows of features already in m->X; keep_h: store the
// pre-activations for the backward pass; mcount (may be null): only rows
// r < *mcount - mbase exist (see EpiArgs)
void forward_rows(const ff_mlp* m, int64_t R, bool keep_h, hipStream_t s, const int64_t* mcount = nullptr,
                  int64_t mbase = 0)
{
    const int r = (int)R;
    for (int l = 0; l < 3; ++l) {
        const __bf16* in = l == 0 ? m->X : m->A[l - 1];
        const int kin = m->map.in_pad[l];
        EpiArgs ep{m->params + m->map.off_b[l], m->H[l], m->h[l], m->A[l], m->h[l], nullptr, 0, mcount, mbase};
        const __bf16* w = m->wb + m->map.off_wb[l];
        if (m->h[l] % kFN == 0) {
            if (keep_h) gemm_fwd<EPI_FWD_GELU>(r, m->h[l], kin, in, kin, w, kin, ep, s);
            else gemm_fwd<EPI_FWD_GELU_NOH>(r, m->h[l], kin, in, kin, w, kin, ep, s);
        } else if (keep_h)
            gemm<false, true, EPI_FWD_GELU>(r, m->h[l], r, m->h[l], kin, in, kin, m->wb + m->map.off_wb[l], kin, ep, s);
        else
            gemm<false, true, EPI_FWD_GELU_NOH>(r, m->h[l], r, m->h[l], kin, in, kin, m->wb + m->map.off_wb[l], kin, ep, s);
    }
    EpiArgs ep{m->params + m->map.off_b[3], m->Y, 16, nullptr, 0, nullptr, 0, mcount, mbase};
    gemm<false, true, EPI_FWD_LINEAR>(r, m->n_out, r, 16, m->h[2], m->A[2], m->h[2], m->wb + m->map.off_wb[3],
                                      m->h[2], ep, s);
}

void colsum(ff_mlp* m, const __bf16* D, int64_t R, int N, int ld, float* out, hipStream_t s)
{
    const int chunks = (int)cdiv(R, kColChunk);
    hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)cdiv(N, 64), (unsigned)chunks), dim3(256), 0, s, D, R, N,
                       ld, m->part);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, s, m->part, chunks, N, out);
}

// Weight gradient gw[M][N] = sum_r Dop[r][m] Xop[r][n] over the R = K rows
// of the batch.  A batch's 2,048-row reduction into at most 512 x 512
// outputs is only 64 output tiles, a quarter of the CUs: the rows are split
// into S slices (at least 256 rows each), each slice's partial product goes
// to its own plane of m->wpart, and the planes are summed in a fixed order,
// so the result does not depend on scheduling.
void gemm_wgrad(ff_mlp* m, int M, int N, int Ml, int Nl, int K, const __bf16* D, int ldd, const __bf16* X, int ldx,
                float* gw, hipStream_t s)
{
    const int64_t tiles = cdiv(N, kBN) * cdiv(M, kBM);
    int S = (int)std::min<int64_t>({(int64_t)kWgradSplit, std::max<int64_t>(1, K / 256), cdiv(512, tiles)});
    if (S < 1) S = 1;
    if (S == 1) {
        gemm<true, false, EPI_F32>(M, N, Ml, Nl, K, D, ldd, X, ldx, EpiArgs{nullptr, gw, N, nullptr, 0, nullptr, 0}, s);
        return;
    }
    dim3 grid((unsigned)cdiv(N, kBN), (unsigned)cdiv(M, kBM), (unsigned)S);
    hipLaunchKernelGGL((gemm_bf16<true, false, EPI_F32>), grid, dim3(kGemmThreads), 0, s, M, N, Ml, Nl, K, D, ldd, X,
                       ldx, EpiArgs{nullptr, m->wpart, N, nullptr, 0, nullptr, 0});
    const int64_t n = (int64_t)M * N;
    hipLaunchKernelGGL(sum_planes_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, m->wpart, S, n, gw);
}

// backward pass of R rows: dY in m->dY -> all gradients into m->grads
void backward_rows(ff_mlp* m, int64_t R, hipStream_t s)
{
    const int r = (int)R;
    const int h1 = m->h[0], h2 = m->h[1], h3 = m->h[2];
    float* gw = m->grads;
    const LayerMap& mp = m->map;
    // output layer
    gemm_wgrad(m, m->n_out, h3, 16, h3, r, m->dY, 16, m->A[2], h3, gw + mp.off_w[3], s);
    colsum(m, m->dY, R, m->n_out, 16, gw + mp.off_b[3], s);
    gemm<false, false, EPI_BWD_GELU>(r, h3, r, h3, 16, m->dY, 16, m->wb + mp.off_wb[3], h3,
                                     EpiArgs{nullptr, nullptr, 0, m->dH[2], h3, m->H[2], h3}, s);
    // hidden layers 3, 2, 1
    const int hs[3] = {h1, h2, h3};
    for (int l = 2; l >= 0; --l) {
        const int nout = hs[l];
        const int nin = l == 0 ? m->n_in : hs[l - 1];
        const int nin_pad = mp.in_pad[l];
        const __bf16* xin = l == 0 ? m->X : m->A[l - 1];
        gemm_wgrad(m, nout, nin, nout, nin_pad, r, m->dH[l], nout, xin, nin_pad, gw + mp.off_w[l], s);
        colsum(m, m->dH[l], R, nout, nout, gw + mp.off_b[l], s);
        if (l > 0)
            gemm<false, false, EPI_BWD_GELU>(r, nin, r, nin, nout, m->dH[l], nout, m->wb + mp.off_wb[l], nin_pad,
                                             EpiArgs{nullptr, nullptr, 0, m->dH[l - 1], nin, m->H[l - 1], nin}, s);
    }
}

ff_status check_mlp(const ff_mlp* m, const char* what)
{
    if (!m) return set_error(FF_EINVAL, std::string(what) + ": NULL network");
    return FF_OK;
}

}  // namespace

extern "C" ff_status ff_mlp_create(int32_t n_in, int32_t h1, int32_t h2, int32_t h3, int32_t n_out, uint64_t seed,
                                   ff_mlp** out)
{
    if (!out) return set_error(FF_EINVAL, "ff_mlp_create: out is NULL");
    *out = nullptr;
    const int hs[3] = {h1, h2, h3};
    if (n_in < 1 || n_in > 1024 || n_out < 1 || n_out > 16)
        return set_error(FF_EINVAL, "ff_mlp_create: need 1 <= n_in <= 1024 and 1 <= n_out <= 16");
    for (int i = 0; i < 3; ++i)
        if (hs[i] < 64 || hs[i] > 1024 || hs[i] % 64)
            return set_error(FF_EINVAL, "ff_mlp_create: hidden sizes must be multiples of 64 in [64, 1024]");
    ff_mlp* m = new ff_mlp();
    hipGetDevice(&m->device);
    m->n_in = n_in;
    m->n_out = n_out;
    for (int i = 0; i < 3; ++i) m->h[i] = hs[i];
    m->kin = (int)cdiv(n_in, 32) * 32;
    const int ins[4] = {n_in, h1, h2, h3}, outs[4] = {h1, h2, h3, n_out};
    const int inp[4] = {m->kin, h1, h2, h3}, outp[4] = {h1, h2, h3, 16};
    int64_t off = 0, offb = 0;
    for (int l = 0; l < 4; ++l) {
        m->map.in_dim[l] = ins[l];
        m->map.out_dim[l] = outs[l];
        m->map.in_pad[l] = inp[l];
        m->map.off_w[l] = off;
        off += (int64_t)outs[l] * ins[l];
        m->map.off_b[l] = off;
        off += outs[l];
        m->map.off_wb[l] = offb;
        offb += (int64_t)outp[l] * inp[l];
    }
    m->n_params = off;
    m->n_wb = offb;
    // He-normal weights from Philox normals keyed by the seed; zero biases;
    // the output layer scaled by 0.1 so the initial z0 is near the box centre
    std::vector<float> p((size_t)off, 0.f);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int l = 0; l < 4; ++l) {
        const double sd = std::sqrt(2.0 / ins[l]) * (l == 3 ? 0.1 : 1.0);
        const int64_t nw = (int64_t)outs[l] * ins[l];
        for (int64_t i = 0; i < nw; i += 2) {
            const U32x4 r = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)l, 7u, k0, k1);
            const double rr = std::sqrt(-2.0 * std::log(u01(r.v[0])));
            const double th = 6.283185307179586 * u01(r.v[1]);
            p[(size_t)(m->map.off_w[l] + i)] = (float)(sd * rr * std::cos(th));
            if (i + 1 < nw) p[(size_t)(m->map.off_w[l] + i + 1)] = (float)(sd * rr * std::sin(th));
        }
    }
    std::vector<float> zeros_in((size_t)n_in, 0.f), ones_in((size_t)n_in, 1.f);
    hipError_t e = hipMalloc(&m->params, off * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->grads, off * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->adam_m, off * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->adam_v, off * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->wb, offb * sizeof(__bf16));
    if (e == hipSuccess) e = hipMalloc(&m->mean, n_in * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->inv_std, n_in * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->wb, 0, offb * sizeof(__bf16));
    if (e == hipSuccess) e = hipMemcpy(m->mean, zeros_in.data(), n_in * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->inv_std, ones_in.data(), n_in * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ff_mlp_destroy(m);
        return hip_error(e, "ff_mlp_create");
    }
    *out = m;
    ff_status s = ff_mlp_set_params(m, p.data());
    if (s != FF_OK) {
        ff_mlp_destroy(m);
        *out = nullptr;
        return s;
    }
    return clear_error();
}

extern "C" void ff_mlp_destroy(ff_mlp* m)
{
    if (!m) return;
    m->pins = 0;
    free_ws(m);
    for (void* b : m->retired) (void)hipFree(b);
    hipFree(m->params);
    hipFree(m->grads);
    hipFree(m->adam_m);
    hipFree(m->adam_v);
    hipFree(m->wb);
    hipFree(m->mean);
    hipFree(m->inv_std);
    delete m;
}

extern "C" int64_t ff_mlp_n_params(const ff_mlp* m) { return m ? m->n_params : 0; }

extern "C" ff_status ff_mlp_get_params(const ff_mlp* m, float* host)
{
    if (check_mlp(m, "ff_mlp_get_params") || !host) return set_error(FF_EINVAL, "ff_mlp_get_params: NULL argument");
    FF_HIP_TRY(hipMemcpy(host, m->params, m->n_params * sizeof(float), hipMemcpyDeviceToHost));
    return clear_error();
}

extern "C" ff_status ff_mlp_set_params(ff_mlp* m, const float* host)
{
    if (check_mlp(m, "ff_mlp_set_params") || !host) return set_error(FF_EINVAL, "ff_mlp_set_params: NULL argument");
    FF_HIP_TRY(hipMemcpy(m->params, host, m->n_params * sizeof(float), hipMemcpyHostToDevice));
    FF_HIP_TRY(hipMemset(m->adam_m, 0, m->n_params * sizeof(float)));
    FF_HIP_TRY(hipMemset(m->adam_v, 0, m->n_params * sizeof(float)));
    m->step = 0;
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((unsigned)cdiv(m->n_params, 256)), dim3(256), 0, 0, m->params,
                       m->n_params, m->wb, m->map);
    FF_HIP_TRY(hipGetLastError());
    FF_HIP_TRY(hipDeviceSynchronize());
    return clear_error();
}

extern "C" ff_status ff_mlp_set_normalization(ff_mlp* m, const float* mean, const float* inv_std, float floor_v)
{
    if (check_mlp(m, "ff_mlp_set_normalization") || !mean || !inv_std)
        return set_error(FF_EINVAL, "ff_mlp_set_normalization: NULL argument");
    if (!(floor_v > 0.f)) return set_error(FF_EINVAL, "ff_mlp_set_normalization: floor must be > 0");
    FF_HIP_TRY(hipMemcpy(m->mean, mean, m->n_in * sizeof(float), hipMemcpyHostToDevice));
    FF_HIP_TRY(hipMemcpy(m->inv_std, inv_std, m->n_in * sizeof(float), hipMemcpyHostToDevice));
    m->floor_v = floor_v;
    return clear_error();
}

extern "C" ff_status ff_mlp_get_normalization(const ff_mlp* m, float* mean, float* inv_std, float* floor_v)
{
    if (check_mlp(m, "ff_mlp_get_normalization") || !mean || !inv_std || !floor_v)
        return set_error(FF_EINVAL, "ff_mlp_get_normalization: NULL argument");
    FF_HIP_TRY(hipMemcpy(mean, m->mean, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
    FF_HIP_TRY(hipMemcpy(inv_std, m->inv_std, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
    *floor_v = m->floor_v;
    return clear_error();
}

extern "C" ff_status ff_mlp_fit_normalization(ff_mlp* m, const float* rad, int64_t P, float floor_v, void* stream)
{
    if (check_mlp(m, "ff_mlp_fit_normalization") || !rad || P <= 0 || !(floor_v > 0.f))
        return set_error(FF_EINVAL, "ff_mlp_fit_normalization: bad argument");
    m->floor_v = floor_v;
    hipLaunchKernelGGL(fit_norm_kernel, dim3(m->n_in), dim3(256), 0, (hipStream_t)stream, rad, P, m->n_in, floor_v,
                       m->mean, m->inv_std);
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

namespace ff {
void mlp_dims(const ff_mlp* m, int* n_in, int* n_out)
{
    *n_in = m ? m->n_in : 0;
    *n_out = m ? m->n_out : 0;
}

void mlp_pin(const ff_mlp* m, int delta)
{
    if (m) const_cast<ff_mlp*>(m)->pins += delta;
}
}  // namespace ff

extern "C" ff_status ff_mlp_infer(const ff_mlp* mc, const float* rad, int64_t P, float* z0, void* stream)
{
    if (check_mlp(mc, "ff_mlp_infer")) return FF_EINVAL;
    if (P < 0) return set_error(FF_EINVAL, "ff_mlp_infer: P < 0");
    if (P == 0) return clear_error();
    if (!rad || !z0) return set_error(FF_EINVAL, "ff_mlp_infer: NULL buffer");
    ff_mlp* m = const_cast<ff_mlp*>(mc);
    hipStream_t s = (hipStream_t)stream;
    const int64_t chunk = std::min<int64_t>(P, 1 << 18);
    ff_status st = ensure_ws(m, chunk, s);
    if (st != FF_OK) return st;
    for (int64_t p0 = 0; p0 < P; p0 += chunk) {
        const int64_t R = std::min(chunk, P - p0);
        hipLaunchKernelGGL(features_kernel, dim3((unsigned)cdiv(R * m->kin / 8, 256)), dim3(256), 0, s,
                           rad + p0 * m->n_in, (int)R, m->n_in, m->kin, m->mean, m->inv_std, m->floor_v, m->X);
        forward_rows(m, R, false, s);
        hipLaunchKernelGGL(output_kernel, dim3((unsigned)cdiv(R * m->n_out, 256)), dim3(256), 0, s, m->Y, R, m->n_out,
                           z0 + p0 * m->n_out);
    }
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

extern "C" ff_status ff_mlp_infer_listed(const ff_mlp* mc, const float* rad, int64_t P, const int64_t* index,
                                        int64_t n_listed, float* z0, void* stream)
{
    if (check_mlp(mc, "ff_mlp_infer_listed")) return FF_EINVAL;
    if (P < 0 || n_listed < 0) return set_error(FF_EINVAL, "ff_mlp_infer_listed: P < 0 or n_listed < 0");
    if (n_listed == 0 || P == 0) return clear_error();
    if (!rad || !index || !z0) return set_error(FF_EINVAL, "ff_mlp_infer_listed: NULL buffer");
    ff_mlp* m = const_cast<ff_mlp*>(mc);
    hipStream_t s = (hipStream_t)stream;
    const int64_t chunk = std::min<int64_t>(n_listed, 1 << 18);
    ff_status st = ensure_ws(m, chunk, s);
    if (st != FF_OK) return st;
    for (int64_t i0 = 0; i0 < n_listed; i0 += chunk) {
        const int64_t R = std::min(chunk, n_listed - i0);
        hipLaunchKernelGGL(features_listed_kernel, dim3((unsigned)cdiv(R * m->kin / 8, 256)), dim3(256), 0, s, rad,
                           index + i0, P, (int)R, m->n_in, m->kin, m->mean, m->inv_std, m->floor_v, m->X,
                           (const int64_t*)nullptr, (int64_t)0);
        forward_rows(m, R, false, s);
        hipLaunchKernelGGL(output_listed_kernel, dim3((unsigned)cdiv(R * m->n_out, 256)), dim3(256), 0, s, m->Y,
                           index + i0, P, R, m->n_out, z0, (const int64_t*)nullptr, (int64_t)0);
    }
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

namespace ff {

// z0 rows of the first *count_dev entries of index_dev (at most P) from the
// network; the row count is read on the device, so the launch sequence
// (sized for all P rows, chunks past the count doing nothing) can be
// captured into a graph.
ff_status mlp_infer_listed_dev(const ff_mlp* mc, const float* rad, int64_t P, const int64_t* index,
                               const int64_t* count_dev, float* z0, hipStream_t s)
{
    if (P <= 0) return FF_OK;
    ff_mlp* m = const_cast<ff_mlp*>(mc);
    const int64_t chunk = std::min<int64_t>(P, 1 << 18);
    ff_status st = ensure_ws(m, chunk, s);
    if (st != FF_OK) return st;
    for (int64_t i0 = 0; i0 < P; i0 += chunk) {
        const int64_t R = std::min(chunk, P - i0);
        hipLaunchKernelGGL(features_listed_kernel, dim3((unsigned)cdiv(R * m->kin / 8, 256)), dim3(256), 0, s, rad,
                           index + i0, P, (int)R, m->n_in, m->kin, m->mean, m->inv_std, m->floor_v, m->X, count_dev,
                           i0);
        forward_rows(m, R, false, s, count_dev, i0);
        hipLaunchKernelGGL(output_listed_kernel, dim3((unsigned)cdiv(R * m->n_out, 256)), dim3(256), 0, s, m->Y,
                           index + i0, P, R, m->n_out, z0, count_dev, i0);
    }
    FF_HIP_TRY(hipGetLastError());
    return FF_OK;
}

// Every row of z0 [P][n] marked "no start" (its first entry NaN).
__global__ void nan_rows_kernel(float* __restrict__ z0, int64_t P, int n)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) z0[p * n] = __builtin_nanf("");
}

ff_status mark_no_start(float* z0, int64_t P, int n, hipStream_t s)
{
    if (P <= 0) return FF_OK;
    hipLaunchKernelGGL(nan_rows_kernel, dim3((unsigned)cdiv(P, 256)), dim3(256), 0, s, z0, P, n);
    FF_HIP_TRY(hipGetLastError());
    return FF_OK;
}

}  // namespace ff

static ff_status grads_impl(ff_mlp* m, const float* rad, const float* target, int64_t P, double* loss,
                            hipStream_t s)
{
    ff_status st = ensure_ws(m, P, s);
    if (st != FF_OK) return st;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)cdiv(P * m->kin / 8, 256)), dim3(256), 0, s, rad, (int)P,
                       m->n_in, m->kin, m->mean, m->inv_std, m->floor_v, m->X);
    forward_rows(m, P, true, s);
    if (loss) hipLaunchKernelGGL(zero_f64, dim3(1), dim3(64), 0, s, loss);
    hipLaunchKernelGGL(loss_kernel, dim3((unsigned)cdiv(P, 256)), dim3(256), 0, s, m->Y, target, P, m->n_out, m->dY,
                       loss);
    backward_rows(m, P, s);
    FF_HIP_TRY(hipGetLastError());
    return FF_OK;
}

extern "C" ff_status ff_mlp_gradients(ff_mlp* m, const float* rad, const float* target, int64_t P, double* loss,
                                      float* grads, void* stream)
{
    if (check_mlp(m, "ff_mlp_gradients")) return FF_EINVAL;
    if (P <= 0 || P > 65536 || !rad || !target) return set_error(FF_EINVAL, "ff_mlp_gradients: bad batch");
    hipStream_t s = (hipStream_t)stream;
    ff_status st = grads_impl(m, rad, target, P, loss, s);
    if (st != FF_OK) return st;
    if (grads) FF_HIP_TRY(hipMemcpyAsync(grads, m->grads, m->n_params * sizeof(float), hipMemcpyDeviceToDevice, s));
    return clear_error();
}

extern "C" ff_status ff_mlp_train_step(ff_mlp* m, const float* rad, const float* target, int64_t P, float lr,
                                       double* loss, void* stream)
{
    if (check_mlp(m, "ff_mlp_train_step")) return FF_EINVAL;
    if (P <= 0 || P > 65536 || !rad || !target || !(lr >= 0.f))
        return set_error(FF_EINVAL, "ff_mlp_train_step: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    ff_status st = grads_impl(m, rad, target, P, loss, s);
    if (st != FF_OK) return st;
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)cdiv(m->n_params, 256)), dim3(256), 0, s, m->params, m->grads,
                       m->adam_m, m->adam_v, m->n_params, lr, b1, b2, eps, bc1, bc2, m->wb, m->map);
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

extern "C" ff_status ff_mlp_generate(const ff_scene* sc, const ff_prior* prior, uint64_t seed, uint64_t offset,
                                     int64_t P, double snr, double bg, float* rad, float* target, float* state,
                                     void* stream)
{
    if (!sc || !prior || prior->model != FF_MODEL_LOGNORMAL_1)
        return set_error(FF_EINVAL, "ff_mlp_generate: needs a scene and a one-component prior");
    if (P < 0 || !(bg >= 0.0 && bg <= 1.0)) return set_error(FF_EINVAL, "ff_mlp_generate: bad P or bg_fraction");
    if (P == 0) return clear_error();
    if (!rad || !target) return set_error(FF_EINVAL, "ff_mlp_generate: NULL output");
    GenArgs ga{};
    for (int j = 0; j < 5; ++j) {
        ga.lo[j] = prior->lo[j];
        ga.hi[j] = prior->hi[j];
        ga.x0[j] = prior->x0[j];
        if (!(ga.hi[j] > ga.lo[j])) return set_error(FF_EINVAL, "ff_mlp_generate: prior box");
    }
    ga.k0 = (uint32_t)seed;
    ga.k1 = (uint32_t)(seed >> 32);
    ga.offset = offset;
    ga.snr = snr;
    ga.bg = bg;
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    if (!ensure_quad<float, 32>(dev)) return set_error(FF_EDEVICE, "quadrature rule could not be placed on the device");
    const int chunks = gen_chunks(sc->n_bands);
    if (P * chunks / 256 + 1 > 0x7fffffff) return set_error(FF_EINVAL, "ff_mlp_generate: P too large");
    hipLaunchKernelGGL(generate_kernel<32>, dim3((unsigned)cdiv(P * chunks, 256)), dim3(256), 0, (hipStream_t)stream,
                       sc->table_f32, sc->n_bands, P, chunks, ga, rad, target, state);
    FF_HIP_TRY(hipGetLastError());
    return clear_error();
}

extern "C" ff_status ff_mlp_train_span(ff_mlp* m, const ff_scene* sc, const ff_prior* prior, int64_t total_steps,
                                       int64_t first_step, int64_t n_steps, int32_t batch, uint64_t seed, double snr,
                                       double bg, float lr, float lr_final, double* loss_hist, void* stream)
{
    if (check_mlp(m, "ff_mlp_train_span")) return FF_EINVAL;
    if (!sc || sc->n_bands != m->n_in) return set_error(FF_EINVAL, "ff_mlp_train_span: scene band count != n_in");
    if (total_steps < 0 || first_step < 0 || n_steps < 0 || first_step + n_steps > total_steps || batch <= 0 ||
        batch > 65536)
        return set_error(FF_EINVAL, "ff_mlp_train_span: need 0 <= first_step <= first_step + n_steps <= total_steps "
                                    "and 0 < batch <= 65536");
    const int64_t steps = total_steps;
    hipStream_t s = (hipStream_t)stream;
    // The spectra of up to kGenPool steps are generated by one launch (sample
    // g = i batch + p of step i, the same counter-based stream as one launch
    // per step), which fills the chip where a single batch would not.
    const int64_t pool = std::max<int64_t>(1, std::min<int64_t>(kGenPool, n_steps));
    float* rad = nullptr;
    float* tgt = nullptr;
    FF_HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&rad), (size_t)pool * batch * m->n_in * sizeof(float), s));
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&tgt), (size_t)pool * batch * 5 * sizeof(float), s);
    ff_status st = e == hipSuccess ? FF_OK : hip_error(e, "ff_mlp_train");
    for (int64_t i = first_step; i < first_step + n_steps && st == FF_OK; ++i) {
        const int64_t j = (i - first_step) % pool;
        if (j == 0) {
            const int64_t n = std::min<int64_t>(pool, first_step + n_steps - i);
            st = ff_mlp_generate(sc, prior, seed, (uint64_t)i * (uint64_t)batch, n * batch, snr, bg, rad, tgt, nullptr,
                                 s);
            if (st != FF_OK) break;
        }
        const double c = steps > 1 ? 0.5 * (1.0 + std::cos(M_PI * (double)i / (double)(steps - 1))) : 1.0;
        const float lr_i = (float)(lr_final + (lr - lr_final) * c);
        st = ff_mlp_train_step(m, rad + (size_t)j * batch * m->n_in, tgt + (size_t)j * batch * 5, batch, lr_i,
                               loss_hist ? loss_hist + (i - first_step) : nullptr, s);
        if (st == FF_OK) m->train_steps = i + 1;
    }
    hipFreeAsync(rad, s);
    hipFreeAsync(tgt, s);
    if (st != FF_OK) return st;
    return clear_error();
}

extern "C" ff_status ff_mlp_train(ff_mlp* m, const ff_scene* sc, const ff_prior* prior, int64_t steps, int32_t batch,
                                  uint64_t seed, double snr, double bg, float lr, float lr_final,
                                  double* loss_hist, void* stream)
{
    return ff_mlp_train_span(m, sc, prior, steps, 0, steps, batch, seed, snr, bg, lr, lr_final, loss_hist, stream);
}

extern "C" int64_t ff_mlp_steps_done(const ff_mlp* m) { return m ? m->train_steps : -1; }

extern "C" ff_status ff_mlp_sizes(const ff_mlp* m, int32_t* sizes_host)
{
    if (check_mlp(m, "ff_mlp_sizes") || !sizes_host) return set_error(FF_EINVAL, "ff_mlp_sizes: NULL argument");
    sizes_host[0] = m->n_in;
    for (int i = 0; i < 3; ++i) sizes_host[1 + i] = m->h[i];
    sizes_host[4] = m->n_out;
    return clear_error();
}

// ---------------------------------------------------------------- checkpoints
// File layout (little-endian): "FFWS" magic, u32 version 1, i32 n_in, h1,
// h2, h3, n_out, f32 floor, i64 Adam step, i64 schedule steps, i64 n_params,
// then f32 params, Adam first and second moments [n_params] each, mean and
// inv_std [n_in].  The BF16 copies are rebuilt from the FP32 master weights.
namespace {
constexpr char kMagic[4] = {'F', 'F', 'W', 'S'};
constexpr uint32_t kVersion = 1;
}  // namespace

extern "C" ff_status ff_warmstart_save(const ff_mlp* m, const char* path)
{
    if (check_mlp(m, "ff_warmstart_save") || !path) return set_error(FF_EINVAL, "ff_warmstart_save: NULL argument");
    FF_HIP_TRY(hipSetDevice(m->device));
    FF_HIP_TRY(hipDeviceSynchronize());
    const size_t np = (size_t)m->n_params;
    std::vector<float> buf(3 * np + 2 * (size_t)m->n_in);
    FF_HIP_TRY(hipMemcpy(buf.data(), m->params, np * sizeof(float), hipMemcpyDeviceToHost));
    FF_HIP_TRY(hipMemcpy(buf.data() + np, m->adam_m, np * sizeof(float), hipMemcpyDeviceToHost));
    FF_HIP_TRY(hipMemcpy(buf.data() + 2 * np, m->adam_v, np * sizeof(float), hipMemcpyDeviceToHost));
    FF_HIP_TRY(hipMemcpy(buf.data() + 3 * np, m->mean, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
    FF_HIP_TRY(hipMemcpy(buf.data() + 3 * np + m->n_in, m->inv_std, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(FF_EINVAL, std::string("ff_warmstart_save: cannot open ") + path);
    const int32_t dims[5] = {m->n_in, m->h[0], m->h[1], m->h[2], m->n_out};
    const int64_t counts[3] = {m->step, m->train_steps, m->n_params};
    bool ok = std::fwrite(kMagic, 1, 4, f) == 4 && std::fwrite(&kVersion, 4, 1, f) == 1 &&
              std::fwrite(dims, 4, 5, f) == 5 && std::fwrite(&m->floor_v, 4, 1, f) == 1 &&
              std::fwrite(counts, 8, 3, f) == 3 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return set_error(FF_EDEVICE, std::string("ff_warmstart_save: write failed: ") + path);
    return clear_error();
}

extern "C" ff_status ff_warmstart_load(const char* path, ff_mlp** out)
{
    if (!path || !out) return set_error(FF_EINVAL, "ff_warmstart_load: NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(FF_EINVAL, std::string("ff_warmstart_load: cannot open ") + path);
    char magic[4];
    uint32_t version = 0;
    int32_t dims[5];
    float floor_v = 0.f;
    int64_t counts[3];
    bool ok = std::fread(magic, 1, 4, f) == 4 && std::memcmp(magic, kMagic, 4) == 0 &&
              std::fread(&version, 4, 1, f) == 1 && version == kVersion && std::fread(dims, 4, 5, f) == 5 &&
              std::fread(&floor_v, 4, 1, f) == 1 && std::fread(counts, 8, 3, f) == 3;
    if (!ok) {
        std::fclose(f);
        return set_error(FF_EINVAL, std::string("ff_warmstart_load: not a warm-start checkpoint: ") + path);
    }
    ff_mlp* m = nullptr;
    ff_status st = ff_mlp_create(dims[0], dims[1], dims[2], dims[3], dims[4], 0, &m);
    if (st != FF_OK) {
        std::fclose(f);
        return st;
    }
    const size_t np = (size_t)m->n_params;
    std::vector<float> buf(3 * np + 2 * (size_t)m->n_in);
    ok = counts[2] == m->n_params && counts[0] >= 0 && counts[1] >= 0 &&
         std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) {
        ff_mlp_destroy(m);
        return set_error(FF_EINVAL, std::string("ff_warmstart_load: truncated or inconsistent checkpoint: ") + path);
    }
    st = ff_mlp_set_params(m, buf.data());          // rebuilds the BF16 copies, clears Adam
    if (st == FF_OK) st = ff_mlp_set_normalization(m, buf.data() + 3 * np, buf.data() + 3 * np + m->n_in, floor_v);
    if (st == FF_OK) {
        hipError_t e = hipMemcpy(m->adam_m, buf.data() + np, np * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->adam_v, buf.data() + 2 * np, np * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) st = hip_error(e, "ff_warmstart_load");
    }
    if (st != FF_OK) {
        ff_mlp_destroy(m);
        return st;
    }
    m->step = counts[0];
    m->train_steps = counts[1];
    *out = m;
    return clear_error();
}
