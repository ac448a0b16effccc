// Device-side forward model of the fire-temperature inversion (Keely et al.,
// Sec. 2.2): solar term (eq. solar) over a linear or endmember-mixture
// surface, thermal term (eq. thermal) with a lognormal (or two-lognormal
// mixture) sub-pixel temperature density integrated by Gauss-Hermite
// quadrature in log T, or the paper's two Gaussians summed over a uniform
// temperature grid, and the per-band basis from which the Jacobian follows.
//
// Range-safe Planck: with x2 = a2 / T (a2 = c2 / lambda * log2 e) and
// e = 2^(-x2) in (0, 1],
//   B       = cb * e / (1 - e)                 (cb = c1 lambda^-5 per nm)
//   T dB/dT = cj * x2 * e / (1 - e)^2          (cj = cb ln 2)
// x2 runs from ~1e-3 (hottest quadrature node of the widest distribution,
// longest band) to ~4e4 (coldest node, shortest band).  The FP64 path forms
// e directly (it underflows to 0 for large x2); the FP32 path forms
// e / (1 - e) as 1 / (2^x2 - 1), where 2^x2 overflows to +inf for x2 > 128
// and the reciprocal returns the exact limit 0.
#pragma once

#include <algorithm>
#include <mutex>

#include "ff_internal.hpp"

#ifndef FF_NODE_GROUP
#define FF_NODE_GROUP 8
#endif

namespace ff {

template <int MODEL> struct ModelDims;
template <> struct ModelDims<FF_MODEL_LOGNORMAL_1> { static constexpr int N = 5; static constexpr int C = 1; };
template <> struct ModelDims<FF_MODEL_LOGNORMAL_2> { static constexpr int N = 8; static constexpr int C = 2; };
template <> struct ModelDims<FF_MODEL_GAUSS_GRID_2> { static constexpr int N = 8; static constexpr int C = 2; };
template <> struct ModelDims<FF_MODEL_ENDMEMBER_1> { static constexpr int N = 8; static constexpr int C = 1; };
template <> struct ModelDims<FF_MODEL_FULL> { static constexpr int N = 11; static constexpr int C = 2; };

// First state index of a block of surface fractions on the unit simplex
// (x = (z + 1)/2 per fraction, box [0, 1]), or -1 when the model has none.
template <int MODEL>
constexpr int simplex_first_v = MODEL == FF_MODEL_ENDMEMBER_1 ? 3 : (MODEL == FF_MODEL_FULL ? 6 : -1);

// Models whose thermal term is the Gaussian mixture on the temperature grid.
template <int MODEL>
constexpr bool grid_thermal_v = MODEL == FF_MODEL_GAUSS_GRID_2 || MODEL == FF_MODEL_FULL;

// Quadrature rule of order Q in constant memory (filled once per device by
// the host before the first launch).  Kernels index it with a laundered zero
// offset so each use is a scalar load at the point of use.
// (internal linkage: one instance per translation unit, see ensure_quad)
namespace {
template <typename R, int Q>
__constant__ Quad<R, Q> c_quad;
}

__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// packed lower triangle, (i, j) with j <= i
__host__ __device__ constexpr int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// Lognormal of mean m and s.d. s: log T ~ N(mu, sig^2), sig^2 = ln(1 + s^2/m^2),
// mu = ln m - sig^2 / 2; and d(mu, sig)/d(m, s).
struct LogNormal {
    double mu, sig, dmu_dm, dmu_ds, dsig_dm, dsig_ds;
};

__device__ inline LogNormal lognormal(double m, double s)
{
    LogNormal r;
    const double q = m * m + s * s;
    const double sig2 = log1p(s * s / (m * m));
    r.sig = sqrt(sig2);
    r.mu = log(m) - 0.5 * sig2;
    const double ds2_dm = -2.0 * s * s / (m * q);
    const double ds2_ds = 2.0 * s / q;
    r.dmu_dm = 1.0 / m - 0.5 * ds2_dm;
    r.dmu_ds = -0.5 * ds2_ds;
    r.dsig_dm = ds2_dm / (2.0 * r.sig);
    r.dsig_ds = ds2_ds / (2.0 * r.sig);
    return r;
}

// Cold-end nodes left out of the FP32 quadrature sums.  The rule's nodes are
// in ascending abscissa, so node k < c (c the largest weight) is colder than
// node c: x_k > x_c.  q(x) = 1/(2^x - 1) and y(x) = x q (1 + q) both fall
// strictly with x (dy/dx = y/x (1 - z coth(z/2)), z = x ln 2, and
// z coth(z/2) >= 2), so w_k q_k <= (w_k / w_c) w_c q_c and w_k y_k <=
// (w_k / w_c) w_c y_c, and |v_k| y_k <= |s_k| (w_k / w_c) w_c y_c with
// |s_k| < 11.  The first kColdSkip nodes have w_k / w_c < 2^-32 (checked on
// the host when the rule is built): leaving them out changes sI and sM by
// less than 2^-29 of themselves and sS by less than 2^-26 of sM's scale, below
// the rounding of an FP32 sum (2^-24).  The FP64 sums keep every node.
template <int Q>
constexpr int kColdSkip = Q >= 32 ? 5 : (Q >= 24 ? 2 : 0);
constexpr double kColdSkipRatio = 2.3283064365386963e-10;   // 2^-32

template <typename R, int Q>
constexpr int cold_skip_v = sizeof(R) == 4 ? kColdSkip<Q> : 0;

// Inverse node temperatures u_k = 1 / T_k = exp(-mu - sqrt2 x_k sig), formed
// in FP64 and rounded once to R (the FP32 rule's skipped cold nodes are not
// formed).
template <typename R, int Q>
__device__ inline void node_inverse_temperatures(const LogNormal& ln, R (&u)[Q])
{
    // one node at a time (each exponent depends, through an empty asm, on the
    // previous node's result): interleaving Q FP64 exponentials would hold
    // ~3Q registers in a prologue that runs once per evaluation
    const int o = opaque_zero();
    double mu = ln.mu;
#pragma unroll
    for (int k = 0; k < cold_skip_v<R, Q>; ++k) u[k] = (R)0;
#pragma unroll
    for (int k = cold_skip_v<R, Q>; k < Q; ++k) {
        u[k] = (R)exp(-mu - (double)c_quad<R, Q>.s[k + o] * ln.sig);
        asm volatile("" : "+v"(mu) : "v"(u[k]));
    }
}

// Quadrature sums over the nodes of one component at one band:
//   sI = sum_k w_k e/(1-e),  sM = sum_k w_k x2 e/(1-e)^2,  sS = sum_k v_k x2 e/(1-e)^2
// (w_k = GH weight / sqrt(pi), v_k = sqrt2 x_k w_k, e = 2^-x2).  Then
//   I = cb sI,  dI/dmu = cj sM,  dI/dsig = cj sS.
// FP32: q = e/(1-e) is taken as 1/(2^x2 - 1): for x2 > 128 the power is +inf
// and the reciprocal returns the exact limit 0, so no overflow handling is
// needed; 2 transcendental (exp2, rcp) + 7 VALU per node.  The first
// kColdSkip<Q> nodes are left out (bound above).
template <int Q>
__device__ __forceinline__ void thermal_sums(float a2, const float (&u)[Q], int o,
                                             float& sI, float& sM, float& sS)
{
    // Nodes are processed in groups of kGroup.  An empty asm after each group
    // makes the next group's exponent depend on this group's last reciprocal,
    // so the compiler cannot hoist all Q exponentials ahead of the sums (which
    // would keep ~2Q temporaries live); the FMA chains still overlap the
    // next group's transcendentals.
    constexpr int kGroup = FF_NODE_GROUP;
    const Quad<float, Q>& qd = c_quad<float, Q>;
    float i0 = 0.f, m0 = 0.f, s0 = 0.f;
    float a = a2;
    constexpr int k0 = kColdSkip<Q>;
#pragma unroll
    for (int k = k0; k < Q; ++k) {
        const float x = a * u[k];
        const float q = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(x) - 1.0f);
        const float wk = qd.w[k + o], vk = qd.v[k + o];
        i0 = __builtin_fmaf(wk, q, i0);
        const float y = x * __builtin_fmaf(q, q, q);   // x q (1 + q) = x e / (1 - e)^2
        m0 = __builtin_fmaf(wk, y, m0);
        s0 = __builtin_fmaf(vk, y, s0);
        if ((k + 1 - k0) % kGroup == 0) asm volatile("" : "+v"(a) : "v"(i0), "v"(m0), "v"(s0));
    }
    sI = i0;
    sM = m0;
    sS = s0;
}

template <int Q>
__device__ __forceinline__ void thermal_sums(double a2, const double (&u)[Q], int o,
                                             double& sI, double& sM, double& sS)
{
    const Quad<double, Q>& qd = c_quad<double, Q>;
    double i0 = 0.0, m0 = 0.0, s0 = 0.0;
#pragma unroll 4
    for (int k = 0; k < Q; ++k) {
        const double x = a2 * u[k];
        const double e = exp2(-x);
        const double r = 1.0 / (1.0 - e);
        const double q = e * r;
        const double wk = qd.w[k + o], vk = qd.v[k + o];
        i0 = fma(wk, q, i0);
        const double y = x * fma(q, q, q);
        m0 = fma(wk, y, m0);
        s0 = fma(vk, y, s0);
    }
    sI = i0;
    sM = m0;
    sS = s0;
}

template <typename R> __device__ __forceinline__ R fast_rcp(R x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }

// One band row of the scene table (see TableCol).
template <typename R>
struct BandRow {
    R K, tau2, tup, ratm, S, lsat, a2, cb, cj, dl;
};

__device__ __forceinline__ BandRow<float> load_row(const float* __restrict__ t)
{
    const float4 p0 = *reinterpret_cast<const float4*>(t);
    const float4 p1 = *reinterpret_cast<const float4*>(t + 4);
    const float4 p2 = *reinterpret_cast<const float4*>(t + 8);
    BandRow<float> r;
    r.K = p0.y; r.tau2 = p0.z; r.tup = p0.w;
    r.ratm = p1.x; r.S = p1.y; r.lsat = p1.z; r.a2 = p1.w;
    r.cb = p2.x; r.cj = p2.y; r.dl = p2.z;
    return r;
}

__device__ __forceinline__ BandRow<double> load_row(const double* __restrict__ t)
{
    const double2 p0 = *reinterpret_cast<const double2*>(t);
    const double2 p1 = *reinterpret_cast<const double2*>(t + 2);
    const double2 p2 = *reinterpret_cast<const double2*>(t + 4);
    const double2 p3 = *reinterpret_cast<const double2*>(t + 6);
    const double2 p4 = *reinterpret_cast<const double2*>(t + 8);
    const double2 p5 = *reinterpret_cast<const double2*>(t + 10);
    BandRow<double> r;
    r.K = p0.y; r.tau2 = p1.x; r.tup = p1.y;
    r.ratm = p2.x; r.S = p2.y; r.lsat = p3.x; r.a2 = p3.y;
    r.cb = p4.x; r.cj = p4.y; r.dl = p5.x;
    (void)p5;
    return r;
}

// Endmember row b of a scene table (the library section after the band rows).
template <typename R>
struct EndmRow {
    R e[FF_N_ENDMEMBERS];
};

__device__ __forceinline__ EndmRow<float> load_endm(const float* __restrict__ t)
{
    const float4 p0 = *reinterpret_cast<const float4*>(t);
    EndmRow<float> r;
    r.e[0] = p0.x; r.e[1] = p0.y; r.e[2] = p0.z; r.e[3] = p0.w;
    r.e[4] = t[4];
    return r;
}

__device__ __forceinline__ EndmRow<double> load_endm(const double* __restrict__ t)
{
    const double2 p0 = *reinterpret_cast<const double2*>(t);
    const double2 p1 = *reinterpret_cast<const double2*>(t + 2);
    EndmRow<double> r;
    r.e[0] = p0.x; r.e[1] = p0.y; r.e[2] = p1.x; r.e[3] = p1.y;
    r.e[4] = t[4];
    return r;
}

// Per-pixel constants of one model evaluation.
// Broadcast the value of lane M of each aligned group of G lanes (G = 2 or 4,
// so a group lies inside a quad) to the whole group: one DPP quad_perm move
// per 32-bit word.
template <int G, int M>
struct QuadBcast {
    static constexpr int ctrl = G == 4 ? M * 0x55 : (M | (M << 2) | ((2 + M) << 4) | ((2 + M) << 6));
    __device__ static __forceinline__ float run(float v)
    {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
    }
    __device__ static __forceinline__ double run(double v)
    {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), ctrl, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, false);
        return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    }
};

template <int G, int M, typename R, int Q>
__device__ __forceinline__ void fill_from_group(R (&u)[Q], int base, R t)
{
    u[base + M] = QuadBcast<G, M>::run(t);
    if constexpr (M + 1 < G) fill_from_group<G, M + 1>(u, base, t);
}

// The same node temperatures computed by G cooperating lanes (lane `sub` of
// an aligned group of G = 2 or 4 forms nodes j G + sub) and gathered with
// DPP: every lane ends with the values node_inverse_temperatures gives.
template <typename R, int Q, int G>
__device__ inline void node_inverse_temperatures_split(const LogNormal& ln, R (&u)[Q], int sub)
{
    static_assert(Q % G == 0, "node count must divide among the group");
    const int o = opaque_zero();
    double mu = ln.mu;
    constexpr int j0 = cold_skip_v<R, Q> / G;
#pragma unroll
    for (int k = 0; k < j0 * G; ++k) u[k] = (R)0;
#pragma unroll
    for (int j = j0; j < Q / G; ++j) {
        double sk = (double)c_quad<R, Q>.s[j * G + o];
#pragma unroll
        for (int m = 1; m < G; ++m) sk = sub == m ? (double)c_quad<R, Q>.s[j * G + m + o] : sk;
        const R t = (R)exp(-mu - sk * ln.sig);
        asm volatile("" : "+v"(mu) : "v"(t));
        fill_from_group<G, 0>(u, j * G, t);
    }
}

// Node temperatures for a pixel evaluated by L lanes: the work is split
// among the lanes of each quad of the group (L >= 4: four ways, L = 2: two).
template <typename R, int Q>
__device__ __forceinline__ void node_inverse_temperatures_lanes(const LogNormal& ln, R (&u)[Q], int lane, int L)
{
    if (L >= 4) node_inverse_temperatures_split<R, Q, 4>(ln, u, lane & 3);
    else if (L == 2) node_inverse_temperatures_split<R, Q, 2>(ln, u, lane & 1);
    else node_inverse_temperatures<R, Q>(ln, u);
}

template <typename R, int MODEL, int Q> struct PixelModel;

template <typename R, int Q>
struct PixelModel<R, FF_MODEL_LOGNORMAL_1, Q> {
    static constexpr int N = 5;
    R f, r0, r1;
    R u[Q];
    // lane / L: this lane and the number of lanes evaluating the pixel
    __device__ void setup(const double (&x)[N], int lane = 0, int L = 1)
    {
        f = (R)x[0];
        r0 = (R)x[3];
        r1 = (R)x[4];
        node_inverse_temperatures_lanes<R, Q>(lognormal(x[1], x[2]), u, lane, L);
    }
    // Basis u_b (J row = -D M u_b) and model radiance at one band.  S0: the
    // table's S is 0 on every band, so 1/(1 - S rho) is 1 (the reciprocal of
    // exactly 1 is exactly 1 on this hardware) and is not formed.
    template <bool S0 = false>
    __device__ __forceinline__ R band(const BandRow<R>& t, int o, R (&ub)[N]) const
    {
        R sI, sM, sS;
        thermal_sums<Q>(t.a2, u, o, sI, sM, sS);
        const R rho = r0 + r1 * t.dl;
        const R rden = S0 ? (R)1 : fast_rcp<R>((R)1 - t.S * rho);
        const R ls = t.K * (t.ratm + t.tau2 * rho * rden);
        ub[0] = t.tup * t.cb * sI;
        ub[1] = t.tup * t.cj * sM;
        ub[2] = t.tup * t.cj * sS;
        ub[3] = t.K * t.tau2 * rden * rden;
        ub[4] = ub[3] * t.dl;
        return ls + f * ub[0];
    }
    // Coefficients of the physical Jacobian rows in the basis:
    // dL/dx_i = c1_i u[s1_i] + c2_i u[s2_i].
    static constexpr int s1[N] = {0, 1, 1, 3, 4};
    static constexpr int s2[N] = {-1, 2, 2, -1, -1};
    __device__ static void coefficients(const double (&x)[N], double (&c1)[N], double (&c2)[N])
    {
        const LogNormal l = lognormal(x[1], x[2]);
        const double f = x[0];
        c1[0] = 1.0; c2[0] = 0.0;
        c1[1] = f * l.dmu_dm; c2[1] = f * l.dsig_dm;
        c1[2] = f * l.dmu_ds; c2[2] = f * l.dsig_ds;
        c1[3] = 1.0; c2[3] = 0.0;
        c1[4] = 1.0; c2[4] = 0.0;
    }
    __device__ static void moments(const double (&x)[N], double& et, double& sd)
    {
        et = x[1];
        sd = x[2];
    }
};

// One lognormal fire component over the endmember surface (Sec. 2.2,
// library Sec. 2.4): rho = sum_k x_k E_k, dL/dx_k = K tau2 E_k / (1 - S rho)^2.
template <typename R, int Q>
struct PixelModel<R, FF_MODEL_ENDMEMBER_1, Q> {
    static constexpr int N = 8;
    static constexpr int NE = FF_N_ENDMEMBERS;
    R f, xs[NE];
    R u[Q];
    __device__ void setup(const double (&x)[N], int lane = 0, int L = 1)
    {
        f = (R)x[0];
#pragma unroll
        for (int k = 0; k < NE; ++k) xs[k] = (R)x[3 + k];
        node_inverse_temperatures_lanes<R, Q>(lognormal(x[1], x[2]), u, lane, L);
    }
    __device__ __forceinline__ R band(const BandRow<R>& t, const EndmRow<R>& em, int o, R (&ub)[N]) const
    {
        R sI, sM, sS;
        thermal_sums<Q>(t.a2, u, o, sI, sM, sS);
        R rho = xs[0] * em.e[0];
#pragma unroll
        for (int k = 1; k < NE; ++k) rho += xs[k] * em.e[k];
        const R rden = fast_rcp<R>((R)1 - t.S * rho);
        const R ls = t.K * (t.ratm + t.tau2 * rho * rden);
        ub[0] = t.tup * t.cb * sI;
        ub[1] = t.tup * t.cj * sM;
        ub[2] = t.tup * t.cj * sS;
        const R ds = t.K * t.tau2 * rden * rden;
#pragma unroll
        for (int k = 0; k < NE; ++k) ub[3 + k] = ds * em.e[k];
        return ls + f * ub[0];
    }
    static constexpr int s1[N] = {0, 1, 1, 3, 4, 5, 6, 7};
    static constexpr int s2[N] = {-1, 2, 2, -1, -1, -1, -1, -1};
    __device__ static void coefficients(const double (&x)[N], double (&c1)[N], double (&c2)[N])
    {
        const LogNormal l = lognormal(x[1], x[2]);
        const double f = x[0];
        c1[0] = 1.0; c2[0] = 0.0;
        c1[1] = f * l.dmu_dm; c2[1] = f * l.dsig_dm;
        c1[2] = f * l.dmu_ds; c2[2] = f * l.dsig_ds;
#pragma unroll
        for (int k = 3; k < N; ++k) { c1[k] = 1.0; c2[k] = 0.0; }
    }
    __device__ static void moments(const double (&x)[N], double& et, double& sd)
    {
        et = x[1];
        sd = x[2];
    }
};

// Model radiance and basis at band b of a scene table (tab: band rows, then
// for the endmember model the library rows); row receives the band row.
template <int MODEL, bool S0 = false, typename PM, typename R>
__device__ __forceinline__ R band_of(const PM& pm, const R* __restrict__ tab, int B, int b, int o,
                                     const BandRow<R>& row, R (&ub)[PM::N])
{
    static_assert(!S0 || MODEL == FF_MODEL_LOGNORMAL_1, "the S = 0 path exists for the one-component model");
    // grid models: the band's row of grid Planck ratios (FP32 tables only)
    const R* qrow = tab + (size_t)B * (FF_TABLE_COLS + kEndmCols) + (size_t)b * kGridNodes;
    if constexpr (grid_thermal_v<MODEL> && simplex_first_v<MODEL> >= 0)
        return pm.band(row, load_endm(tab + (size_t)B * FF_TABLE_COLS + (size_t)b * kEndmCols), o, ub, qrow);
    else if constexpr (grid_thermal_v<MODEL>)
        return pm.band(row, o, ub, qrow);
    else if constexpr (simplex_first_v<MODEL> >= 0)
        return pm.band(row, load_endm(tab + (size_t)B * FF_TABLE_COLS + (size_t)b * kEndmCols), o, ub);
    else if constexpr (S0)
        return pm.template band<true>(row, o, ub);
    else
        return pm.band(row, o, ub);
}

// Surface variables of a model: the trailing NS state variables, (rho0,
// rho1) of the linear reflectance or the endmember fractions.
template <int MODEL>
struct SurfaceDims {
    static constexpr int NS = simplex_first_v<MODEL> >= 0 ? FF_N_ENDMEMBERS : 2;
};

// Solar term of eq. (solar) at band b in FP64:
//   L_s = K [rho_atm + tau2 rho / (1 - S rho)],
// rho = rho0 + rho1 (lambda - 1440 nm) or sum_k x_k E_k, from the scene's
// FP64 table (band rows, then the library rows) and the FP64 surface
// variables sv.  1/(1 - S rho) is the FP32 reciprocal refined by one Newton
// step (relative error ~1e-14; exactly 1 when S rho = 0).  S0 (S = 0 on every
// band): the reciprocal is the caller's `one`, an opaque 1, so the FMA and
// its rounding are those of the general path.
template <int MODEL, bool S0 = false>
__device__ __forceinline__ double solar_fp64(const double* __restrict__ t64, int B, int b,
                                             const double (&sv)[SurfaceDims<MODEL>::NS], double one = 1.0)
{
    const double* row = t64 + (size_t)b * FF_TABLE_COLS;
    const double2 p0 = *reinterpret_cast<const double2*>(row);       // lambda, K
    const double2 p1 = *reinterpret_cast<const double2*>(row + 2);   // tau2, tau_up
    const double2 p2 = *reinterpret_cast<const double2*>(row + 4);   // rho_atm, S
    double rho;
    if constexpr (simplex_first_v<MODEL> >= 0) {
        const double* e = t64 + (size_t)B * FF_TABLE_COLS + (size_t)b * kEndmCols;
        const double2 e01 = *reinterpret_cast<const double2*>(e);
        const double2 e23 = *reinterpret_cast<const double2*>(e + 2);
        const double e4 = e[4];
        rho = sv[0] * e01.x;
        rho = fma(sv[1], e01.y, rho);
        rho = fma(sv[2], e23.x, rho);
        rho = fma(sv[3], e23.y, rho);
        rho = fma(sv[4], e4, rho);
    } else {
        const double dl = row[10];
        rho = fma(sv[1], dl, sv[0]);
    }
    if constexpr (S0) {
        return p0.y * fma(p1.x * rho, one, p2.x);
    } else {
        (void)one;
        const double den = fma(-p2.y, rho, 1.0);
        const double r0 = (double)__builtin_amdgcn_rcpf((float)den);
        const double rden = fma(r0, fma(-den, r0, 1.0), r0);
        return p0.y * fma(p1.x * rho, rden, p2.x);
    }
}

template <typename R, int Q>
struct PixelModel<R, FF_MODEL_LOGNORMAL_2, Q> {
    static constexpr int N = 8;
    R f, eta, r0, r1;
    R us[Q], uh[Q];
    __device__ void setup(const double (&x)[N], int lane = 0, int L = 1)
    {
        f = (R)x[0];
        eta = (R)x[1];
        r0 = (R)x[6];
        r1 = (R)x[7];
        node_inverse_temperatures_lanes<R, Q>(lognormal(x[2], x[3]), us, lane, L);
        node_inverse_temperatures_lanes<R, Q>(lognormal(x[4], x[5]), uh, lane, L);
    }
    __device__ __forceinline__ R band(const BandRow<R>& t, int o, R (&ub)[N]) const
    {
        R sIs, sMs, sSs, sIh, sMh, sSh;
        thermal_sums<Q>(t.a2, us, o, sIs, sMs, sSs);
        thermal_sums<Q>(t.a2, uh, o, sIh, sMh, sSh);
        const R rho = r0 + r1 * t.dl;
        const R rden = fast_rcp<R>((R)1 - t.S * rho);
        const R ls = t.K * (t.ratm + t.tau2 * rho * rden);
        const R tb = t.tup * t.cb, tj = t.tup * t.cj;
        const R is_ = tb * sIs, ih = tb * sIh;
        ub[0] = is_ + eta * (ih - is_);   // tau_up (eta I_h + (1 - eta) I_s)
        ub[1] = ih - is_;                  // tau_up (I_h - I_s)
        ub[2] = tj * sMs;
        ub[3] = tj * sSs;
        ub[4] = tj * sMh;
        ub[5] = tj * sSh;
        ub[6] = t.K * t.tau2 * rden * rden;
        ub[7] = ub[6] * t.dl;
        return ls + f * ub[0];
    }
    static constexpr int s1[N] = {0, 1, 2, 2, 4, 4, 6, 7};
    static constexpr int s2[N] = {-1, -1, 3, 3, 5, 5, -1, -1};
    __device__ static void coefficients(const double (&x)[N], double (&c1)[N], double (&c2)[N])
    {
        const LogNormal ls = lognormal(x[2], x[3]);
        const LogNormal lh = lognormal(x[4], x[5]);
        const double f = x[0], eta = x[1];
        const double fs = f * (1.0 - eta), fh = f * eta;
        c1[0] = 1.0; c2[0] = 0.0;
        c1[1] = f; c2[1] = 0.0;
        c1[2] = fs * ls.dmu_dm; c2[2] = fs * ls.dsig_dm;
        c1[3] = fs * ls.dmu_ds; c2[3] = fs * ls.dsig_ds;
        c1[4] = fh * lh.dmu_dm; c2[4] = fh * lh.dsig_dm;
        c1[5] = fh * lh.dmu_ds; c2[5] = fh * lh.dsig_ds;
        c1[6] = 1.0; c2[6] = 0.0;
        c1[7] = 1.0; c2[7] = 0.0;
    }
    // Sec. 2.2 moment matching: E[T] = eta m_h + (1 - eta) m_s,
    // Var[T] = eta s_h^2 + (1 - eta) s_s^2 + eta (1 - eta)(m_h - m_s)^2.
    __device__ static void moments(const double (&x)[N], double& et, double& sd)
    {
        const double eta = x[1], ms = x[2], ss = x[3], mh = x[4], sh = x[5];
        et = eta * mh + (1.0 - eta) * ms;
        const double dm = mh - ms;
        sd = sqrt(eta * sh * sh + (1.0 - eta) * ss * ss + eta * (1.0 - eta) * dm * dm);
    }
};

// ------------------------------------------------------------------------
// The paper's thermal form (Sec. 2.2): two Gaussian components summed over a
// temperature grid of Q uniform nodes T_i = 350 + i (2200 - 350)/(Q - 1) K.
// Node weights of a component: p_i = w_i / sum_j w_j, w_i = exp(-(T_i -
// mu)^2 / (2 sig^2)) (the normalisation truncates to the grid); d_i = T_i -
// mu, m1 = sum p_i d_i, m2 = sum p_i d_i^2.  With B_i = B(lambda, T_i):
//   I = sum p_i B_i,  dI/dmu = S1 / sig^2,  dI/dsig = S2 / sig^3,
//   S1 = sum p_i (d_i - m1) B_i,  S2 = sum p_i (d_i^2 - m2) B_i
// (dp_i/dmu = p_i (d_i - m1)/sig^2, dp_i/dsig = p_i (d_i^2 - m2)/sig^3); the
// centred forms avoid subtracting two large sums in FP32.
// (grid_node<Q>(i), the i-th node temperature, is in ff_internal.hpp)

// Node temperatures and their inverses in constant memory (pairs, so one
// scalar load fetches both); read with a laundered zero offset at the point
// of use so they do not occupy registers across the band loop.
template <typename R, int Q>
struct GridNodes {
    R ti[2 * Q];   // T_0, 1/T_0, T_1, 1/T_1, ...
};
namespace {
template <typename R, int Q>
__constant__ GridNodes<R, Q> c_grid;
}

struct GridComponent {
    double mu1;   // mu + m1: d_i - m1 = T_i - mu1
    double m2;
};

// Normalised node weights (FP64, rounded once to R) and the centring
// constants of one component.
template <typename R, int Q>
__device__ inline GridComponent grid_component(double mu, double sig, R (&p)[Q])
{
    const double inv2s2 = 0.5 / (sig * sig);
    // the largest exponent is at the node nearest mu (clamped to the grid)
    const double h = (2200.0 - 350.0) / (Q - 1);
    double kn = rint((mu - 350.0) / h);
    kn = fmin((double)(Q - 1), fmax(0.0, kn));
    const double dn = 350.0 + h * kn - mu;
    const double emax = -dn * dn * inv2s2;
    // one node at a time (each exponent depends, through an empty asm, on the
    // previous result), the unnormalised weight parked in p
    double W = 0.0, m = mu;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double d = grid_node<Q>(i) - m;
        const double w = exp(-d * d * inv2s2 - emax);
        W += w;
        p[i] = (R)w;
        asm volatile("" : "+v"(m) : "v"(p[i]));
    }
    const double iW = 1.0 / W;
    double m1 = 0.0, m2 = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double pi = (double)p[i] * iW;
        const double d = grid_node<Q>(i) - mu;
        m1 += pi * d;
        m2 += pi * d * d;
        p[i] = (R)pi;
    }
    return GridComponent{mu + m1, m2};
}

// Grid sums of both components at one band: per node one Planck ratio
// q = e/(1 - e) (e = 2^(-a2/T_i), as in thermal_sums) shared by the two
// components, then I, S1, S2 of each: 6 FMA-class + 2 subtractions per
// component per node.
// FP32 with the kGridNodes-node grid: the band's ratios come from the scene
// table (qrow, written at scene creation by the same FP32 operations, so the
// values are the ones computed here otherwise).
template <int Q>
__device__ __forceinline__ void grid_sums(float a2, const float (&ps)[Q], const float (&ph)[Q], float mus, float mus1,
                                          float m2s, float muh, float muh1, float m2h, int o, float (&out)[6],
                                          const float* __restrict__ qrow)
{
    float i0 = 0.f, s1 = 0.f, s2 = 0.f, j0 = 0.f, t1 = 0.f, t2 = 0.f;
    float a = a2;
    const GridNodes<float, Q>& gn = c_grid<float, Q>;
    constexpr bool kTable = Q == kGridNodes;
    float4 q4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const float T = gn.ti[2 * k + o];
        float q;
        if constexpr (kTable) {
            if (k % 4 == 0) q4 = reinterpret_cast<const float4*>(qrow)[k / 4];
            q = k % 4 == 0 ? q4.x : k % 4 == 1 ? q4.y : k % 4 == 2 ? q4.z : q4.w;
        } else {
            (void)qrow;
            const float x = a * gn.ti[2 * k + 1 + o];
            q = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(x) - 1.0f);
        }
        const float ys = ps[k] * q;
        i0 += ys;
        s1 = __builtin_fmaf(ys, T - mus1, s1);
        const float ds = T - mus;
        s2 = __builtin_fmaf(ys, __builtin_fmaf(ds, ds, -m2s), s2);
        const float yh = ph[k] * q;
        j0 += yh;
        t1 = __builtin_fmaf(yh, T - muh1, t1);
        const float dh = T - muh;
        t2 = __builtin_fmaf(yh, __builtin_fmaf(dh, dh, -m2h), t2);
        if ((k + 1) % FF_NODE_GROUP == 0) asm volatile("" : "+v"(a) : "v"(i0), "v"(j0), "v"(s2), "v"(t2));
    }
    out[0] = i0; out[1] = s1; out[2] = s2; out[3] = j0; out[4] = t1; out[5] = t2;
}

template <int Q>
__device__ __forceinline__ void grid_sums(double a2, const double (&ps)[Q], const double (&ph)[Q], double mus,
                                          double mus1, double m2s, double muh, double muh1, double m2h, int o,
                                          double (&out)[6], const double* qrow)
{
    (void)qrow;
    double i0 = 0.0, s1 = 0.0, s2 = 0.0, j0 = 0.0, t1 = 0.0, t2 = 0.0;
    const GridNodes<double, Q>& gn = c_grid<double, Q>;
#pragma unroll 4
    for (int k = 0; k < Q; ++k) {
        const double T = gn.ti[2 * k + o];
        const double e = exp2(-a2 * gn.ti[2 * k + 1 + o]);
        const double q = e / (1.0 - e);
        const double ys = ps[k] * q;
        i0 += ys;
        s1 = fma(ys, T - mus1, s1);
        const double ds = T - mus;
        s2 = fma(ys, fma(ds, ds, -m2s), s2);
        const double yh = ph[k] * q;
        j0 += yh;
        t1 = fma(yh, T - muh1, t1);
        const double dh = T - muh;
        t2 = fma(yh, fma(dh, dh, -m2h), t2);
    }
    out[0] = i0; out[1] = s1; out[2] = s2; out[3] = j0; out[4] = t1; out[5] = t2;
}

template <typename R, int Q>
struct PixelModel<R, FF_MODEL_GAUSS_GRID_2, Q> {
    static constexpr int N = 8;
    static_assert(Q >= 2, "the temperature grid needs two nodes");
    R f, eta, r0, r1;
    R mus, mus1, m2s, muh, muh1, m2h;
    R ps[Q], ph[Q];
    // (node weights are computed by every lane of a group)
    __device__ void setup(const double (&x)[N], int lane = 0, int L = 1)
    {
        (void)lane;
        (void)L;
        f = (R)x[0];
        eta = (R)x[1];
        r0 = (R)x[6];
        r1 = (R)x[7];
        const GridComponent gs = grid_component<R, Q>(x[2], x[3], ps);
        const GridComponent gh = grid_component<R, Q>(x[4], x[5], ph);
        mus = (R)x[2];
        mus1 = (R)gs.mu1;
        m2s = (R)gs.m2;
        muh = (R)x[4];
        muh1 = (R)gh.mu1;
        m2h = (R)gh.m2;
    }
    // qrow: the band's grid Planck ratios in the scene table (FP32)
    __device__ __forceinline__ R band(const BandRow<R>& t, int o, R (&ub)[N], const R* qrow) const
    {
        R g[6];
        grid_sums<Q>(t.a2, ps, ph, mus, mus1, m2s, muh, muh1, m2h, o, g, qrow);
        const R rho = r0 + r1 * t.dl;
        const R rden = fast_rcp<R>((R)1 - t.S * rho);
        const R ls = t.K * (t.ratm + t.tau2 * rho * rden);
        const R tb = t.tup * t.cb;
        const R is_ = tb * g[0], ih = tb * g[3];
        ub[0] = is_ + eta * (ih - is_);   // tau_up (eta I_h + (1 - eta) I_s)
        ub[1] = ih - is_;
        ub[2] = tb * g[1];
        ub[3] = tb * g[2];
        ub[4] = tb * g[4];
        ub[5] = tb * g[5];
        ub[6] = t.K * t.tau2 * rden * rden;
        ub[7] = ub[6] * t.dl;
        return ls + f * ub[0];
    }
    static constexpr int s1[N] = {0, 1, 2, 3, 4, 5, 6, 7};
    static constexpr int s2[N] = {-1, -1, -1, -1, -1, -1, -1, -1};
    __device__ static void coefficients(const double (&x)[N], double (&c1)[N], double (&c2)[N])
    {
        const double f = x[0], eta = x[1], ss = x[3], sh = x[5];
        const double fs = f * (1.0 - eta), fh = f * eta;
        c1[0] = 1.0;
        c1[1] = f;
        c1[2] = fs / (ss * ss);
        c1[3] = fs / (ss * ss * ss);
        c1[4] = fh / (sh * sh);
        c1[5] = fh / (sh * sh * sh);
        c1[6] = 1.0;
        c1[7] = 1.0;
#pragma unroll
        for (int i = 0; i < N; ++i) c2[i] = 0.0;
    }
    // Sec. 2.2 moment matching (as for the lognormal mixture, on the
    // components' nominal means and spreads)
    __device__ static void moments(const double (&x)[N], double& et, double& sd)
    {
        const double eta = x[1], ms = x[2], ss = x[3], mh = x[4], sh = x[5];
        et = eta * mh + (1.0 - eta) * ms;
        const double dm = mh - ms;
        sd = sqrt(eta * sh * sh + (1.0 - eta) * ss * ss + eta * (1.0 - eta) * dm * dm);
    }
};

// The paper's full forward model (Sec. 2.2, library Sec. 2.4): the Gaussian
// mixture on the temperature grid over the endmember surface; state (f, eta,
// mu_s, sig_s, mu_h, sig_h, x_1 .. x_5).
template <typename R, int Q>
struct PixelModel<R, FF_MODEL_FULL, Q> {
    static constexpr int N = 11;
    static constexpr int NE = FF_N_ENDMEMBERS;
    static_assert(Q >= 2, "the temperature grid needs two nodes");
    R f, eta, xs[NE];
    R mus, mus1, m2s, muh, muh1, m2h;
    R ps[Q], ph[Q];
    __device__ void setup(const double (&x)[N], int lane = 0, int L = 1)
    {
        (void)lane;
        (void)L;
        f = (R)x[0];
        eta = (R)x[1];
#pragma unroll
        for (int k = 0; k < NE; ++k) xs[k] = (R)x[6 + k];
        const GridComponent gs = grid_component<R, Q>(x[2], x[3], ps);
        const GridComponent gh = grid_component<R, Q>(x[4], x[5], ph);
        mus = (R)x[2];
        mus1 = (R)gs.mu1;
        m2s = (R)gs.m2;
        muh = (R)x[4];
        muh1 = (R)gh.mu1;
        m2h = (R)gh.m2;
    }
    __device__ __forceinline__ R band(const BandRow<R>& t, const EndmRow<R>& em, int o, R (&ub)[N],
                                      const R* qrow) const
    {
        R g[6];
        grid_sums<Q>(t.a2, ps, ph, mus, mus1, m2s, muh, muh1, m2h, o, g, qrow);
        R rho = xs[0] * em.e[0];
#pragma unroll
        for (int k = 1; k < NE; ++k) rho += xs[k] * em.e[k];
        const R rden = fast_rcp<R>((R)1 - t.S * rho);
        const R ls = t.K * (t.ratm + t.tau2 * rho * rden);
        const R tb = t.tup * t.cb;
        const R is_ = tb * g[0], ih = tb * g[3];
        ub[0] = is_ + eta * (ih - is_);
        ub[1] = ih - is_;
        ub[2] = tb * g[1];
        ub[3] = tb * g[2];
        ub[4] = tb * g[4];
        ub[5] = tb * g[5];
        const R ds = t.K * t.tau2 * rden * rden;
#pragma unroll
        for (int k = 0; k < NE; ++k) ub[6 + k] = ds * em.e[k];
        return ls + f * ub[0];
    }
    static constexpr int s1[N] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10};
    static constexpr int s2[N] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    __device__ static void coefficients(const double (&x)[N], double (&c1)[N], double (&c2)[N])
    {
        const double f = x[0], eta = x[1], ss = x[3], sh = x[5];
        const double fs = f * (1.0 - eta), fh = f * eta;
        c1[0] = 1.0;
        c1[1] = f;
        c1[2] = fs / (ss * ss);
        c1[3] = fs / (ss * ss * ss);
        c1[4] = fh / (sh * sh);
        c1[5] = fh / (sh * sh * sh);
#pragma unroll
        for (int k = 6; k < N; ++k) c1[k] = 1.0;
#pragma unroll
        for (int i = 0; i < N; ++i) c2[i] = 0.0;
    }
    __device__ static void moments(const double (&x)[N], double& et, double& sd)
    {
        const double eta = x[1], ms = x[2], ss = x[3], mh = x[4], sh = x[5];
        et = eta * mh + (1.0 - eta) * ms;
        const double dm = mh - ms;
        sd = sqrt(eta * sh * sh + (1.0 - eta) * ss * ss + eta * (1.0 - eta) * dm * dm);
    }
};

// ---------------------------------------------------------------- host side
// The quadrature rule (computed once per process) and its copy into this
// translation unit's constant memory on each device.  Internal linkage: with
// separate device code objects per translation unit, each unit owns its own
// c_quad instances and must fill them itself.
namespace {

template <typename R, int Q>
const Quad<R, Q>* cached_quad()
{
    static Quad<R, Q> q;
    static bool ok = false;
    static std::once_flag once;
    std::call_once(once, [] {
        if constexpr (sizeof(R) == 4) ok = make_quad_f32(Q, q.w, q.v, q.s);
        else ok = make_quad_f64(Q, q.w, q.v, q.s);
        // the FP32 sums leave out the cold-end nodes: their weights must be
        // below 2^-32 of the largest, in ascending abscissa
        double wmax = 0.0;
        for (int k = 0; k < Q; ++k) wmax = std::max(wmax, (double)q.w[k]);
        for (int k = 0; ok && k < cold_skip_v<R, Q>; ++k)
            ok = (double)q.w[k] <= kColdSkipRatio * wmax && q.s[k] < q.s[k + 1];
    });
    return ok ? &q : nullptr;
}

template <typename R, int Q>
bool ensure_quad(int dev)
{
    static std::mutex mtx;
    static bool done[64] = {};
    if (dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lock(mtx);
    if (!done[dev]) {
        const Quad<R, Q>* host = cached_quad<R, Q>();
        if (!host) return false;
        const void* sym = reinterpret_cast<const void*>(&c_quad<R, Q>);
        if (hipMemcpyToSymbol(sym, host, sizeof(Quad<R, Q>), 0, hipMemcpyHostToDevice) != hipSuccess)
            return false;
        done[dev] = true;
    }
    return true;
}

// The temperature grid of the Gaussian-mixture model in this translation
// unit's constant memory on each device.
template <typename R, int Q>
bool ensure_grid(int dev)
{
    static std::mutex mtx;
    static bool done[64] = {};
    if (dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lock(mtx);
    if (!done[dev]) {
        GridNodes<R, Q> g;
        for (int i = 0; i < Q; ++i) {
            g.ti[2 * i] = (R)grid_node<Q>(i);
            g.ti[2 * i + 1] = (R)(1.0 / grid_node<Q>(i));
        }
        const void* sym = reinterpret_cast<const void*>(&c_grid<R, Q>);
        if (hipMemcpyToSymbol(sym, &g, sizeof(g), 0, hipMemcpyHostToDevice) != hipSuccess) return false;
        done[dev] = true;
    }
    return true;
}

// Constant tables a model's kernels read: the quadrature rule, and for the
// Gaussian-mixture model the temperature grid.
template <typename R, int MODEL, int Q>
bool ensure_tables(int dev)
{
    if (!ensure_quad<R, Q>(dev)) return false;
    if constexpr (grid_thermal_v<MODEL>) return ensure_grid<R, Q>(dev);
    return true;
}

}  // namespace
}  // namespace ff
