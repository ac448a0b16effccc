// Gauss-Hermite rule for the weight e^{-x^2}, computed on the host in long
// double.  Used to integrate the lognormal sub-pixel temperature density of
// the thermal term (eq. thermal) in log T.
//
// Method: the orthonormal Hermite polynomials satisfy
//   p_0 = pi^{-1/4},  p_{j+1}(x) = sqrt(2/(j+1)) x p_j(x) - sqrt(j/(j+1)) p_{j-1}(x),
//   p_q'(x) = sqrt(2 q) p_{q-1}(x).
// The q roots of p_q all lie in (-sqrt(2q+1), sqrt(2q+1)); they are bracketed
// by sign changes of p_q on a fine grid, then refined by Newton steps kept
// inside their bracket.  The weights follow from the Christoffel-Darboux
// identity: w_k = 1 / (q p_{q-1}(x_k)^2).
#include <cmath>
#include <vector>

#include "ff_internal.hpp"

namespace ff {
namespace {

// returns p_q(x), sets *pm1 = p_{q-1}(x)
long double hermite_orthonormal(int q, long double x, long double* pm1)
{
    long double p0 = powl(3.14159265358979323846264338327950288L, -0.25L);
    if (q == 0) { *pm1 = 0.0L; return p0; }
    long double p1 = sqrtl(2.0L) * x * p0;
    for (int j = 1; j < q; ++j) {
        long double p2 = sqrtl(2.0L / (j + 1)) * x * p1 - sqrtl((long double)j / (j + 1)) * p0;
        p0 = p1;
        p1 = p2;
    }
    *pm1 = p0;
    return p1;
}

}  // namespace

bool gauss_hermite(int q, double* xo, double* wo)
{
    if (q < 1 || q > 64) return false;
    const long double lim = sqrtl(2.0L * q + 1.0L) + 0.5L;
    const int ngrid = 400 * q;
    std::vector<long double> roots;
    long double pm1;
    long double xa = -lim, fa = hermite_orthonormal(q, xa, &pm1);
    for (int i = 1; i <= ngrid && (int)roots.size() < q; ++i) {
        long double xb = -lim + 2.0L * lim * i / ngrid;
        long double fb = hermite_orthonormal(q, xb, &pm1);
        if (fb == 0.0L) { roots.push_back(xb); xa = xb; fa = 1.0L; continue; }
        if ((fa < 0) != (fb < 0) && fa != 0.0L) {
            // safeguarded Newton inside [lo, hi]
            long double lo = xa, hi = xb, flo = fa;
            long double x = 0.5L * (lo + hi);
            for (int it = 0; it < 100; ++it) {
                long double d1;
                long double f = hermite_orthonormal(q, x, &d1);
                long double df = sqrtl(2.0L * q) * d1;
                if ((f < 0) == (flo < 0)) { lo = x; flo = f; } else { hi = x; }
                long double xn = x - f / df;
                if (!(xn > lo && xn < hi)) xn = 0.5L * (lo + hi);
                if (fabsl(xn - x) <= 1e-19L * (1.0L + fabsl(x))) { x = xn; break; }
                x = xn;
            }
            roots.push_back(x);
        }
        xa = xb;
        fa = fb;
    }
    if ((int)roots.size() != q) return false;
    for (int k = 0; k < q; ++k) {
        // symmetric rule: average each root with its mirror image
        long double x = 0.5L * (roots[k] - roots[q - 1 - k]);
        long double p;
        hermite_orthonormal(q, x, &p);
        xo[k] = (double)x;
        wo[k] = (double)(1.0L / ((long double)q * p * p));
    }
    return true;
}

template <typename R>
static bool make_quad(int q, R* w, R* v, R* s)
{
    double x[64], wt[64];
    if (!gauss_hermite(q, x, wt)) return false;
    const long double rpi = 1.0L / sqrtl(3.14159265358979323846264338327950288L);
    for (int k = 0; k < q; ++k) {
        long double wh = (long double)wt[k] * rpi;
        long double sk = sqrtl(2.0L) * (long double)x[k];
        w[k] = (R)wh;
        s[k] = (R)sk;
        v[k] = (R)(sk * wh);
    }
    return true;
}

bool make_quad_f32(int q, float* w, float* v, float* s) { return make_quad<float>(q, w, v, s); }
bool make_quad_f64(int q, double* w, double* v, double* s) { return make_quad<double>(q, w, v, s); }

}  // namespace ff
