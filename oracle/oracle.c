/*
 * FP64 CPU oracle for the per-pixel sub-pixel fire-temperature inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product never does.
 * It shares no code, header, table or constant generator with the GPU path.
 *
 * What it computes (cited to Keely et al., "Real-time physics inversion for
 * retrieval of sub-pixel wildfire temperatures from VSWIR imaging
 * spectroscopy"):
 *   - Planck spectral radiance B(lambda, T)                 (Sec. 2.2, eq. thermal)
 *   - forward model L = L_s + L_t                           (Sec. 2.2, eq. fm)
 *       L_s = E cos(sza)/pi [rho_atm + tau_dn tau_up rho / (1 - S rho)]   (eq. solar)
 *       L_t = f tau_up  int p(T) B(lambda, T) dT                            (eq. thermal)
 *     with p(T) a lognormal of mean m and s.d. s (one component) or the
 *     eta-weighted mixture of a smouldering and a flaming lognormal (Sec. 2.2,
 *     two-component mixture), integrated by Gauss-Hermite quadrature in log T,
 *     or the paper's own form: the eta-weighted mixture of two Gaussians
 *     summed over a temperature grid spanning [350, 2200] K (model 3), and a
 *     linear reflectance rho = rho0 + rho1 (lambda - 1440 nm).
 *   - analytic Jacobian of L with respect to the physical state
 *   - the masked least-squares loss (Sec. 2.5, eq. loss) minimised in the
 *     normalised coordinate z of eq. (affine) with z clipped to [-1, 1]
 *     after every update (Sec. 2.5)
 *   - a Levenberg-Marquardt solve (the damped Gauss-Newton scheme follows
 *     Madsen, Nielsen & Tingleff 2004 with Marquardt diagonal scaling,
 *     gain-ratio damping updates and an active set for variables held at a
 *     bound)
 *   - the paper's own solver: staged Adam (Sec. 2.5, eq. adam; Kingma & Ba
 *     2015) on the windowed loss, with a global-norm gradient clip, the
 *     z-clip after every update and per-stage free variables and windows
 *   - the Gauss-Newton state covariance at convergence, and the
 *     moment-matched E[T], sigma[T] of the temperature mixture (Sec. 2.2,
 *     mixture moments).
 * Everything is IEEE double with libm exp/expm1/log1p; no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NMAX 12
#define QMAX 128

/* ---- physical constants: exact SI values ---------------------------------- */
static const double H_PLANCK = 6.62607015e-34;
static const double C_LIGHT = 299792458.0;
static const double K_BOLTZ = 1.380649e-23;
static const double LAMBDA_REF_NM = 1440.0;

/* status bits (mirrors the public status word, defined independently) */
#define ST_GTOL 1u
#define ST_XTOL 2u
#define ST_FTOL 4u
#define ST_MAXITER 8u
#define ST_NONFINITE 16u
#define ST_DAMPING 32u
#define ST_COVSING 64u
#define ST_ATBOUND 128u
#define ST_NODOF 1024u

int orc_version(void) { return 1; }

/* Planck radiance per nm, W m^-2 sr^-1 nm^-1, and its log-temperature
 * derivative T dB/dT.  x = h c / (lambda k T);
 *   B = 2 h c^2 lambda^-5 / (e^x - 1) = 2 h c^2 lambda^-5 e^-x / (1 - e^-x),
 *   T dB/dT = B x e^x / (e^x - 1) = B x / (1 - e^-x). */
double orc_planck(double lam_nm, double T, double* tdbdt)
{
    const double lam = lam_nm * 1e-9;
    const double x = H_PLANCK * C_LIGHT / (lam * K_BOLTZ * T);
    const double one_minus = -expm1(-x);           /* 1 - e^-x, no cancellation */
    const double b = 2.0 * H_PLANCK * C_LIGHT * C_LIGHT / pow(lam, 5.0) * exp(-x) / one_minus * 1e-9;
    if (tdbdt) *tdbdt = b * x / one_minus;
    return b;
}

void orc_planck_many(long n, const double* lam_nm, const double* T, double* out, double* tdbdt)
{
    for (long i = 0; i < n; ++i) out[i] = orc_planck(lam_nm[i], T[i], tdbdt ? &tdbdt[i] : 0);
}

/* Lognormal with mean m and s.d. s: log T ~ N(mu, sig^2) with
 * sig^2 = ln(1 + s^2/m^2), mu = ln m - sig^2/2.  Also the partial
 * derivatives of (mu, sig) with respect to (m, s). */
static void lognormal_params(double m, double s, double* mu, double* sig,
                             double dmu[2], double dsig[2])
{
    const double q = m * m + s * s;
    const double sig2 = log1p(s * s / (m * m));
    *sig = sqrt(sig2);
    *mu = log(m) - 0.5 * sig2;
    const double dsig2_dm = -2.0 * s * s / (m * q);
    const double dsig2_ds = 2.0 * s / q;
    dmu[0] = 1.0 / m - 0.5 * dsig2_dm;
    dmu[1] = -0.5 * dsig2_ds;
    dsig[0] = dsig2_dm / (2.0 * (*sig));
    dsig[1] = dsig2_ds / (2.0 * (*sig));
}

/* Quadrature of the Planck radiance over one lognormal component:
 *   I     = pi^-1/2 sum_k w_k B(lam, T_k),   T_k = exp(mu + sqrt2 sig x_k)
 *   I_mu  = dI/dmu  = pi^-1/2 sum_k w_k T_k dB/dT
 *   I_sig = dI/dsig = pi^-1/2 sum_k w_k sqrt2 x_k T_k dB/dT                */
static void component_integrals(double lam, double mu, double sig, int Q,
                                const double* gx, const double* gw,
                                double* I, double* Imu, double* Isig)
{
    const double inv_sqrt_pi = 1.0 / sqrt(M_PI);
    double si = 0.0, sm = 0.0, ss = 0.0;
    for (int k = 0; k < Q; ++k) {
        const double t = exp(mu + M_SQRT2 * sig * gx[k]);
        double tdb;
        const double b = orc_planck(lam, t, &tdb);
        const double w = gw[k] * inv_sqrt_pi;
        si += w * b;
        sm += w * tdb;
        ss += w * M_SQRT2 * gx[k] * tdb;
    }
    *I = si; *Imu = sm; *Isig = ss;
}

/* Gaussian component on the temperature grid of Sec. 2.2 (the thermal
 * integral is a discrete sum over a grid spanning [350, 2200] K): G uniform
 * nodes T_i = 350 + i (2200 - 350)/(G - 1), weights
 *   p_i = w_i / sum_j w_j,  w_i = exp(-(T_i - mu)^2 / (2 sig^2))
 * (the normalisation truncates the Gaussian to the grid).  Also the
 * weighted moments m1 = sum p_i d_i and m2 = sum p_i d_i^2, d_i = T_i - mu. */
static const double GRID_T_LO = 350.0, GRID_T_HI = 2200.0;

static double grid_node(int G, int i) { return GRID_T_LO + (GRID_T_HI - GRID_T_LO) * i / (G - 1); }

static void grid_weights(int G, double mu, double sig, double* pw, double* m1, double* m2)
{
    double emax = -INFINITY;
    for (int i = 0; i < G; ++i) {
        const double d = grid_node(G, i) - mu;
        pw[i] = -d * d / (2.0 * sig * sig);
        if (pw[i] > emax) emax = pw[i];
    }
    double W = 0.0;
    for (int i = 0; i < G; ++i) { pw[i] = exp(pw[i] - emax); W += pw[i]; }
    *m1 = *m2 = 0.0;
    for (int i = 0; i < G; ++i) {
        pw[i] /= W;
        const double d = grid_node(G, i) - mu;
        *m1 += pw[i] * d;
        *m2 += pw[i] * d * d;
    }
}

/* Grid sums of one component at one band: I = sum p_i B(lam, T_i) and its
 * derivatives from dp_i/dmu = p_i (d_i - m1)/sig^2 and
 * dp_i/dsig = p_i (d_i^2 - m2)/sig^3:
 *   dI/dmu = sum p_i (d_i - m1) B_i / sig^2,  dI/dsig = sum p_i (d_i^2 - m2) B_i / sig^3
 * (summed in this centred form, which keeps full precision when one node
 * carries nearly all the weight). */
static void grid_integrals(double lam, int G, double mu, double sig, double* I, double* Imu, double* Isig)
{
    double pw[QMAX], m1, m2, M0 = 0.0, S1 = 0.0, S2 = 0.0;
    grid_weights(G, mu, sig, pw, &m1, &m2);
    for (int i = 0; i < G; ++i) {
        const double T = grid_node(G, i), d = T - mu;
        const double b = orc_planck(lam, T, 0) * pw[i];
        M0 += b;
        S1 += b * (d - m1);
        S2 += b * (d * d - m2);
    }
    *I = M0;
    *Imu = S1 / (sig * sig);
    *Isig = S2 / (sig * sig * sig);
}

#define N_ENDMEMBERS 5

typedef struct {
    int B;
    const double *lam, *K, *tau2, *tup, *ratm, *S;
    int Q;
    const double *gx, *gw;
    const double* endm;   /* [N_ENDMEMBERS][B] endmember reflectance (model 4) */
} scene_t;

static int n_of_model(int model)
{
    switch (model) {
    case 1: return 5;
    case 2: case 3: case 4: return 8;
    case 5: return 11;
    default: return -1;
    }
}

/* the temperature-grid thermal term (models 3 and 5) needs two nodes */
static int grid_model(int model) { return model == 3 || model == 5; }

/* models 4 and 5 keep their surface fractions (state 3..7, 6..10) on the
 * unit simplex */
static int simplex_first(int model) { return model == 4 ? 3 : (model == 5 ? 6 : -1); }

/* Euclidean projection of v[0..k) onto the unit simplex {x >= 0, sum x = 1}
 * (sort-based, Duchi, Shalev-Shwartz, Singer & Chandra 2008). */
static void project_simplex(int k, double* v)
{
    double u[NMAX];
    for (int i = 0; i < k; ++i) u[i] = v[i];
    for (int i = 1; i < k; ++i) {           /* insertion sort, descending */
        const double t = u[i];
        int j = i - 1;
        while (j >= 0 && u[j] < t) { u[j + 1] = u[j]; --j; }
        u[j + 1] = t;
    }
    double cum = 0.0, theta = 0.0;
    for (int j = 0; j < k; ++j) {
        cum += u[j];
        const double t = (cum - 1.0) / (j + 1);
        if (u[j] - t > 0.0) theta = t;
    }
    for (int i = 0; i < k; ++i) v[i] = v[i] - theta > 0.0 ? v[i] - theta : 0.0;
}

/* The simplex step works in x = (z + 1)/2, so a simplex block needs the
 * box [0, 1] on each of its fractions. */
static int simplex_box_ok(int model, const double* lo, const double* hi)
{
    const int sf = simplex_first(model);
    if (sf < 0) return 1;
    for (int k = sf; k < sf + N_ENDMEMBERS; ++k)
        if (lo[k] != 0.0 || hi[k] != 1.0) return 0;
    return 1;
}

/* exported for the projection's own tests */
void orc_project_simplex(int k, double* v)
{
    if (k >= 1 && k <= NMAX) project_simplex(k, v);
}

/* Forward model at one band for physical state x; fills dL/dx if dl != 0. */
static double model_band(const scene_t* sc, int b, int model, const double* x, double* dl)
{
    const double lam = sc->lam[b];
    const int n = n_of_model(model);
    double rho;
    const int sf = simplex_first(model);
    if (sf >= 0) {
        /* Sec. 2.2: surface reflectance as a mixture of the endmember library */
        rho = 0.0;
        for (int k = 0; k < N_ENDMEMBERS; ++k) rho += x[sf + k] * sc->endm[k * sc->B + b];
    } else {
        rho = x[n - 2] + x[n - 1] * (lam - LAMBDA_REF_NM);
    }
    const double den = 1.0 - sc->S[b] * rho;
    const double ls = sc->K[b] * (sc->ratm[b] + sc->tau2[b] * rho / den);
    const double f = x[0];
    const double tup = sc->tup[b];
    double thermal_I;
    if (model == 1 || model == 4) {
        double mu, sig, dmu[2], dsig[2], I, Imu, Isig;
        lognormal_params(x[1], x[2], &mu, &sig, dmu, dsig);
        component_integrals(lam, mu, sig, sc->Q, sc->gx, sc->gw, &I, &Imu, &Isig);
        thermal_I = I;
        if (dl) {
            dl[0] = tup * I;
            dl[1] = f * tup * (Imu * dmu[0] + Isig * dsig[0]);
            dl[2] = f * tup * (Imu * dmu[1] + Isig * dsig[1]);
        }
    } else if (grid_model(model)) {
        /* the paper's mixture: eta-weighted flaming and smouldering Gaussians
         * on the temperature grid (Q = grid nodes) */
        const double eta = x[1];
        double Is, Ism, Iss, Ih, Ihm, Ihs;
        grid_integrals(lam, sc->Q, x[2], x[3], &Is, &Ism, &Iss);
        grid_integrals(lam, sc->Q, x[4], x[5], &Ih, &Ihm, &Ihs);
        thermal_I = eta * Ih + (1.0 - eta) * Is;
        if (dl) {
            dl[0] = tup * thermal_I;
            dl[1] = f * tup * (Ih - Is);
            dl[2] = f * tup * (1.0 - eta) * Ism;
            dl[3] = f * tup * (1.0 - eta) * Iss;
            dl[4] = f * tup * eta * Ihm;
            dl[5] = f * tup * eta * Ihs;
        }
    } else {
        const double eta = x[1];
        double mus, sigs, dmus[2], dsigs[2], Is, Imus, Isigs;
        double muh, sigh, dmuh[2], dsigh[2], Ih, Imuh, Isigh;
        lognormal_params(x[2], x[3], &mus, &sigs, dmus, dsigs);
        lognormal_params(x[4], x[5], &muh, &sigh, dmuh, dsigh);
        component_integrals(lam, mus, sigs, sc->Q, sc->gx, sc->gw, &Is, &Imus, &Isigs);
        component_integrals(lam, muh, sigh, sc->Q, sc->gx, sc->gw, &Ih, &Imuh, &Isigh);
        thermal_I = eta * Ih + (1.0 - eta) * Is;
        if (dl) {
            dl[0] = tup * thermal_I;
            dl[1] = f * tup * (Ih - Is);
            dl[2] = f * tup * (1.0 - eta) * (Imus * dmus[0] + Isigs * dsigs[0]);
            dl[3] = f * tup * (1.0 - eta) * (Imus * dmus[1] + Isigs * dsigs[1]);
            dl[4] = f * tup * eta * (Imuh * dmuh[0] + Isigh * dsigh[0]);
            dl[5] = f * tup * eta * (Imuh * dmuh[1] + Isigh * dsigh[1]);
        }
    }
    if (dl) {
        const double drho = sc->K[b] * sc->tau2[b] / (den * den);
        if (sf >= 0) {
            for (int k = 0; k < N_ENDMEMBERS; ++k) dl[sf + k] = drho * sc->endm[k * sc->B + b];
        } else {
            dl[n - 2] = drho;
            dl[n - 1] = drho * (lam - LAMBDA_REF_NM);
        }
    }
    return ls + f * tup * thermal_I;
}

/* Forward model (and optionally dL/dx, layout [P][B][n]) for P states. */
int orc_forward(int B, const double* lam, const double* K, const double* tau2,
                const double* tup, const double* ratm, const double* S, const double* endm,
                int Q, const double* gx, const double* gw,
                int model, long P, const double* state, double* L, double* dLdx,
                int nthreads)
{
    const int n = n_of_model(model);
    if (n < 0 || Q <= 0 || Q > QMAX || (grid_model(model) && Q < 2) || (simplex_first(model) >= 0 && !endm) || B <= 0) return -1;
    scene_t sc = {B, lam, K, tau2, tup, ratm, S, Q, gx, gw, endm};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (long p = 0; p < P; ++p) {
        for (int b = 0; b < B; ++b) {
            double dl[NMAX];
            L[p * B + b] = model_band(&sc, b, model, state + p * n, dLdx ? dl : 0);
            if (dLdx) for (int j = 0; j < n; ++j) dLdx[(p * B + b) * n + j] = dl[j];
        }
    }
    return 0;
}

/* ---- small dense linear algebra -------------------------------------------- */
/* Cholesky M = C C^T of an n x n symmetric matrix (row-major, lower C).
 * Returns 0 if a pivot is not strictly positive. */
static int cholesky(int n, const double* M, double* C)
{
    memset(C, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double d = M[j * n + j];
        for (int k = 0; k < j; ++k) d -= C[j * n + k] * C[j * n + k];
        if (!(d > 0.0)) return 0;
        const double cjj = sqrt(d);
        C[j * n + j] = cjj;
        for (int i = j + 1; i < n; ++i) {
            double v = M[i * n + j];
            for (int k = 0; k < j; ++k) v -= C[i * n + k] * C[j * n + k];
            C[i * n + j] = v / cjj;
        }
    }
    return 1;
}

/* Solve C C^T x = rhs. */
static void chol_solve(int n, const double* C, const double* rhs, double* x)
{
    double y[NMAX];
    for (int i = 0; i < n; ++i) {
        double v = rhs[i];
        for (int k = 0; k < i; ++k) v -= C[i * n + k] * y[k];
        y[i] = v / C[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= C[k * n + i] * x[k];
        x[i] = v / C[i * n + i];
    }
}

/* ---- one pixel's least-squares problem in z ------------------------------- */
typedef struct {
    const scene_t* sc;
    int model, n;
    const double *lo, *hi;
    const float* lobs;      /* [B] */
    const unsigned char* mask;  /* [B] 1 = band used */
} problem_t;

static void z_to_x(const problem_t* pb, const double* z, double* x)
{
    for (int j = 0; j < pb->n; ++j)
        x[j] = pb->lo[j] + 0.5 * (pb->hi[j] - pb->lo[j]) * (z[j] + 1.0);
}

/* r = m (L_obs - L(x(z))), J = dr/dz; returns F = r.r and fills A = J^T J,
 * g = J^T r (A row-major n x n). */
static double evaluate(const problem_t* pb, const double* z, double* A, double* g)
{
    const int n = pb->n;
    double x[NMAX], dx[NMAX];
    z_to_x(pb, z, x);
    for (int j = 0; j < n; ++j) dx[j] = 0.5 * (pb->hi[j] - pb->lo[j]);
    memset(A, 0, sizeof(double) * n * n);
    memset(g, 0, sizeof(double) * n);
    double F = 0.0;
    for (int b = 0; b < pb->sc->B; ++b) {
        if (!pb->mask[b]) continue;
        double dl[NMAX], jrow[NMAX];
        const double L = model_band(pb->sc, b, pb->model, x, dl);
        const double r = (double)pb->lobs[b] - L;
        for (int j = 0; j < n; ++j) jrow[j] = -dl[j] * dx[j];
        F += r * r;
        for (int i = 0; i < n; ++i) {
            g[i] += jrow[i] * r;
            for (int j = 0; j < n; ++j) A[i * n + j] += jrow[i] * jrow[j];
        }
    }
    return F;
}

/* Variables held at a bound by a gradient pointing out of the box.  For a
 * simplex block (fractions sf .. sf+4 of model 4, x = (z + 1)/2 summing to
 * one) a fraction at zero is held when its gradient exceeds the mean
 * gradient of the fractions above zero (moving weight onto it would raise
 * the loss). */
static void active_set(int n, int sf, const double* z, const double* g, int* act)
{
    for (int j = 0; j < n; ++j)
        act[j] = (z[j] <= -1.0 && g[j] > 0.0) || (z[j] >= 1.0 && g[j] < 0.0);
    if (sf < 0) return;
    double gs = 0.0;
    int m = 0;
    for (int k = sf; k < sf + N_ENDMEMBERS; ++k)
        if (z[k] > -1.0) { gs += g[k]; ++m; }
    const double gbar = m > 0 ? gs / m : 0.0;
    for (int k = sf; k < sf + N_ENDMEMBERS; ++k) act[k] = z[k] <= -1.0 && g[k] - gbar > 0.0;
}

/* projected-gradient test: max_j |g_j| / sqrt(A_jj F) over free j; in a
 * simplex block the gradient less its mean over the free fractions */
static int gradient_small(int n, int sf, const double* z, const double* A, const double* g,
                          double F, double gtol)
{
    if (!(F > 0.0)) return 1;
    int act[NMAX];
    active_set(n, sf, z, g, act);
    double gr[NMAX];
    for (int j = 0; j < n; ++j) gr[j] = g[j];
    if (sf >= 0) {
        double gs = 0.0;
        int m = 0;
        for (int k = sf; k < sf + N_ENDMEMBERS; ++k)
            if (!act[k]) { gs += g[k]; ++m; }
        for (int k = sf; k < sf + N_ENDMEMBERS; ++k) gr[k] = g[k] - (m > 0 ? gs / m : 0.0);
    }
    for (int j = 0; j < n; ++j) {
        if (act[j] || !(A[j * n + j] > 0.0)) continue;
        if (fabs(gr[j]) > gtol * sqrt(A[j * n + j] * F)) return 0;
    }
    return 1;
}

/* The simplex block of z (fractions x = (z + 1)/2) projected onto the unit
 * simplex: the step the paper applies to the surface mixture after each
 * optimiser update (Sec. 2.5). */
static void project_block(int sf, double* z)
{
    if (sf < 0) return;
    double x[NMAX];
    for (int k = 0; k < N_ENDMEMBERS; ++k) x[k] = 0.5 * (z[sf + k] + 1.0);
    project_simplex(N_ENDMEMBERS, x);
    for (int k = 0; k < N_ENDMEMBERS; ++k) z[sf + k] = 2.0 * x[k] - 1.0;
}

/* Levenberg-Marquardt trial point z + a delta: the box variables clipped to
 * [-1, 1]; with a simplex block the step is first shortened (a <= 1, the
 * ratio test of active-set methods) so that no fraction goes below zero,
 * and the fraction that stops it is set to exactly zero, where the next
 * step can hold it.  The step keeps its direction, so a descent step of the
 * damped model stays one, and keeps the fractions' sum up to rounding (no
 * projection here: shifting every fraction by the rounding of the sum would
 * lift the zeros off zero).  Returns 1 when the step was shortened. */
static int trial_point(int n, int sf, const double* z, const double* delta, double* zt)
{
    double a = 1.0;
    int stop = -1;
    if (sf >= 0)
        for (int k = sf; k < sf + N_ENDMEMBERS; ++k) {
            const double x = 0.5 * (z[k] + 1.0), dx = 0.5 * delta[k];
            if (dx < 0.0 && x + dx < 0.0 && x / -dx < a) { a = x / -dx; stop = k; }
        }
    for (int j = 0; j < n; ++j) {
        const double zz = z[j] + a * delta[j];
        zt[j] = zz < -1.0 ? -1.0 : (zz > 1.0 ? 1.0 : zz);
    }
    if (stop >= 0) zt[stop] = -1.0;
    return stop >= 0;
}

typedef struct {
    int max_iter;
    double xtol, ftol, gtol, kappa, tau;
    double ftol_undetected, f_detect;   /* FTOL while the fire fraction x_0 < f_detect */
} lmopt_t;

/* Levenberg-Marquardt from z (in/out).  Returns status bits; *iters counts
 * model evaluations after the initial one. */
static unsigned lm_solve(const problem_t* pb, const lmopt_t* o, double* z,
                         double* A, double* g, double* Fout, int* iters)
{
    const int n = pb->n;
    const int sf = simplex_first(pb->model);
    double At[NMAX * NMAX], gt[NMAX], M[NMAX * NMAX], C[NMAX * NMAX];
    double d[NMAX], zt[NMAX], h[NMAX], delta[NMAX], rhs[NMAX];
    int act[NMAX];
    unsigned st = 0;
    *iters = 0;
    double F = evaluate(pb, z, A, g);
    if (!isfinite(F)) { *Fout = F; return ST_NONFINITE; }
    if (gradient_small(n, sf, z, A, g, F, o->gtol)) { *Fout = F; return ST_GTOL; }
    double amax = 0.0;
    for (int j = 0; j < n; ++j) amax = fmax(amax, A[j * n + j]);
    if (!(amax > 0.0)) amax = 1.0;
    for (int j = 0; j < n; ++j) d[j] = fmax(A[j * n + j], 1e-12 * amax);
    double mu = o->tau * amax, nu = 2.0;

    for (;;) {
        if (*iters >= o->max_iter) { st = ST_MAXITER; break; }
        /* damped step on the free variables, retried with more damping
         * until it is a descent step of the quadratic model */
        double pred = 0.0;
        int have_step = 0, tries = 0, cut = 0;
        while (!have_step) {
            if (++tries > 64 || mu > 1e30 * amax) { st = ST_DAMPING; break; }
            active_set(n, sf, z, g, act);
            int factored = 1;
            for (;;) {
                for (int i = 0; i < n; ++i) {
                    for (int j = 0; j < n; ++j)
                        M[i * n + j] = (act[i] || act[j]) ? 0.0 : A[i * n + j];
                    M[i * n + i] = act[i] ? 1.0 : A[i * n + i] + mu * d[i];
                    rhs[i] = act[i] ? 0.0 : -g[i];
                }
                if (!cholesky(n, M, C)) { factored = 0; break; }
                chol_solve(n, C, rhs, delta);
                if (sf < 0) break;
                /* keep the free fractions' sum: delta -= nu' M^-1 c with c the
                 * indicator of the free fractions and nu' = c.delta / c.M^-1 c
                 * (the equality-constrained minimiser of the damped model) */
                double c[NMAX], y[NMAX], cd = 0.0, cy = 0.0;
                for (int j = 0; j < n; ++j) c[j] = (j >= sf && j < sf + N_ENDMEMBERS && !act[j]) ? 1.0 : 0.0;
                chol_solve(n, C, c, y);
                for (int j = 0; j < n; ++j) { cd += c[j] * delta[j]; cy += c[j] * y[j]; }
                if (cy > 0.0)
                    for (int j = 0; j < n; ++j) delta[j] -= cd / cy * y[j];
                /* a fraction at zero that the step would push below zero is
                 * held too, and the step is solved again (at most once per
                 * fraction), so the projection only ever stops fractions that
                 * start above zero */
                int more = 0;
                for (int k = sf; k < sf + N_ENDMEMBERS; ++k)
                    if (!act[k] && z[k] <= -1.0 && delta[k] < 0.0) { act[k] = 1; more = 1; }
                if (!more) break;
            }
            if (!factored) { mu *= nu; nu *= 2.0; continue; }
            /* a step cut short by the simplex is no sign of convergence: the
             * fraction it stops at zero is held from the next step on, so
             * neither the step-size nor the decrease test is taken on it */
            cut = trial_point(n, sf, z, delta, zt);
            double hmax = 0.0;
            for (int j = 0; j < n; ++j) {
                h[j] = zt[j] - z[j];
                hmax = fmax(hmax, fabs(h[j]));
            }
            if (hmax <= o->xtol && !cut) { st = ST_XTOL; break; }
            double hg = 0.0, hah = 0.0;
            for (int i = 0; i < n; ++i) {
                hg += h[i] * g[i];
                for (int j = 0; j < n; ++j) hah += h[i] * A[i * n + j] * h[j];
            }
            pred = -(2.0 * hg + hah);
            if (pred > 0.0) have_step = 1;
            else { mu *= nu; nu *= 2.0; }
        }
        if (st) break;

        const double Ft = evaluate(pb, zt, At, gt);
        ++*iters;
        const double rho = (F - Ft) / pred;
        if (isfinite(Ft) && (rho > 0.0 || pred <= o->kappa * F)) {
            const double Fold = F;
            memcpy(z, zt, sizeof(double) * n);
            memcpy(A, At, sizeof(double) * n * n);
            memcpy(g, gt, sizeof(double) * n);
            F = Ft;
            const double rc = rho < 0.0 ? 0.0 : (rho > 1.0 ? 1.0 : rho);
            const double t = 2.0 * rc - 1.0;
            mu *= fmax(1.0 / 3.0, 1.0 - t * t * t);
            nu = 2.0;
            for (int j = 0; j < n; ++j) d[j] = fmax(d[j], A[j * n + j]);
            /* the decrease test: ftol, or ftol_undetected while the fire
             * fraction is below the detection level (no identified thermal
             * variables: the loss there is the noise valley of the
             * area-temperature degeneracy) */
            const double xf = pb->lo[0] + 0.5 * (pb->hi[0] - pb->lo[0]) * (z[0] + 1.0);
            const double ft = xf < o->f_detect ? o->ftol_undetected : o->ftol;
            if (pred <= ft * Fold && !cut) { st = ST_FTOL; break; }
            if (gradient_small(n, sf, z, A, g, F, o->gtol)) { st = ST_GTOL; break; }
        } else {
            mu *= nu;
            nu *= 2.0;
        }
    }
    *Fout = F;
    return st;
}

/* Gauss-Newton covariance sigma^2 A^-1 in z (sigma^2 = F / (N - n)), mapped
 * to x; state variables whose Jacobian column is identically zero are
 * unidentified: their rows/columns are NaN and COV_SINGULAR is set.  Output
 * is the packed upper triangle, row-major. */
static unsigned covariance(int n, const double* A, double F, int nvalid,
                           const double* lo, const double* hi, double* cov)
{
    int keep[NMAX], nk = 0, idx[NMAX];
    unsigned st = 0;
    for (int j = 0; j < n; ++j) {
        keep[j] = A[j * n + j] > 0.0;
        if (keep[j]) idx[nk++] = j;
    }
    if (nk < n) st |= ST_COVSING;
    double Ak[NMAX * NMAX], C[NMAX * NMAX], inv[NMAX * NMAX];
    for (int a = 0; a < nk; ++a)
        for (int b = 0; b < nk; ++b) Ak[a * nk + b] = A[idx[a] * n + idx[b]];
    int ok = nk > 0 && cholesky(nk, Ak, C);
    if (ok) {
        for (int c = 0; c < nk; ++c) {
            double e[NMAX] = {0}, col[NMAX];
            e[c] = 1.0;
            chol_solve(nk, C, e, col);
            for (int r = 0; r < nk; ++r) inv[r * nk + c] = col[r];
        }
    } else {
        st |= ST_COVSING;
    }
    const double s2 = F / (double)(nvalid - n);
    int pos = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = i; j < n; ++j, ++pos) {
            double v = NAN;
            if (ok && keep[i] && keep[j]) {
                int a = 0, b = 0;
                while (idx[a] != i) ++a;
                while (idx[b] != j) ++b;
                v = s2 * inv[a * nk + b] * 0.25 * (hi[i] - lo[i]) * (hi[j] - lo[j]);
            }
            cov[pos] = v;
        }
    }
    return st;
}

/* moment-matched mean and s.d. of the temperature distribution */
static void moments_of(int model, const double* x, double* et, double* sdt)
{
    if (model == 1 || model == 4) { *et = x[1]; *sdt = x[2]; return; }
    const double eta = x[1], ms = x[2], ss = x[3], mh = x[4], sh = x[5];
    *et = eta * mh + (1.0 - eta) * ms;
    const double dm = mh - ms;
    const double var = eta * sh * sh + (1.0 - eta) * ss * ss + eta * (1.0 - eta) * dm * dm;
    *sdt = sqrt(var);
}

/* Saturation mask of one pixel (a band is used iff L_obs < L_sat), the
 * number of used bands and the squared norm of their radiance.  Returns 0 if
 * some radiance is not finite. */
static int pixel_bands(int B, const float* lp, const float* lsat, unsigned char* mask,
                       int* nvalid, double* lnorm2)
{
    int fin = 1;
    *nvalid = 0;
    *lnorm2 = 0.0;
    for (int b = 0; b < B; ++b) {
        if (!isfinite(lp[b])) fin = 0;
        mask[b] = lsat ? (lp[b] < lsat[b]) : 1;
        if (mask[b]) { ++*nvalid; *lnorm2 += (double)lp[b] * (double)lp[b]; }
    }
    return fin;
}

/* Starting z of one pixel: z0 if given, else x0 mapped by eq. (affine);
 * clipped to [-1, 1]. */
static void start_z(int n, int sf, const double* lo, const double* hi, const double* x0,
                    const double* z0p, double* z)
{
    for (int j = 0; j < n; ++j) {
        const double zz = z0p ? z0p[j] : 2.0 * (x0[j] - lo[j]) / (hi[j] - lo[j]) - 1.0;
        z[j] = zz < -1.0 ? -1.0 : (zz > 1.0 ? 1.0 : zz);
    }
    project_block(sf, z);
}

/* Outputs of pixel p from its final z, J^T J (A) and loss F over all used
 * bands; st carries the status bits so far. */
static void write_pixel(int model, int n, long p, unsigned st, const double* z, const double* A,
                        double F, int nvalid, double lnorm2, const double* lo, const double* hi,
                        double* state, double* cov, double* moments, double* rrr,
                        unsigned* status)
{
    const int ncov = n * (n + 1) / 2;
    double* cv = cov + p * ncov;
    if (st & (ST_NONFINITE | ST_NODOF)) {
        for (int j = 0; j < n; ++j) state[p * n + j] = NAN;
        for (int j = 0; j < ncov; ++j) cv[j] = NAN;
        moments[2 * p] = moments[2 * p + 1] = NAN;
        rrr[p] = NAN;
    } else {
        double x[NMAX];
        for (int j = 0; j < n; ++j) {
            x[j] = lo[j] + 0.5 * (hi[j] - lo[j]) * (z[j] + 1.0);
            state[p * n + j] = x[j];
            if (z[j] <= -1.0 || z[j] >= 1.0) st |= ST_ATBOUND;
        }
        st |= covariance(n, A, F, nvalid, lo, hi, cv);
        moments_of(model, x, &moments[2 * p], &moments[2 * p + 1]);
        rrr[p] = lnorm2 > 0.0 ? sqrt(F / lnorm2) : NAN;
    }
    status[p] = st;
}

/* Retrieve P pixels.  lobs is [P][B] float32 (widened to double).
 * lsat: [B] saturation levels or NULL.  z0: [P][n] starting z or NULL
 * (then x0 is mapped to z for every pixel).  Outputs are double:
 * state [P][n] physical, cov [P][n(n+1)/2], moments [P][2], rrr [P],
 * iters [P], status [P]. */
int orc_retrieve(int B, const double* lam, const double* K, const double* tau2,
                 const double* tup, const double* ratm, const double* S, const double* endm,
                 const float* lsat, int Q, const double* gx, const double* gw,
                 int model, const double* lo, const double* hi, const double* x0,
                 const double* z0, long P, const float* lobs,
                 int max_iter, double xtol, double ftol, double gtol, double kappa,
                 double tau, double ftol_undetected, double f_detect, int nthreads,
                 double* state, double* cov, double* moments, double* rrr,
                 int* iters, unsigned* status)
{
    const int n = n_of_model(model);
    if (n < 0 || Q <= 0 || Q > QMAX || (grid_model(model) && Q < 2) || (simplex_first(model) >= 0 && !endm) || B <= 0 || P < 0) return -1;
    for (int j = 0; j < n; ++j) if (!(hi[j] > lo[j])) return -1;
    if (!simplex_box_ok(model, lo, hi)) return -1;
    scene_t sc = {B, lam, K, tau2, tup, ratm, S, Q, gx, gw, endm};
    lmopt_t o = {max_iter, xtol, ftol, gtol, kappa, tau, ftol_undetected, f_detect};
    if (!(tau > 0.0)) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long p = 0; p < P; ++p) {
        const float* lp = lobs + p * B;
        unsigned char* mask = (unsigned char*)malloc(B);
        unsigned st = 0;
        int nvalid;
        double lnorm2;
        const int finite_in = pixel_bands(B, lp, lsat, mask, &nvalid, &lnorm2);
        double z[NMAX], A[NMAX * NMAX], g[NMAX], F = NAN;
        int it = 0;
        if (!finite_in) st = ST_NONFINITE;
        else if (nvalid <= n) st = ST_NODOF;
        if (!st) {
            start_z(n, simplex_first(model), lo, hi, x0, z0 ? z0 + p * n : 0, z);
            problem_t pb = {&sc, model, n, lo, hi, lp, mask};
            st = lm_solve(&pb, &o, z, A, g, &F, &it);
        }
        write_pixel(model, n, p, st, z, A, F, nvalid, lnorm2, lo, hi, state, cov, moments, rrr,
                    status);
        iters[p] = it;
        free(mask);
    }
    return 0;
}

/* ---- the paper's solver: staged Adam (Sec. 2.5) ---------------------------- */
typedef struct {
    int steps;
    unsigned free_mask;        /* bit j set: z_j is a variable of this stage */
    double lr;                 /* learning rate in z */
    double clip;               /* maximum global norm of the gradient (<= 0: none) */
    const double *wlo, *whi;   /* [n] band window (nm, inclusive) of each variable's loss */
    const double* zset;        /* [n] NaN: z_j carried over; else z_j at the stage start */
} adam_stage_t;

static double clamp1(double v) { return v < -1.0 ? -1.0 : (v > 1.0 ? 1.0 : v); }

/* Gradient of the windowed loss (eq. loss) with respect to each free z_j,
 * taken over the used bands inside variable j's window:
 *   G_j = d/dz_j sum_b (L_obs,b - L_b(x(z)))^2
 *       = -2 sum_b (L_obs,b - L_b) dL_b/dx_j (hi_j - lo_j)/2.
 * Held variables get G_j = 0.  Returns 0 if some G_j is not finite. */
static int windowed_gradient(const problem_t* pb, const adam_stage_t* s, const double* z,
                             double* G)
{
    const int n = pb->n;
    double x[NMAX];
    z_to_x(pb, z, x);
    for (int j = 0; j < n; ++j) G[j] = 0.0;
    for (int b = 0; b < pb->sc->B; ++b) {
        if (!pb->mask[b]) continue;
        const double lam = pb->sc->lam[b];
        int in[NMAX], any = 0;
        for (int j = 0; j < n; ++j) {
            in[j] = ((s->free_mask >> j) & 1u) && lam >= s->wlo[j] && lam <= s->whi[j];
            any |= in[j];
        }
        if (!any) continue;
        double dl[NMAX];
        const double r = (double)pb->lobs[b] - model_band(pb->sc, b, pb->model, x, dl);
        for (int j = 0; j < n; ++j)
            if (in[j]) G[j] += -2.0 * r * dl[j] * 0.5 * (pb->hi[j] - pb->lo[j]);
    }
    for (int j = 0; j < n; ++j)
        if (!isfinite(G[j])) return 0;
    return 1;
}

/* Adam (eq. adam) through the stages in order, from z (in/out).  Each stage
 * starts a fresh optimiser (t = 1, m = v = 0) on its free variables; the
 * gradient is scaled down to the stage's maximum global norm when it is
 * longer, and z is clipped to [-1, 1] after every update.  Returns the number
 * of steps taken, or -1 when a gradient is not finite. */
static int adam_solve(const problem_t* pb, int nst, const adam_stage_t* stages, double beta1,
                      double beta2, double eps, double* z)
{
    const int n = pb->n;
    int steps = 0;
    for (int k = 0; k < nst; ++k) {
        const adam_stage_t* s = &stages[k];
        double m[NMAX], v[NMAX], G[NMAX];
        for (int j = 0; j < n; ++j) {
            m[j] = v[j] = 0.0;
            if (!isnan(s->zset[j])) z[j] = clamp1(s->zset[j]);
        }
        project_block(simplex_first(pb->model), z);
        for (int t = 1; t <= s->steps; ++t) {
            if (!windowed_gradient(pb, s, z, G)) return -1;
            double norm2 = 0.0;
            for (int j = 0; j < n; ++j) norm2 += G[j] * G[j];
            const double norm = sqrt(norm2);
            if (s->clip > 0.0 && norm > s->clip)
                for (int j = 0; j < n; ++j) G[j] *= s->clip / norm;
            const double bc1 = 1.0 - pow(beta1, t), bc2 = 1.0 - pow(beta2, t);
            for (int j = 0; j < n; ++j) {
                if (!((s->free_mask >> j) & 1u)) continue;
                m[j] = beta1 * m[j] + (1.0 - beta1) * G[j];
                v[j] = beta2 * v[j] + (1.0 - beta2) * G[j] * G[j];
                const double mhat = m[j] / bc1, vhat = v[j] / bc2;
                z[j] = clamp1(z[j] - s->lr * mhat / (sqrt(vhat) + eps));
            }
            /* the surface mixture back onto the unit simplex (Sec. 2.5) */
            project_block(simplex_first(pb->model), z);
            ++steps;
        }
    }
    return steps;
}

/* Staged-Adam retrieval of P pixels; inputs and outputs as orc_retrieve.
 * Stage k: steps[k], free[k] (bit mask), lr[k], clip[k], and [n_stages][n]
 * arrays wlo, whi (window of each variable's loss, nm) and zset (NaN: carry
 * over).  iters = Adam steps taken.  The covariance, moments and relative
 * residual are those of the final z over all used bands. */
int orc_adam_retrieve(int B, const double* lam, const double* K, const double* tau2,
                      const double* tup, const double* ratm, const double* S, const double* endm,
                      const float* lsat, int Q, const double* gx, const double* gw,
                      int model, const double* lo, const double* hi, const double* x0,
                      const double* z0, long P, const float* lobs,
                      int n_stages, const int* steps, const unsigned* free_mask,
                      const double* lr, const double* clip, const double* wlo,
                      const double* whi, const double* zset,
                      double beta1, double beta2, double eps, int nthreads,
                      double* state, double* cov, double* moments, double* rrr,
                      int* iters, unsigned* status)
{
    const int n = n_of_model(model);
    if (n < 0 || Q <= 0 || Q > QMAX || (grid_model(model) && Q < 2) || (simplex_first(model) >= 0 && !endm) || B <= 0 || P < 0 || n_stages < 0 || n_stages > 16) return -1;
    for (int j = 0; j < n; ++j) if (!(hi[j] > lo[j])) return -1;
    if (!simplex_box_ok(model, lo, hi)) return -1;
    adam_stage_t st[16];
    for (int k = 0; k < n_stages; ++k) {
        if (steps[k] < 0 || !(lr[k] > 0.0)) return -1;
        st[k].steps = steps[k];
        st[k].free_mask = free_mask[k];
        st[k].lr = lr[k];
        st[k].clip = clip[k];
        st[k].wlo = wlo + k * n;
        st[k].whi = whi + k * n;
        st[k].zset = zset + k * n;
    }
    scene_t sc = {B, lam, K, tau2, tup, ratm, S, Q, gx, gw, endm};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long p = 0; p < P; ++p) {
        const float* lp = lobs + p * B;
        unsigned char* mask = (unsigned char*)malloc(B);
        unsigned s = 0;
        int nvalid;
        double lnorm2;
        const int finite_in = pixel_bands(B, lp, lsat, mask, &nvalid, &lnorm2);
        double z[NMAX], A[NMAX * NMAX], g[NMAX], F = NAN;
        int it = 0;
        if (!finite_in) s = ST_NONFINITE;
        else if (nvalid <= n) s = ST_NODOF;
        if (!s) {
            start_z(n, simplex_first(model), lo, hi, x0, z0 ? z0 + p * n : 0, z);
            problem_t pb = {&sc, model, n, lo, hi, lp, mask};
            it = adam_solve(&pb, n_stages, st, beta1, beta2, eps, z);
            if (it < 0) {
                s = ST_NONFINITE;
                it = 0;
            } else {
                F = evaluate(&pb, z, A, g);
                if (!isfinite(F)) s = ST_NONFINITE;
            }
        }
        write_pixel(model, n, p, s, z, A, F, nvalid, lnorm2, lo, hi, state, cov, moments, rrr,
                    status);
        iters[p] = it;
        free(mask);
    }
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
