/*
 * hs_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain, slow, obviously-correct FP64 CPU definition of what the Heston
 * Longstaff-Schwartz Greek engine computes.  Only tests/, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library; the product
 * (the HIP library behind include/hs_api.h) never links, calls or includes it,
 * and this file includes nothing from the product.
 *
 * Source of the method (arXiv 2206.03719, "Low-power option Greeks"):
 *   - Sec. 2.2 (STAC-A2): Greeks are sensitivities of option values to market
 *     moves; paths come from a Monte Carlo simulation of the Heston
 *     stochastic-volatility model, and Longstaff-Schwartz regression decides
 *     early exercise.
 *   - Sec. 2.2.1 (general code structure): each asset carries its own Heston
 *     configuration; the work spans paths x assets x timesteps; the model is
 *     advanced in log price and then exponentiated; the LS stage is a
 *     reduction followed by a quadratic curve fit.
 *   - Sec. 4.1 (algorithmic optimisations): the LS path reduction takes, for
 *     each path and timestep, the maximum value over assets.
 * The paper prints no equations.  Every convention below (discretisation,
 * random-number layout, basis, bump sizes) is the reading recorded in the
 * design notes; each function states the one it implements.
 *
 * Precision: FP64 everywhere, built with -ffp-contract=off, libm
 * exp/log/sin/cos/sqrt.  Parallelism only over fixed 4096-path chunks, and
 * every sum over paths is formed per chunk in path order and then over chunks
 * in chunk order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CHUNK 4096

/* status codes (documented integers of the public interface) */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTSPD (-2)
#define ORC_ENOMEM (-3)

/* option codes */
#define ORC_PUT 0
#define ORC_CALL 1
#define ORC_EUROPEAN 0
#define ORC_AMERICAN 1

/* bump mask bits */
#define ORC_DELTA_GAMMA 1u
#define ORC_VEGA 2u
#define ORC_THETA 4u
#define ORC_RHO 8u
#define ORC_CORR 16u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  A round multiplies
 * counter words 0 and 2 by two fixed odd constants, keeps the 64-bit
 * products' high and low halves, and recombines them with the other two
 * counter words and the key; the key is advanced by two Weyl constants
 * between rounds.  Ten rounds. */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform map: the top 23 bits of a word select one of the 2^23 odd
 * multiples of 2^-24 in (0,1); each is exact in both FP32 and FP64. */
double orc_uniform(uint32_t w)
{
    uint32_t odd = 2u * (w >> 9) + 1u;
    return (double)odd * 0x1p-24;
}

/* Box-Muller on one pair of words: R = sqrt(-2 ln u1), eps = R cos(2 pi u2),
 * eta = R sin(2 pi u2). */
void orc_normal_pair(uint32_t w1, uint32_t w2, double out[2])
{
    double u1 = orc_uniform(w1);
    double u2 = orc_uniform(w2);
    double R = sqrt(-2.0 * log(u1));
    double a = 2.0 * M_PI * u2;
    out[0] = R * cos(a);
    out[1] = R * sin(a);
}

/* The normals of one path and one step (the step from date k to k+1).
 * Counter (p mod 2^32, k, j, p >> 32) for Philox block j; key = (seed mod
 * 2^32, seed >> 32).  Words (w0,w1) drive asset 2j and (w2,w3) asset 2j+1;
 * an odd asset count discards the last pair.  The counter does not involve
 * the scenario: every bumped scenario sees the same numbers. */
void orc_normals(int32_t N, uint64_t seed, int64_t p, int32_t k, double *eps, double *eta)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int nblk = (N + 1) / 2;
    for (int j = 0; j < nblk; ++j) {
        uint32_t ctr[4] = {(uint32_t)((uint64_t)p), (uint32_t)k, (uint32_t)j,
                           (uint32_t)((uint64_t)p >> 32)};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        double z[2];
        int a = 2 * j;
        orc_normal_pair(w[0], w[1], z);
        eps[a] = z[0];
        eta[a] = z[1];
        if (a + 1 < N) {
            orc_normal_pair(w[2], w[3], z);
            eps[a + 1] = z[0];
            eta[a + 1] = z[1];
        }
    }
}

/* Cholesky-Banachiewicz, row by row: C = L L^T with L lower triangular
 * (row-major, N x N, upper part zeroed).  Returns ORC_ENOTSPD when a pivot is
 * not positive. */
int orc_cholesky(int32_t N, const double *C, double *L)
{
    for (int i = 0; i < N * N; ++i) L[i] = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = C[i * N + j];
            for (int k = 0; k < j; ++k) s -= L[i * N + k] * L[j * N + k];
            if (i == j) {
                if (!(s > 0.0)) return ORC_ENOTSPD;
                L[i * N + i] = sqrt(s);
            } else {
                L[i * N + j] = s / L[j * N + j];
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One scenario of the model.  scheme: ORC_EULER_FT or ORC_QE. */
#define ORC_EULER_FT 0
#define ORC_QE 1
typedef struct {
    int32_t N;
    const double *S0, *v0, *kappa, *theta, *xi, *rho;
    double r;
    int32_t scheme;
} orc_model;

/* ------------------------------------------------------------------------ */
/* Andersen's quadratic-exponential (QE) step (Andersen 2008, the scheme the
 * paper's STAC-A2 code uses, Sec. 2.2 and 2.2.1), written from its definition.
 *
 * Variance: the next variance is drawn from a distribution with the exact
 * conditional mean m and variance s^2 of the CIR process over dt,
 *   m = theta + (v - theta) e^{-kappa dt},
 *   s^2 = v xi^2 e^{-kappa dt} (1 - e^{-kappa dt}) / kappa
 *         + theta xi^2 (1 - e^{-kappa dt})^2 / (2 kappa),
 * chosen by psi = s^2 / m^2 against psi_c = 1.5:
 *   psi <= psi_c: v' = a (b + Z_v)^2 with b^2 = 2/psi - 1 + sqrt(2/psi)
 *                 sqrt(2/psi - 1) and a = m / (1 + b^2);
 *   psi > psi_c:  p = (psi - 1)/(psi + 1), beta = (1 - p)/m, and with the
 *                 uniform U = Phi(Z_v): v' = 0 if U <= p, else
 *                 ln((1 - p)/(1 - U)) / beta.
 * (xi = 0: s^2 = 0 and v' = m.)  Log price, with gamma1 = gamma2 = 1/2:
 *   X' = X + r dt + K0 + K1 v + K2 v' + sqrt(K3 v + K4 v') Z_x,
 *   K0 = -rho kappa theta dt / xi, K1 = gamma1 dt (kappa rho/xi - 1/2) - rho/xi,
 *   K2 = gamma2 dt (kappa rho/xi - 1/2) + rho/xi, K3 = gamma1 dt (1 - rho^2),
 *   K4 = gamma2 dt (1 - rho^2)  (rho/xi read as 0 when xi = 0, which the
 *   interface allows only with rho = 0).
 * The K2 v' term carries rho times the variance shock, so Z_x is the part of
 * the spot shock orthogonal to the variance shock.  Random inputs per asset
 * and step (the paper's two numbers per element), with Z^S = L eps the
 * correlated spot normals of the Euler scheme:
 *   Z_v = rho Z^S_i + sqrt(1 - rho^2) eta_i   (the Euler scheme's Z^v),
 *   Z_x = sqrt(1 - rho^2) Z^S_i - rho eta_i,
 * independent unit normals whose spot combination rho Z_v + sqrt(1 - rho^2)
 * Z_x is Z^S_i itself: the spot shocks of different assets keep the
 * correlation C, and the variance shocks the Euler scheme's rho_i rho_j C_ij,
 * under both schemes.  For one asset (Z_v, Z_x) is a rotation of (eta, eps),
 * the same joint law. */
#define ORC_PSI_C 1.5

typedef struct {
    double E, mth, c1, c2, K0, K1, K2, K3, K4;
} qe_consts;

static void qe_consts_for(double kappa, double theta, double xi, double rho, double r, double dt,
                          qe_consts *q)
{
    const double E = exp(-kappa * dt);
    const double f = kappa > 0.0 ? -expm1(-kappa * dt) / kappa : dt; /* (1 - E)/kappa */
    const double g1 = 0.5, g2 = 0.5;
    const double rx = xi > 0.0 ? rho / xi : 0.0;
    q->E = E;
    q->mth = theta * (1.0 - E);
    q->c1 = xi * xi * E * f;
    q->c2 = 0.5 * theta * xi * xi * (1.0 - E) * f;
    q->K0 = r * dt - rx * kappa * theta * dt;
    q->K1 = g1 * dt * (kappa * rx - 0.5) - rx;
    q->K2 = g2 * dt * (kappa * rx - 0.5) + rx;
    q->K3 = g1 * dt * (1.0 - rho * rho);
    q->K4 = g2 * dt * (1.0 - rho * rho);
}

static double qe_variance(const qe_consts *q, double v, double zv)
{
    const double m = q->mth + v * q->E;
    const double s2 = v * q->c1 + q->c2;
    if (!(s2 > 0.0)) return m;
    const double psi = s2 / (m * m);
    if (psi <= ORC_PSI_C) {
        const double t = 2.0 / psi;
        const double b2 = t - 1.0 + sqrt(t) * sqrt(t - 1.0);
        const double a = m / (1.0 + b2);
        const double b = sqrt(b2);
        return a * (b + zv) * (b + zv);
    }
    const double p = (psi - 1.0) / (psi + 1.0);
    const double beta = (1.0 - p) / m;
    const double u = 0.5 * erfc(-zv / sqrt(2.0));
    return u <= p ? 0.0 : log((1.0 - p) / (1.0 - u)) / beta;
}

/* One QE step of the variance from v with normal zv (test access). */
double orc_qe_variance_step(double kappa, double theta, double xi, double rho, double dt, double v,
                            double zv)
{
    qe_consts q;
    qe_consts_for(kappa, theta, xi, rho, 0.0, dt, &q);
    return qe_variance(&q, v, zv);
}

/* Heston paths and the per-date LS path reduction for one scenario.
 *
 * Model (risk-neutral, no dividends), per asset i:
 *   dS_i = r S_i dt + sqrt(v_i) S_i dW^S_i,  dv_i = kappa_i (theta_i - v_i) dt
 *   + xi_i sqrt(v_i) dW^v_i.
 * Correlation: Z^S = L eps with L = chol(C); Z^v_i = rho_i Z^S_i +
 * sqrt(1 - rho_i^2) eta_i.
 * Scheme ORC_EULER_FT: full-truncation Euler (Lord, Koekkoek & van Dijk 2010)
 * in log price:
 *   v+ = max(v, 0);  X += (r - v+/2) dt + sqrt(v+ dt) Z^S;
 *   v += kappa (theta - v+) dt + xi sqrt(v+ dt) Z^v;  S = S0 exp(X), X_0 = 0.
 * Scheme ORC_QE: the quadratic-exponential step above, with Z_v and Z_x
 * formed from Z^S and eta as stated there (v stays >= 0, so max(v, 0) = v).
 * Reduction at each date k = 1..n (Sec. 4.1): U = max_i S_i (U = S for one
 * asset) and A = (1/N) sum_i max(v_i, 0).
 * Output feat[((k-1) P + p) * 2 + {0,1}] = (U, A). */
/* One path p: n steps from X = 0, v = v0; writes (U, A) of date k = 1..n to
 * out[(k-1) stride * 2 + {0,1}].  work holds 5 N doubles. */
/* Step k (date k to k + 1) of every asset of path p: (X, v) in place.  work
 * holds 3 N doubles. */
static void step(const orc_model *m, const double *L, double dt, int32_t k, int64_t p,
                 uint64_t seed, double *X, double *v, double *work)
{
    const int N = m->N;
    double *eps = work, *eta = work + N, *ZS = work + 2 * N;
    orc_normals(N, seed, p, k, eps, eta);
    for (int a = 0; a < N; ++a) {
        double z = 0.0;
        for (int b = 0; b <= a; ++b) z += L[a * N + b] * eps[b];
        ZS[a] = z;
    }
    if (m->scheme == ORC_QE) {
        for (int a = 0; a < N; ++a) {
            qe_consts q;
            qe_consts_for(m->kappa[a], m->theta[a], m->xi[a], m->rho[a], m->r, dt, &q);
            const double rho = m->rho[a], rhobar = sqrt(1.0 - rho * rho);
            const double Zv = rho * ZS[a] + rhobar * eta[a];
            const double Zx = rhobar * ZS[a] - rho * eta[a];
            const double vn = qe_variance(&q, v[a], Zv);
            X[a] = X[a] + q.K0 + q.K1 * v[a] + q.K2 * vn + sqrt(q.K3 * v[a] + q.K4 * vn) * Zx;
            v[a] = vn;
        }
    } else
    for (int a = 0; a < N; ++a) {
        double rho = m->rho[a];
        double Zv = rho * ZS[a] + sqrt(1.0 - rho * rho) * eta[a];
        double vp = v[a] > 0.0 ? v[a] : 0.0;
        double sq = sqrt(vp * dt);
        X[a] = X[a] + (m->r - 0.5 * vp) * dt + sq * ZS[a];
        v[a] = v[a] + m->kappa[a] * (m->theta[a] - vp) * dt + m->xi[a] * sq * Zv;
    }
}

static void one_path(const orc_model *m, const double *L, double dt, int32_t n, int64_t p,
                     uint64_t seed, double *work, double *out, int64_t stride)
{
    const int N = m->N;
    double *X = work, *v = work + N;
    for (int a = 0; a < N; ++a) {
        X[a] = 0.0;
        v[a] = m->v0[a];
    }
    for (int32_t k = 0; k < n; ++k) {
        step(m, L, dt, k, p, seed, X, v, work + 2 * N);
        double U = -INFINITY, sv = 0.0;
        for (int a = 0; a < N; ++a) {
            double S = m->S0[a] * exp(X[a]);
            if (S > U) U = S;
            sv += v[a] > 0.0 ? v[a] : 0.0;
        }
        double *f = out + (int64_t)k * stride * 2;
        f[0] = U;
        f[1] = sv / (double)N;
    }
}

int orc_features(const orc_model *m, const double *C, double T, int32_t n, int64_t P,
                 uint64_t seed, int32_t nthreads, double *feat)
{
    const int N = m->N;
    if (N < 1 || n < 1 || P < 1 || !(T > 0.0)) return ORC_EINVAL;
    double *L = (double *)malloc(sizeof(double) * N * N);
    if (!L) return ORC_ENOMEM;
    int st = orc_cholesky(N, C, L);
    if (st != ORC_OK) {
        free(L);
        return st;
    }
    const double dt = T / (double)n;
    const int64_t nchunk = (P + ORC_CHUNK - 1) / ORC_CHUNK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * N * 5);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nchunk; ++c) {
            int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
            for (int64_t p = c * ORC_CHUNK; p < pend; ++p)
                one_path(m, L, dt, n, p, seed, work, feat + p * 2, P);
        }
        free(work);
    }
    free(L);
    return ORC_OK;
}

/* The same paths for a list of path indices (any p >= 0, so single paths of a
 * large run can be checked): feat[(i n + k - 1) * 2 + {0,1}] for path paths[i]. */
int orc_features_at(const orc_model *m, const double *C, double T, int32_t n, int64_t npaths,
                    const int64_t *paths, uint64_t seed, double *feat)
{
    const int N = m->N;
    if (N < 1 || n < 1 || npaths < 0 || !(T > 0.0)) return ORC_EINVAL;
    double *L = (double *)malloc(sizeof(double) * N * N);
    double *work = (double *)malloc(sizeof(double) * N * 5);
    if (!L || !work) {
        free(L); free(work);
        return ORC_ENOMEM;
    }
    int st = orc_cholesky(N, C, L);
    if (st == ORC_OK) {
        const double dt = T / (double)n;
        for (int64_t i = 0; i < npaths; ++i) {
            if (paths[i] < 0) { st = ORC_EINVAL; break; }
            one_path(m, L, dt, n, paths[i], seed, work, feat + i * (int64_t)n * 2, 1);
        }
    }
    free(L);
    free(work);
    return st;
}

/* Per-asset state after n steps of every path p < P (test access: the joint
 * law of the assets' log prices and variances):
 * out[(p N + a) * 2 + {0,1}] = (X_{a,n}, v_{a,n}), X from 0. */
int orc_states(const orc_model *m, const double *C, double T, int32_t n, int64_t P,
               uint64_t seed, int32_t nthreads, double *out)
{
    const int N = m->N;
    if (N < 1 || n < 1 || P < 1 || !(T > 0.0)) return ORC_EINVAL;
    double *L = (double *)malloc(sizeof(double) * N * N);
    if (!L) return ORC_ENOMEM;
    int st = orc_cholesky(N, C, L);
    if (st != ORC_OK) {
        free(L);
        return st;
    }
    const double dt = T / (double)n;
    const int64_t nchunk = (P + ORC_CHUNK - 1) / ORC_CHUNK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * N * 5);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nchunk; ++c) {
            int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
            for (int64_t p = c * ORC_CHUNK; p < pend; ++p) {
                double *X = work, *v = work + N;
                for (int a = 0; a < N; ++a) {
                    X[a] = 0.0;
                    v[a] = m->v0[a];
                }
                for (int32_t k = 0; k < n; ++k) step(m, L, dt, k, p, seed, X, v, work + 2 * N);
                for (int a = 0; a < N; ++a) {
                    out[(p * N + a) * 2] = X[a];
                    out[(p * N + a) * 2 + 1] = v[a];
                }
            }
        }
        free(work);
    }
    free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Longstaff-Schwartz (2001) regression-based exercise, cited in Sec. 2.2 and
 * kept as a quadratic curve fit in Sec. 2.2.1.
 *
 * Payoff h = max(K - U, 0) (put) or max(U - K, 0) (call).  Exercise dates are
 * k = 1..n (not k = 0).  Regression set at date k: paths with h_k > 0.
 * Basis (m = 3): 1, x, x^2; (m = 5): 1, x, x^2, w, x w; with x = (U - cU)/K and
 * w = (A - cA)/theta_bar, where cU, cA are the means of U and A over the
 * regression set at that date.  (Centering and scaling leave the span, hence
 * the fitted values, unchanged in exact arithmetic.)  The fit solves the
 * normal equations by Cholesky; a date with fewer than m regression paths or
 * a pivot at or below 1e-12 of its diagonal entry is skipped (no exercise).
 * Exercise iff h_k > fitted continuation value (strict). */

static double payoff(int cp, double K, double U)
{
    double h = (cp == ORC_PUT) ? K - U : U - K;
    return h > 0.0 ? h : 0.0;
}

static void basis(int m, double U, double A, double cU, double cA, double K, double tbar,
                  double *phi)
{
    double x = (U - cU) / K;
    phi[0] = 1.0;
    phi[1] = x;
    phi[2] = x * x;
    if (m == 5) {
        double w = (A - cA) / tbar;
        phi[3] = w;
        phi[4] = x * w;
    }
}

/* Solve G beta = b for symmetric G (m x m) by Cholesky; 0 on success, -1 if a
 * pivot is not above 1e-12 of its diagonal entry. */
static int chol_solve(int m, const double *G, const double *b, double *beta)
{
    double L[25];
    double y[5];
    for (int i = 0; i < m * m; ++i) L[i] = 0.0;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = G[i * m + j];
            for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
            if (i == j) {
                if (!(s > 1e-12 * G[i * m + i])) return -1;
                L[i * m + i] = sqrt(s);
            } else {
                L[i * m + j] = s / L[j * m + j];
            }
        }
    }
    for (int i = 0; i < m; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * m + k] * y[k];
        y[i] = s / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * beta[k];
        beta[i] = s / L[i * m + i];
    }
    return 0;
}

/* Price from a feature array (one scenario).  out[0] = V = (1/P) sum_p CF_p
 * exp(-r tau_p dt); out[1] = standard error s/sqrt(P) with the (P-1) sample
 * standard deviation.  Optional outputs: tau[P], cf[P]; *skipped = number of
 * dates whose regression was skipped.  style EUROPEAN uses date n only. */
int orc_lsmc(const double *feat, int64_t P, int32_t n, double T, double r, double K, int32_t cp,
             int32_t style, int32_t m, double theta_bar, int32_t nthreads, double *out,
             int32_t *tau_out, double *cf_out, int64_t *skipped)
{
    if (P < 2 || n < 1 || !(T > 0.0) || (m != 3 && m != 5)) return ORC_EINVAL;
    const double dt = T / (double)n;
    const int64_t nchunk = (P + ORC_CHUNK - 1) / ORC_CHUNK;
    double *CF = (double *)malloc(sizeof(double) * P);
    int32_t *tau = (int32_t *)malloc(sizeof(int32_t) * P);
    /* per-chunk partial sums: count, sum U, sum A, G (m*m), b (m) */
    const int NS = 3 + 25 + 5;
    double *part = (double *)malloc(sizeof(double) * NS * nchunk);
    if (!CF || !tau || !part) {
        free(CF); free(tau); free(part);
        return ORC_ENOMEM;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int64_t p = 0; p < P; ++p) {
        CF[p] = payoff(cp, K, feat[((int64_t)(n - 1) * P + p) * 2]);
        tau[p] = n;
    }
    int64_t nskip = 0;
    if (style == ORC_AMERICAN) {
        for (int32_t k = n - 1; k >= 1; --k) {
            const double *fk = feat + (int64_t)(k - 1) * P * 2;
            /* pass 1: regression-set size and means */
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < nchunk; ++c) {
                double cnt = 0.0, su = 0.0, sa = 0.0;
                int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
                for (int64_t p = c * ORC_CHUNK; p < pend; ++p) {
                    double U = fk[p * 2], A = fk[p * 2 + 1];
                    if (payoff(cp, K, U) > 0.0) {
                        cnt += 1.0;
                        su += U;
                        sa += A;
                    }
                }
                part[c * NS + 0] = cnt;
                part[c * NS + 1] = su;
                part[c * NS + 2] = sa;
            }
            double cnt = 0.0, su = 0.0, sa = 0.0;
            for (int64_t c = 0; c < nchunk; ++c) {
                cnt += part[c * NS + 0];
                su += part[c * NS + 1];
                sa += part[c * NS + 2];
            }
            if (cnt < (double)m) {
                ++nskip;
                continue;
            }
            const double cU = su / cnt, cA = sa / cnt;
            /* pass 2: normal equations over the regression set */
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < nchunk; ++c) {
                double G[25], b[5], phi[5];
                for (int i = 0; i < 25; ++i) G[i] = 0.0;
                for (int i = 0; i < 5; ++i) b[i] = 0.0;
                int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
                for (int64_t p = c * ORC_CHUNK; p < pend; ++p) {
                    double U = fk[p * 2], A = fk[p * 2 + 1];
                    if (!(payoff(cp, K, U) > 0.0)) continue;
                    basis(m, U, A, cU, cA, K, theta_bar, phi);
                    double Y = CF[p] * exp(-r * (double)(tau[p] - k) * dt);
                    for (int i = 0; i < m; ++i) {
                        for (int j = 0; j < m; ++j) G[i * m + j] += phi[i] * phi[j];
                        b[i] += phi[i] * Y;
                    }
                }
                for (int i = 0; i < 25; ++i) part[c * NS + 3 + i] = G[i];
                for (int i = 0; i < 5; ++i) part[c * NS + 28 + i] = b[i];
            }
            double G[25], b[5], beta[5];
            for (int i = 0; i < 25; ++i) G[i] = 0.0;
            for (int i = 0; i < 5; ++i) b[i] = 0.0;
            for (int64_t c = 0; c < nchunk; ++c) {
                for (int i = 0; i < m * m; ++i) G[i] += part[c * NS + 3 + i];
                for (int i = 0; i < m; ++i) b[i] += part[c * NS + 28 + i];
            }
            if (chol_solve(m, G, b, beta) != 0) {
                ++nskip;
                continue;
            }
            /* exercise decision */
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < nchunk; ++c) {
                double phi[5];
                int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
                for (int64_t p = c * ORC_CHUNK; p < pend; ++p) {
                    double U = fk[p * 2], A = fk[p * 2 + 1];
                    double h = payoff(cp, K, U);
                    if (!(h > 0.0)) continue;
                    basis(m, U, A, cU, cA, K, theta_bar, phi);
                    double cont = 0.0;
                    for (int i = 0; i < m; ++i) cont += phi[i] * beta[i];
                    if (h > cont) {
                        CF[p] = h;
                        tau[p] = k;
                    }
                }
            }
        }
    }
    /* price and standard error (two passes: mean, then squared deviations) */
    double s1 = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) {
        double a1 = 0.0;
        int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
        for (int64_t p = c * ORC_CHUNK; p < pend; ++p) a1 += CF[p] * exp(-r * (double)tau[p] * dt);
        s1 += a1;
    }
    const double mean = s1 / (double)P;
    double s2 = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) {
        double a2 = 0.0;
        int64_t pend = (c + 1) * ORC_CHUNK < P ? (c + 1) * ORC_CHUNK : P;
        for (int64_t p = c * ORC_CHUNK; p < pend; ++p) {
            double d = CF[p] * exp(-r * (double)tau[p] * dt) - mean;
            a2 += d * d;
        }
        s2 += a2;
    }
    out[0] = mean;
    out[1] = sqrt(s2 / (double)(P - 1) / (double)P);
    if (tau_out) memcpy(tau_out, tau, sizeof(int32_t) * P);
    if (cf_out) memcpy(cf_out, CF, sizeof(double) * P);
    if (skipped) *skipped = nskip;
    free(CF);
    free(tau);
    free(part);
    return ORC_OK;
}

/* Decision replay: the price of a given exercise-date vector tau (e.g. one
 * exported by another implementation), re-evaluated in FP64 on this feature
 * array: V = (1/P) sum_p h_{tau_p}(p) exp(-r tau_p dt), with the same SE. */
int orc_replay(const double *feat, int64_t P, int32_t n, double T, double r, double K, int32_t cp,
               const int32_t *tau, double *out)
{
    if (P < 2 || n < 1 || !(T > 0.0)) return ORC_EINVAL;
    const double dt = T / (double)n;
    double s1 = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        int32_t t = tau[p];
        if (t < 1 || t > n) return ORC_EINVAL;
        s1 += payoff(cp, K, feat[((int64_t)(t - 1) * P + p) * 2]) * exp(-r * (double)t * dt);
    }
    const double mean = s1 / (double)P;
    double s2 = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        int32_t t = tau[p];
        double d = payoff(cp, K, feat[((int64_t)(t - 1) * P + p) * 2]) * exp(-r * (double)t * dt) - mean;
        s2 += d * d;
    }
    out[0] = mean;
    out[1] = sqrt(s2 / (double)(P - 1) / (double)P);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Greek sets: bump-and-revalue with common random numbers.
 * Scenario order: base; spot+ for assets 0..N-1; spot- for 0..N-1 (if
 * DELTA_GAMMA); v0 up for 0..N-1 (VEGA); T - dT (THETA); r + dr (RHO);
 * C_ij + dc for i < j in lexicographic order (CORR, N > 1). */
int64_t orc_num_scenarios(int32_t N, uint32_t mask)
{
    int64_t S = 1;
    if (mask & ORC_DELTA_GAMMA) S += 2 * (int64_t)N;
    if (mask & ORC_VEGA) S += N;
    if (mask & ORC_THETA) S += 1;
    if (mask & ORC_RHO) S += 1;
    if ((mask & ORC_CORR) && N > 1) S += (int64_t)N * (N - 1) / 2;
    return S;
}

typedef struct {
    int32_t N;
    const double *S0, *v0, *kappa, *theta, *xi, *rho;
    double r;
    const double *C;
    int32_t cp, style, m;
    double K, T;
    int64_t P;
    int32_t n;
    uint32_t mask;
    double spot_rel, v0_rel, T_abs, r_abs, corr_abs;
    uint64_t seed;
    int32_t nthreads;
    int32_t scheme;
} orc_request;

/* Prices of every scenario of the Greek set.  prices/ses/skipped have
 * orc_num_scenarios entries; tau_all (optional) has that many rows of P.
 * With replay_tau (optional, same shape) each scenario is not regressed but
 * priced with the given exercise dates (decision replay). */
static int price_scenarios(const orc_request *q, double *prices, double *ses, int64_t *skipped,
                           int32_t *tau_all, const int32_t *replay_tau, double *dcf_all);

int orc_price_scenarios(const orc_request *q, double *prices, double *ses, int64_t *skipped,
                        int32_t *tau_all)
{
    return price_scenarios(q, prices, ses, skipped, tau_all, NULL, NULL);
}

int orc_price_scenarios_replay(const orc_request *q, double *prices, double *ses,
                               int64_t *skipped, int32_t *tau_all, const int32_t *replay_tau)
{
    return price_scenarios(q, prices, ses, skipped, tau_all, replay_tau, NULL);
}

/* The same, also returning each path's discounted cash flow CF_p exp(-r tau_p
 * dt) per scenario in dcf_all [S][P] (the terms whose mean is the price; the
 * tests take the Monte Carlo standard error of a finite-difference Greek over
 * the paths from it). */
int orc_price_scenarios_dcf(const orc_request *q, double *prices, double *ses, int64_t *skipped,
                            int32_t *tau_all, double *dcf_all)
{
    return price_scenarios(q, prices, ses, skipped, tau_all, NULL, dcf_all);
}

static int price_scenarios(const orc_request *q, double *prices, double *ses, int64_t *skipped,
                           int32_t *tau_all, const int32_t *replay_tau, double *dcf_all)
{
    const int N = q->N;
    if (N < 1 || q->P < 2 || q->n < 1) return ORC_EINVAL;
    const int64_t S = orc_num_scenarios(N, q->mask);
    double tbar = 0.0;
    for (int a = 0; a < N; ++a) tbar += q->theta[a];
    tbar /= (double)N;
    double *S0 = (double *)malloc(sizeof(double) * N * 2 + sizeof(double) * N * N);
    double *v0 = S0 + N;
    double *C = v0 + N;
    double *feat = (double *)malloc(sizeof(double) * 2 * (size_t)q->n * (size_t)q->P);
    if (!S0 || !feat) {
        free(S0); free(feat);
        return ORC_ENOMEM;
    }
    int st = ORC_OK;
    for (int64_t s = 0; s < S && st == ORC_OK; ++s) {
        memcpy(S0, q->S0, sizeof(double) * N);
        memcpy(v0, q->v0, sizeof(double) * N);
        memcpy(C, q->C, sizeof(double) * N * N);
        double r = q->r, T = q->T;
        int64_t idx = s;
        if (idx > 0) {
            idx -= 1;
            int done = 0;
            if (!done && (q->mask & ORC_DELTA_GAMMA)) {
                if (idx < N) { S0[idx] = q->S0[idx] * (1.0 + q->spot_rel); done = 1; }
                else if (idx < 2 * N) { S0[idx - N] = q->S0[idx - N] * (1.0 - q->spot_rel); done = 1; }
                else idx -= 2 * N;
            }
            if (!done && (q->mask & ORC_VEGA)) {
                if (idx < N) { v0[idx] = q->v0[idx] * (1.0 + q->v0_rel); done = 1; }
                else idx -= N;
            }
            if (!done && (q->mask & ORC_THETA)) {
                if (idx == 0) { T = q->T - q->T_abs; done = 1; }
                else idx -= 1;
            }
            if (!done && (q->mask & ORC_RHO)) {
                if (idx == 0) { r = q->r + q->r_abs; done = 1; }
                else idx -= 1;
            }
            if (!done && (q->mask & ORC_CORR) && N > 1) {
                int64_t t = 0;
                for (int i = 0; i < N && !done; ++i)
                    for (int j = i + 1; j < N && !done; ++j, ++t)
                        if (t == idx) {
                            C[i * N + j] += q->corr_abs;
                            C[j * N + i] += q->corr_abs;
                            done = 1;
                        }
            }
            if (!done) { st = ORC_EINVAL; break; }
        }
        orc_model mm = {N, S0, v0, q->kappa, q->theta, q->xi, q->rho, r, q->scheme};
        st = orc_features(&mm, C, T, q->n, q->P, q->seed, q->nthreads, feat);
        if (st != ORC_OK) break;
        double out[2];
        int64_t sk = 0;
        if (replay_tau) {
            st = orc_replay(feat, q->P, q->n, T, r, q->K, q->cp, replay_tau + s * q->P, out);
        } else if (dcf_all) {
            int32_t *tau = (int32_t *)malloc(sizeof(int32_t) * q->P);
            double *cf = dcf_all + s * q->P;
            if (!tau) { st = ORC_ENOMEM; break; }
            st = orc_lsmc(feat, q->P, q->n, T, r, q->K, q->cp, q->style, q->m, tbar, q->nthreads,
                          out, tau, cf, &sk);
            const double dt = T / (double)q->n;
            for (int64_t p = 0; p < q->P; ++p) cf[p] = cf[p] * exp(-r * (double)tau[p] * dt);
            if (tau_all) memcpy(tau_all + s * q->P, tau, sizeof(int32_t) * q->P);
            free(tau);
        } else {
            st = orc_lsmc(feat, q->P, q->n, T, r, q->K, q->cp, q->style, q->m, tbar, q->nthreads,
                          out, tau_all ? tau_all + s * q->P : NULL, NULL, &sk);
        }
        if (st != ORC_OK) break;
        prices[s] = out[0];
        ses[s] = out[1];
        if (skipped) skipped[s] = sk;
    }
    free(S0);
    free(feat);
    return st;
}

/* Finite-difference Greeks from scenario prices (same scenario order).
 *   delta_i = (V+ - V-)/(2 h S0_i);  gamma_i = (V+ - 2V + V-)/(h S0_i)^2;
 *   vega_i = (V(v0_i (1+hv)) - V)/(hv v0_i);  theta = (V(T - dT) - V)/dT;
 *   rho = (V(r + dr) - V)/dr;  corr_ij = (V(C_ij + dc) - V)/dc. */
int orc_greeks(int32_t N, uint32_t mask, const double *S0, const double *v0, double spot_rel,
               double v0_rel, double T_abs, double r_abs, double corr_abs, const double *prices,
               double *delta, double *gamma, double *vega, double *theta, double *rho,
               double *corr)
{
    const double V = prices[0];
    int64_t s = 1;
    if (mask & ORC_DELTA_GAMMA) {
        for (int i = 0; i < N; ++i) {
            double up = prices[s + i], dn = prices[s + N + i];
            double hs = spot_rel * S0[i];
            delta[i] = (up - dn) / (2.0 * hs);
            gamma[i] = (up - 2.0 * V + dn) / (hs * hs);
        }
        s += 2 * N;
    }
    if (mask & ORC_VEGA) {
        for (int i = 0; i < N; ++i) vega[i] = (prices[s + i] - V) / (v0_rel * v0[i]);
        s += N;
    }
    if (mask & ORC_THETA) {
        *theta = (prices[s] - V) / T_abs;
        s += 1;
    }
    if (mask & ORC_RHO) {
        *rho = (prices[s] - V) / r_abs;
        s += 1;
    }
    if ((mask & ORC_CORR) && N > 1) {
        int64_t t = 0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j, ++t) corr[t] = (prices[s + t] - V) / corr_abs;
    }
    return ORC_OK;
}
