/*
 * Reference (oracle) implementation of Subsampling SMC for static Bayesian
 * GLMs (Gunawan, Dang, Quiroz, Kohn, Tran, arXiv:1805.03317).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. It shares no code, header,
 * table or helper with the GPU library and must never be used as a fallback
 * for it.
 *
 * Precision.  Everything is IEEE binary64 except:
 *   - the per-observation remainder d_k = l_k - q_k and its derivative, which
 *     are evaluated by their definition (section 3.2) in binary128 so that the
 *     cancellation between l_k and q_k does not destroy them;
 *   - the m-term sums of the estimator, which are accumulated in binary128;
 *   - the n-term full-data sums A, B, C (section 3.2), accumulated in the
 *     x87 80-bit format.
 * Results are rounded to binary64 on output.
 *
 * Random numbers: one counter-based generator, Philox4x64-10 (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by
 * (seed, 0) with the counter layout
 *   word0 = purpose<<56 | stage<<32 | move<<16 | dataset
 *   word1 = particle, word2 = draw>>2, word3 = 0, output word = draw & 3.
 * Purposes: 0 prior normals, 1 initial subsample, 2 resampling (systematic
 * offset: particle 0 draw 0; multinomial slot k: particle k draw 1),
 * 3 block choice, 4 block indices, 5 u-accept uniform, 6 momentum normals,
 * 7 theta-accept uniform.
 *
 * Parity unpinned: none of the functions below is unpinned; the pins live
 * in the CPU test suite (tests/test_oracle_*.py).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 qd;
typedef long double xd;

enum { ORC_LOGISTIC = 0, ORC_POISSON = 1, ORC_GAUSSIAN = 2, ORC_STUDENT_T = 3 };

/* Student-t regression (Experiment 2): y = x'theta + e, e ~ t_5 with unit
 * scale, l(eta) = log t_5(y - eta). */
#define ORC_T_NU 5
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_NOT_PD = 4, ORC_ERR_NONFINITE = 5 };

/* One dataset: row k of Xy holds x_k (d values) followed by y_k at column d. */
typedef struct {
    int32_t family;
    int32_t cv_order;   /* 2: second-order Taylor control variate; 1: first order */
    int64_t n;
    int32_t d;
    int32_t ld;
    const double *Xy;
    double gauss_s2;    /* noise variance of the Gaussian test family */
} orc_data;

/* Control-variate summaries around theta_bar (section 3.2). */
typedef struct {
    const double *theta_bar; /* d */
    double A;
    const double *B;         /* d */
    const double *C;         /* d*d, row-major */
} orc_cv;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10                                                             */
/* ------------------------------------------------------------------------ */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint64_t orc_rng_word(uint64_t seed, uint32_t purpose, uint32_t stage, uint32_t move,
                      uint32_t dataset, uint64_t particle, uint64_t draw)
{
    uint64_t ctr[4], key[2], out[4];
    ctr[0] = ((uint64_t)(purpose & 0xFF) << 56) | ((uint64_t)(stage & 0xFFFFFF) << 32) |
             ((uint64_t)(move & 0xFFFF) << 16) | (uint64_t)(dataset & 0xFFFF);
    ctr[1] = particle;
    ctr[2] = draw >> 2;
    ctr[3] = 0;
    key[0] = seed;
    key[1] = 0;
    orc_philox4x64_10(ctr, key, out);
    return out[draw & 3];
}

/* uniform index in {0..n-1}: floor(w * n / 2^64) */
static int64_t rng_index(uint64_t w, int64_t n)
{
    return (int64_t)(((unsigned __int128)w * (uint64_t)n) >> 64);
}

/* uniform in (0, 1] */
static double rng_uniform_open0(uint64_t w)
{
    return ((double)(w >> 11) + 1.0) * 0x1.0p-53;
}

/* k-th standard normal of a stream, Box-Muller on words (2*(k/2), 2*(k/2)+1). */
static double rng_normal(uint64_t seed, uint32_t purpose, uint32_t stage, uint32_t move,
                         uint32_t dataset, uint64_t particle, uint64_t k)
{
    uint64_t base = 2 * (k / 2);
    uint64_t wa = orc_rng_word(seed, purpose, stage, move, dataset, particle, base);
    uint64_t wb = orc_rng_word(seed, purpose, stage, move, dataset, particle, base + 1);
    double u1 = rng_uniform_open0(wa);
    double u2 = (double)(wb >> 11) * 0x1.0p-53;
    double r = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    return (k & 1) ? r * sin(ang) : r * cos(ang);
}

double orc_normal(uint64_t seed, uint32_t purpose, uint32_t stage, uint32_t move,
                  uint32_t dataset, uint64_t particle, uint64_t k)
{
    return rng_normal(seed, purpose, stage, move, dataset, particle, k);
}

/* ------------------------------------------------------------------------ */
/* Per-observation log-density and its eta-derivatives                       */
/* logistic: Exp. 1; Poisson with log link and Student-t (t_5, unit scale):  */
/* Exp. 2; Gaussian: test family                                             */
/* ------------------------------------------------------------------------ */

static qd q_softplus(qd x)
{
    return x > 0 ? x + log1pq(expq(-x)) : log1pq(expq(x));
}

static qd q_sigmoid(qd x)
{
    if (x >= 0) return 1 / (1 + expq(-x));
    qd e = expq(x);
    return e / (1 + e);
}

static qd q_f0(int fam, qd y, qd eta, qd s2)
{
    switch (fam) {
    case ORC_LOGISTIC: return y * eta - q_softplus(eta);
    case ORC_POISSON:  return y * eta - expq(eta) - lgammaq(y + 1);
    case ORC_STUDENT_T: {
        const qd nu = ORC_T_NU, r = y - eta;
        return lgammaq((nu + 1) / 2) - lgammaq(nu / 2) - 0.5Q * logq(nu * M_PIq) - (nu + 1) / 2 * log1pq(r * r / nu);
    }
    default: {
        qd r = y - eta;
        return -0.5Q * logq(2 * M_PIq * s2) - r * r / (2 * s2);
    }
    }
}

static qd q_f1(int fam, qd y, qd eta, qd s2)
{
    switch (fam) {
    case ORC_LOGISTIC: return y - q_sigmoid(eta);
    case ORC_POISSON:  return y - expq(eta);
    case ORC_STUDENT_T: { const qd nu = ORC_T_NU, r = y - eta; return (nu + 1) * r / (nu + r * r); }
    default:           return (y - eta) / s2;
    }
}

static qd q_f2(int fam, qd y, qd eta, qd s2)
{
    switch (fam) {
    case ORC_LOGISTIC: { qd s = q_sigmoid(eta); return -s * (1 - s); }
    case ORC_POISSON:  return -expq(eta);
    case ORC_STUDENT_T: {
        const qd nu = ORC_T_NU, r = y - eta, t = nu + r * r;
        return (nu + 1) * (r * r - nu) / (t * t);
    }
    default:           return -1 / s2;
    }
}

/* Same three functions in 80-bit, for the full-data sums. */
static xd x_softplus(xd x) { return x > 0 ? x + log1pl(expl(-x)) : log1pl(expl(x)); }
static xd x_sigmoid(xd x)
{
    if (x >= 0) return 1 / (1 + expl(-x));
    xd e = expl(x);
    return e / (1 + e);
}
static void x_derivs(int fam, xd y, xd eta, xd s2, xd *f0, xd *f1, xd *f2)
{
    switch (fam) {
    case ORC_LOGISTIC: {
        xd s = x_sigmoid(eta);
        *f0 = y * eta - x_softplus(eta);
        *f1 = y - s;
        *f2 = -s * (1 - s);
        break;
    }
    case ORC_POISSON: {
        xd mu = expl(eta);
        *f0 = y * eta - mu - lgammal(y + 1);
        *f1 = y - mu;
        *f2 = -mu;
        break;
    }
    case ORC_STUDENT_T: {
        const xd nu = ORC_T_NU, r = y - eta, t = nu + r * r;
        *f0 = lgammal((nu + 1) / 2) - lgammal(nu / 2) - 0.5L * logl(nu * (xd)M_PI) - (nu + 1) / 2 * log1pl(r * r / nu);
        *f1 = (nu + 1) * r / t;
        *f2 = (nu + 1) * (r * r - nu) / (t * t);
        break;
    }
    default: {
        xd r = y - eta;
        *f0 = -0.5L * logl(2 * (xd)M_PI * s2) - r * r / (2 * s2);
        *f1 = r / s2;
        *f2 = -1 / s2;
    }
    }
}

/*
 * d_k = l_k(theta) - q_k(theta) and its eta-derivative, from the Taylor
 * control variate of section 3.2:
 *   q_k = f(eta_bar) + f'(eta_bar) Delta + 1/2 f''(eta_bar) Delta^2,
 *   Delta = x_k'(theta - theta_bar)   (the last term only for cv_order 2).
 * grad_theta d_k = dprime * x_k with dprime = f'(eta) - f'(eta_bar) - f''(eta_bar) Delta.
 */
static void q_remainder(const orc_data *D, qd y, qd eta_bar, qd Delta, qd *d_out, qd *dp_out)
{
    qd s2 = (qd)D->gauss_s2;
    qd eta = eta_bar + Delta;
    qd f0b = q_f0(D->family, y, eta_bar, s2);
    qd f1b = q_f1(D->family, y, eta_bar, s2);
    qd f2b = q_f2(D->family, y, eta_bar, s2);
    qd q = f0b + f1b * Delta;
    qd qp = f1b;
    if (D->cv_order == 2) {
        q += 0.5Q * f2b * Delta * Delta;
        qp += f2b * Delta;
    }
    *d_out = q_f0(D->family, y, eta, s2) - q;
    *dp_out = q_f1(D->family, y, eta, s2) - qp;
}

void orc_remainder(const orc_data *D, double y, double eta_bar, double Delta,
                   double *d_out, double *dp_out)
{
    qd dq, dpq;
    q_remainder(D, (qd)y, (qd)eta_bar, (qd)Delta, &dq, &dpq);
    *d_out = (double)dq;
    *dp_out = (double)dpq;
}

/* ------------------------------------------------------------------------ */
/* Full-data control-variate summaries A, B, C at theta_bar (section 3.2)    */
/* ------------------------------------------------------------------------ */

void orc_cv_build(const orc_data *D, const double *theta_bar, double *A, double *B, double *C)
{
    const int d = D->d;
    xd Aacc = 0;
    xd *Bacc = calloc((size_t)d, sizeof(xd));
    xd *Cacc = calloc((size_t)d * d, sizeof(xd));
    for (int64_t k = 0; k < D->n; ++k) {
        const double *row = D->Xy + k * (int64_t)D->ld;
        xd eta = 0;
        for (int c = 0; c < d; ++c) eta += (xd)row[c] * (xd)theta_bar[c];
        xd f0, f1, f2;
        x_derivs(D->family, (xd)row[d], eta, (xd)D->gauss_s2, &f0, &f1, &f2);
        Aacc += f0;
        for (int r = 0; r < d; ++r) {
            xd xr = row[r];
            Bacc[r] += f1 * xr;
            for (int c = 0; c < d; ++c) Cacc[(size_t)r * d + c] += f2 * xr * (xd)row[c];
        }
    }
    *A = (double)Aacc;
    for (int r = 0; r < d; ++r) B[r] = (double)Bacc[r];
    for (int i = 0; i < d * d; ++i) C[i] = (double)Cacc[i];
    free(Bacc);
    free(Cacc);
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (textbook Cholesky)                            */
/* ------------------------------------------------------------------------ */

/* S = L L' with L lower triangular (row-major, upper part set to 0). */
int orc_cholesky(int d, const double *S, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)d * d);
    for (int j = 0; j < d; ++j) {
        double s = S[(size_t)j * d + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * d + k] * L[(size_t)j * d + k];
        if (!(s > 0)) return ORC_ERR_NOT_PD;
        double ljj = sqrt(s);
        L[(size_t)j * d + j] = ljj;
        for (int i = j + 1; i < d; ++i) {
            double t = S[(size_t)i * d + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * d + k] * L[(size_t)j * d + k];
            L[(size_t)i * d + j] = t / ljj;
        }
    }
    return ORC_OK;
}

/* Solve L' x = z (back substitution). */
static void solve_upper_from_lower(int d, const double *L, const double *z, double *x)
{
    for (int k = d - 1; k >= 0; --k) {
        double t = z[k];
        for (int j = k + 1; j < d; ++j) t -= L[(size_t)j * d + k] * x[j];
        x[k] = t / L[(size_t)k * d + k];
    }
}

/* Solve L y = b (forward substitution). */
static void solve_lower(int d, const double *L, const double *b, double *y)
{
    for (int k = 0; k < d; ++k) {
        double t = b[k];
        for (int j = 0; j < k; ++j) t -= L[(size_t)k * d + j] * y[j];
        y[k] = t / L[(size_t)k * d + k];
    }
}

/* ------------------------------------------------------------------------ */
/* Posterior mode by Newton's method on l(theta) + log p(theta), used as the  */
/* control-variate centre theta_bar (section 3.2 asks only for an estimate   */
/* of posterior location).                                                   */
/* ------------------------------------------------------------------------ */

static double log_prior_quad(int d, const double *mu0, const double *Q0, const double *th)
{
    double s = 0;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            s += (th[r] - mu0[r]) * Q0[(size_t)r * d + c] * (th[c] - mu0[c]);
    return -0.5 * s;
}

int orc_newton_mode(const orc_data *D, const double *mu0, const double *Q0,
                    double *theta, int max_iter, int *iters_out)
{
    const int d = D->d;
    double *B = malloc(sizeof(double) * d), *C = malloc(sizeof(double) * d * d);
    double *H = malloc(sizeof(double) * d * d), *L = malloc(sizeof(double) * d * d);
    double *g = malloc(sizeof(double) * d), *s = malloc(sizeof(double) * d);
    double *y = malloc(sizeof(double) * d), *tn = malloc(sizeof(double) * d);
    int status = ORC_OK, it;
    for (int r = 0; r < d; ++r) theta[r] = mu0[r];
    double A;
    orc_cv_build(D, theta, &A, B, C);
    double obj = A + log_prior_quad(d, mu0, Q0, theta);
    for (it = 0; it < max_iter; ++it) {
        /* gradient and negative Hessian of the log posterior */
        for (int r = 0; r < d; ++r) {
            double q = 0;
            for (int c = 0; c < d; ++c) q += Q0[(size_t)r * d + c] * (theta[c] - mu0[c]);
            g[r] = B[r] - q;
            for (int c = 0; c < d; ++c) H[(size_t)r * d + c] = -C[(size_t)r * d + c] + Q0[(size_t)r * d + c];
        }
        if (orc_cholesky(d, H, L) != ORC_OK) {
            /* the log posterior is not concave here (e.g. Student-t far from
             * the mode): shift the diagonal, 1e-6 (1 + max |H_rr|) 10^k,
             * until the system is positive definite (a damped step) */
            double hmax = 0;
            for (int r = 0; r < d; ++r) if (fabs(H[(size_t)r * d + r]) > hmax) hmax = fabs(H[(size_t)r * d + r]);
            int k;
            for (k = 0; k < 24; ++k) {
                double lam = 1e-6 * (1 + hmax) * pow(10.0, k);
                for (int r = 0; r < d; ++r) H[(size_t)r * d + r] += lam;
                if (orc_cholesky(d, H, L) == ORC_OK) break;
                for (int r = 0; r < d; ++r) H[(size_t)r * d + r] -= lam;
            }
            if (k == 24) { status = ORC_ERR_NOT_PD; break; }
        }
        solve_lower(d, L, g, y);
        solve_upper_from_lower(d, L, y, s);
        double t = 1.0, newobj = 0;
        int ok = 0;
        for (int h = 0; h < 60; ++h) {
            for (int r = 0; r < d; ++r) tn[r] = theta[r] + t * s[r];
            double An;
            orc_cv_build(D, tn, &An, B, C);
            newobj = An + log_prior_quad(d, mu0, Q0, tn);
            if (newobj >= obj || isnan(obj)) { ok = 1; break; }
            t *= 0.5;
        }
        double stepmax = 0;
        for (int r = 0; r < d; ++r) {
            double st = fabs(tn[r] - theta[r]);
            if (st > stepmax) stepmax = st;
        }
        if (!ok) { /* no ascent possible: at the mode to working precision */
            orc_cv_build(D, theta, &A, B, C);
            ++it;
            break;
        }
        for (int r = 0; r < d; ++r) theta[r] = tn[r];
        obj = newobj;
        if (stepmax < 1e-12) { ++it; break; }
    }
    if (iters_out) *iters_out = it;
    free(B); free(C); free(H); free(L); free(g); free(s); free(y); free(tn);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Difference estimator (eq. difference_estimator_logl), its variance        */
/* estimate (section 3.2) and their gradients, for one particle.             */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lhat, sig2, dhat;
} orc_est;

static void estimate_one(const orc_data *D, const orc_cv *cv, int32_t m, const double *theta,
                         const int32_t *u, orc_est *out, double *grad_l, double *grad_s)
{
    const int d = D->d;
    qd *delta = malloc(sizeof(qd) * d);
    qd *dj = malloc(sizeof(qd) * (size_t)m);
    qd *dpj = malloc(sizeof(qd) * (size_t)m);
    for (int c = 0; c < d; ++c) delta[c] = (qd)theta[c] - (qd)cv->theta_bar[c];

    qd dsum = 0;
    for (int32_t j = 0; j < m; ++j) {
        const double *row = D->Xy + (int64_t)u[j] * D->ld;
        qd eb = 0, De = 0;
        for (int c = 0; c < d; ++c) {
            eb += (qd)row[c] * (qd)cv->theta_bar[c];
            De += (qd)row[c] * delta[c];
        }
        q_remainder(D, (qd)row[d], eb, De, &dj[j], &dpj[j]);
        dsum += dj[j];
    }
    qd nq = (qd)D->n, mq = (qd)m;
    qd dbar = dsum / mq;

    /* sum_k q_k(theta) = A + B'delta + 1/2 delta' C delta; the first-order
     * control variate has no curvature term */
    qd qsum = (qd)cv->A;
    for (int r = 0; r < d; ++r) {
        qsum += (qd)cv->B[r] * delta[r];
        if (D->cv_order == 2)
            for (int c = 0; c < d; ++c) qsum += 0.5Q * delta[r] * (qd)cv->C[(size_t)r * d + c] * delta[c];
    }
    qd dhat = nq / mq * dsum;
    qd ss = 0;
    for (int32_t j = 0; j < m; ++j) ss += (dj[j] - dbar) * (dj[j] - dbar);
    qd sig2 = nq * nq / (mq * mq) * ss;

    out->lhat = (double)(qsum + dhat);
    out->dhat = (double)dhat;
    out->sig2 = (double)sig2;

    if (grad_l || grad_s) {
        for (int r = 0; r < d; ++r) {
            qd s1 = 0, s2v = 0;
            for (int32_t j = 0; j < m; ++j) {
                qd xr = (qd)(D->Xy[(int64_t)u[j] * D->ld + r]);
                s1 += dpj[j] * xr;
                s2v += (dj[j] - dbar) * dpj[j] * xr;
            }
            if (grad_l) {
                qd gl = (qd)cv->B[r];
                if (D->cv_order == 2)
                    for (int c = 0; c < d; ++c) gl += (qd)cv->C[(size_t)r * d + c] * delta[c];
                gl += nq / mq * s1;
                grad_l[r] = (double)gl;
            }
            if (grad_s) grad_s[r] = (double)(2 * nq * nq / (mq * mq) * s2v);
        }
    }
    free(delta);
    free(dj);
    free(dpj);
}

/* Estimator for `count` particles; any output pointer may be NULL. */
void orc_estimate(const orc_data *D, const orc_cv *cv, int32_t count, int32_t m,
                  const double *theta, const int32_t *u, double *lhat, double *sig2,
                  double *dhat, double *grad_l, double *grad_s)
{
    const int d = D->d;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < count; ++i) {
        orc_est e;
        estimate_one(D, cv, m, theta + (size_t)i * d, u + (size_t)i * m, &e,
                     grad_l ? grad_l + (size_t)i * d : NULL, grad_s ? grad_s + (size_t)i * d : NULL);
        if (lhat) lhat[i] = e.lhat;
        if (sig2) sig2[i] = e.sig2;
        if (dhat) dhat[i] = e.dhat;
    }
}

/* ------------------------------------------------------------------------ */
/* Reweighting, adaptive tempering by ESS bisection and the marginal         */
/* likelihood increment (sections 2.2, 3.3, 3.5; Algorithm 2 steps b-c).     */
/* ------------------------------------------------------------------------ */

/* incremental log weight (a - a_prev) l_hat - 1/2 (a^2 - a_prev^2) sigma2_hat */
static double incr(double a, double a_prev, double lh, double s2)
{
    double v = (a - a_prev) * (lh - 0.5 * (a + a_prev) * s2);
    return isfinite(v) ? v : -INFINITY;
}

static double ess_at(int32_t M, const double *logw, const double *lhat, const double *sig2,
                     double a, double a_prev)
{
    double mx = -INFINITY;
    for (int32_t i = 0; i < M; ++i) {
        double lw = logw[i] + incr(a, a_prev, lhat[i], sig2[i]);
        if (lw > mx) mx = lw;
    }
    if (!isfinite(mx)) return 0;
    xd s1 = 0, s2 = 0;
    for (int32_t i = 0; i < M; ++i) {
        double lw = logw[i] + incr(a, a_prev, lhat[i], sig2[i]);
        xd w = expl((xd)(lw - mx));
        s1 += w;
        s2 += w * w;
    }
    return (double)(s1 * s1 / s2);
}

static double logsumexp(int32_t M, const double *v)
{
    double mx = -INFINITY;
    for (int32_t i = 0; i < M; ++i) if (v[i] > mx) mx = v[i];
    if (!isfinite(mx)) return mx;
    xd s = 0;
    for (int32_t i = 0; i < M; ++i) s += expl((xd)(v[i] - mx));
    return mx + (double)logl(s);
}

/* Reweighting at the chosen exponent a (section 3.3) and the log-evidence
 * increment log sum_i W_i exp(nu_i) (section 3.5). */
static int reweight(int32_t M, const double *lhat, const double *sig2, double *logw, double a_prev,
                    double a, double *a_out, double *dlogz_out, double *ess_out)
{
    double *lw = calloc((size_t)M + 1, sizeof(double));
    for (int32_t i = 0; i < M; ++i) lw[i] = logw[i] + incr(a, a_prev, lhat[i], sig2[i]);
    double lse_new = logsumexp(M, lw);
    double lse_old = logsumexp(M, logw);
    if (!isfinite(lse_new)) { free(lw); return ORC_ERR_NONFINITE; }
    *ess_out = ess_at(M, logw, lhat, sig2, a, a_prev);
    *dlogz_out = lse_new - lse_old;
    for (int32_t i = 0; i < M; ++i) logw[i] = lw[i] - lse_new;
    *a_out = a;
    free(lw);
    return ORC_OK;
}

/*
 * Chooses a in (a_prev, 1] with ESS(a) = ess_frac*M by bisection (60 halvings
 * of [a_prev, 1], keeping the side whose ESS is at least the target; a = 1 when
 * ESS(1) already meets it), reweights logw in place (normalised) and returns
 * the log increment of the normalising constant.
 */
int orc_temper(int32_t M, const double *lhat, const double *sig2, double *logw, double a_prev,
               double ess_frac, int32_t n_bisect, double *a_out, double *dlogz_out, double *ess_out)
{
    double target = ess_frac * (double)M;
    double a;
    if (ess_at(M, logw, lhat, sig2, 1.0, a_prev) >= target) {
        a = 1.0;
    } else {
        double lo = a_prev, hi = 1.0;
        for (int it = 0; it < n_bisect; ++it) {
            double mid = 0.5 * (lo + hi);
            if (ess_at(M, logw, lhat, sig2, mid, a_prev) >= target) lo = mid;
            else hi = mid;
        }
        a = (lo > a_prev) ? lo : hi;
    }
    return reweight(M, lhat, sig2, logw, a_prev, a, a_out, dlogz_out, ess_out);
}

/* The paper's own rule (section 2.2): evaluate the ESS on a grid of
 * candidate exponents and take the one whose ESS is closest to the target
 * (the paper uses 0.8 M). The paper does not give the grid; here it is
 * geometric in the step, a_j = a_prev + (1 - a_prev) 2^(-j/4) for
 * j = 0..S-1 (a_0 = 1), written with the correctly rounded constants
 * 2^(-1/4), 2^(-1/2), 2^(-3/4). Ties go to the smaller j (the larger a).
 * Only points above a_prev are candidates (near a = 1 the smallest steps
 * round away), so every stage moves. */
double orc_grid_point(double a_prev, int32_t j)
{
    static const double frac[4] = {1.0, 0x1.ae89f995ad3adp-1, 0x1.6a09e667f3bcdp-1, 0x1.306fe0a31b715p-1};
    if (j == 0) return 1.0;
    return a_prev + (1.0 - a_prev) * ldexp(frac[j & 3], -(j >> 2));
}

int orc_temper_grid(int32_t M, const double *lhat, const double *sig2, double *logw, double a_prev,
                    double ess_frac, int32_t S, double *ess_grid, double *a_out, double *dlogz_out,
                    double *ess_out)
{
    if (S < 1) return ORC_ERR_ARG;
    double target = ess_frac * (double)M;
    int32_t best = 0;
    double bestd = INFINITY;
    for (int32_t j = 0; j < S; ++j) {
        double aj = orc_grid_point(a_prev, j);
        double e = ess_at(M, logw, lhat, sig2, aj, a_prev);
        if (ess_grid) ess_grid[j] = e;
        double dist = fabs(e - target);
        if (aj > a_prev && dist < bestd) { bestd = dist; best = j; }
    }
    return reweight(M, lhat, sig2, logw, a_prev, orc_grid_point(a_prev, best), a_out, dlogz_out, ess_out);
}

/* ------------------------------------------------------------------------ */
/* Mass matrix: weighted covariance of the particles and its Cholesky factor */
/* (Algorithm 2 step d; the HMC mass matrix is the inverse covariance).      */
/* ------------------------------------------------------------------------ */

int orc_moments(int32_t M, int32_t d, const double *theta, const double *logw,
                double *mean, double *Sigma, double *Lchol)
{
    double lse = logsumexp(M, logw);
    xd *mu = calloc((size_t)d, sizeof(xd));
    for (int32_t i = 0; i < M; ++i) {
        xd w = expl((xd)(logw[i] - lse));
        for (int r = 0; r < d; ++r) mu[r] += w * theta[(size_t)i * d + r];
    }
    for (int r = 0; r < d; ++r) mean[r] = (double)mu[r];
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            xd s = 0;
            for (int32_t i = 0; i < M; ++i) {
                xd w = expl((xd)(logw[i] - lse));
                s += w * ((xd)theta[(size_t)i * d + r] - mu[r]) * ((xd)theta[(size_t)i * d + c] - mu[c]);
            }
            Sigma[(size_t)r * d + c] = (double)s;
        }
    free(mu);
    /* jitter ladder when the covariance is numerically singular */
    double tr = 0;
    for (int r = 0; r < d; ++r) tr += Sigma[(size_t)r * d + r];
    double *S2 = malloc(sizeof(double) * d * d);
    int st = ORC_ERR_NOT_PD;
    for (int t = 0; t <= 10; ++t) {
        memcpy(S2, Sigma, sizeof(double) * d * d);
        if (t > 0) {
            double jit = 1e-10 * (tr / d) * pow(10.0, t - 1);
            for (int r = 0; r < d; ++r) S2[(size_t)r * d + r] += jit;
        }
        if (orc_cholesky(d, S2, Lchol) == ORC_OK) {
            memcpy(Sigma, S2, sizeof(double) * d * d);
            st = ORC_OK;
            break;
        }
    }
    free(S2);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Systematic resampling in exact integer arithmetic                         */
/* ------------------------------------------------------------------------ */

/*
 * c_i = floor(exp(logw_i - max) * 2^48), S = sum c_i, one offset U32 (top 32
 * bits of one generator word), points t_k = floor((k 2^32 + U32) S / (M 2^32)),
 * ancestor A_k = smallest j whose inclusive prefix sum exceeds t_k.
 */
void orc_resample_ancestors(int32_t M, const double *logw, uint32_t U32, int32_t *anc)
{
    double mx = -INFINITY;
    for (int32_t i = 0; i < M; ++i) if (logw[i] > mx) mx = logw[i];
    uint64_t *cum = malloc(sizeof(uint64_t) * (size_t)M);
    uint64_t S = 0;
    for (int32_t i = 0; i < M; ++i) {
        double w = exp(logw[i] - mx);
        uint64_t c = (uint64_t)floor(ldexp(w, 48));
        S += c;
        cum[i] = S;
    }
    int32_t j = 0;
    for (int32_t k = 0; k < M; ++k) {
        unsigned __int128 num = ((unsigned __int128)(((uint64_t)k << 32) + U32)) * S;
        uint64_t t = (uint64_t)(num / ((unsigned __int128)(uint64_t)M << 32));
        while (cum[j] <= t) ++j;
        anc[k] = j;
    }
    free(cum);
}

uint32_t orc_resample_offset(uint64_t seed, uint32_t stage, uint32_t dataset)
{
    return (uint32_t)(orc_rng_word(seed, 2, stage, 0, dataset, 0, 0) >> 32);
}

/* Multinomial resampling (section 2.1, the paper's choice): every slot k
 * draws its ancestor independently with probability W_i. In integers, with
 * c_i and S as in the systematic scheme above and a uniform 64-bit word r_k,
 * t_k = floor(r_k S / 2^64) and the ancestor is the smallest j whose
 * inclusive prefix sum exceeds t_k (so i is drawn with probability c_i / S). */
void orc_resample_multinomial_words(int32_t M, const double *logw, const uint64_t *words, int32_t *anc)
{
    double mx = -INFINITY;
    for (int32_t i = 0; i < M; ++i) if (logw[i] > mx) mx = logw[i];
    uint64_t *cum = malloc(sizeof(uint64_t) * (size_t)M);
    uint64_t S = 0;
    for (int32_t i = 0; i < M; ++i) {
        double w = exp(logw[i] - mx);
        S += (uint64_t)floor(ldexp(w, 48));
        cum[i] = S;
    }
    for (int32_t k = 0; k < M; ++k) {
        uint64_t t = (uint64_t)(((unsigned __int128)words[k] * S) >> 64);
        int32_t j = 0;
        while (cum[j] <= t) ++j;
        anc[k] = j;
    }
    free(cum);
}

/* The words: purpose 2 (resampling), the stage, particle slot k, draw 1. */
void orc_resample_multinomial(int32_t M, const double *logw, uint64_t seed, uint32_t stage,
                              uint32_t dataset, int32_t *anc)
{
    uint64_t *words = malloc(sizeof(uint64_t) * (size_t)M);
    for (int32_t k = 0; k < M; ++k) words[k] = orc_rng_word(seed, 2, stage, 0, dataset, (uint64_t)k, 1);
    orc_resample_multinomial_words(M, logw, words, anc);
    free(words);
}

/* ------------------------------------------------------------------------ */
/* Initial particles (Algorithm 2 step 1)                                    */
/* ------------------------------------------------------------------------ */

int orc_init_particles(int32_t M, int32_t d, int32_t m, int64_t n, uint64_t seed, uint32_t dataset,
                       const double *mu0, const double *Q0, double *theta, int32_t *u, double *logw)
{
    double *L0 = malloc(sizeof(double) * d * d);
    if (orc_cholesky(d, Q0, L0) != ORC_OK) { free(L0); return ORC_ERR_NOT_PD; }
    for (int32_t i = 0; i < M; ++i) {
        double z[512], x[512];
        if (d > 512) { free(L0); return ORC_ERR_ARG; }
        for (int k = 0; k < d; ++k) z[k] = rng_normal(seed, 0, 0, 0, dataset, (uint64_t)i, (uint64_t)k);
        /* theta ~ N(mu0, Q0^{-1}): theta = mu0 + L0^{-T} z with Q0 = L0 L0' */
        solve_upper_from_lower(d, L0, z, x);
        for (int k = 0; k < d; ++k) theta[(size_t)i * d + k] = mu0[k] + x[k];
        for (int32_t j = 0; j < m; ++j)
            u[(size_t)i * m + j] = (int32_t)rng_index(orc_rng_word(seed, 1, 0, 0, dataset, (uint64_t)i, (uint64_t)j), n);
        logw[i] = -log((double)M);
    }
    free(L0);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Markov move (Algorithm 1): block pseudo-marginal refresh of u, then HMC   */
/* on theta given u, both targeting the extended target of section 3.1.      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t M, m, G;
    uint64_t seed;
    uint32_t stage;
    uint32_t dataset;    /* dataset field of the random-number counter */
    const double *mu0;   /* prior mean, d */
    const double *Q0;    /* prior precision, d*d */
    const double *Sigma; /* particle covariance (inverse mass matrix), d*d */
    const double *Lchol; /* Cholesky factor of Sigma */
} orc_move_cfg;

static double lambda_of(double a, const orc_est *e)
{
    return a * e->lhat - 0.5 * a * a * e->sig2;
}

/* log target up to a constant: lambda_a + log prior; its gradient into g (if non-NULL) */
static double log_target(const orc_data *D, const orc_cv *cv, const orc_move_cfg *K, double a,
                         const double *th, const int32_t *u, double *g, orc_est *e_out)
{
    const int d = D->d;
    double gl[512], gs[512];
    orc_est e;
    estimate_one(D, cv, K->m, th, u, &e, g ? gl : NULL, g ? gs : NULL);
    double lp = 0;
    for (int r = 0; r < d; ++r) {
        double q = 0;
        for (int c = 0; c < d; ++c) q += K->Q0[(size_t)r * d + c] * (th[c] - K->mu0[c]);
        lp += -0.5 * (th[r] - K->mu0[r]) * q;
        if (g) g[r] = a * gl[r] - 0.5 * a * a * gs[r] - q;
    }
    if (e_out) *e_out = e;
    return lambda_of(a, &e) + lp;
}

static double kinetic(int d, const double *Sigma, const double *p)
{
    double s = 0;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) s += p[r] * Sigma[(size_t)r * d + c] * p[c];
    return 0.5 * s;
}

static void move_one(const orc_data *D, const orc_cv *cv, const orc_move_cfg *K, double a,
                     double eps, int32_t L, uint32_t mv, int32_t i, double *theta, int32_t *u,
                     int32_t *acc_u, int32_t *acc_th, double *lhat_out, double *sig2_out, double *diag)
{
    const int d = D->d;
    const int32_t m = K->m, G = K->G;
    const uint64_t seed = K->seed;
    const uint32_t st = K->stage, ds = K->dataset;

    /* 1. u | theta: replace one block, chosen uniformly, by fresh uniform indices */
    int32_t g = (int32_t)rng_index(orc_rng_word(seed, 3, st, mv, ds, (uint64_t)i, 0), G);
    int64_t b0 = (int64_t)g * m / G, b1 = (int64_t)(g + 1) * m / G;
    int32_t *ustar = malloc(sizeof(int32_t) * (size_t)m);
    memcpy(ustar, u, sizeof(int32_t) * (size_t)m);
    for (int64_t j = b0; j < b1; ++j)
        ustar[j] = (int32_t)rng_index(orc_rng_word(seed, 4, st, mv, ds, (uint64_t)i, (uint64_t)(j - b0)), D->n);
    orc_est e_cur, e_new;
    estimate_one(D, cv, m, theta, u, &e_cur, NULL, NULL);
    estimate_one(D, cv, m, theta, ustar, &e_new, NULL, NULL);
    double logr_u = lambda_of(a, &e_new) - lambda_of(a, &e_cur);
    double logU = log(rng_uniform_open0(orc_rng_word(seed, 5, st, mv, ds, (uint64_t)i, 0)));
    *acc_u = (isfinite(logr_u) && logU < logr_u) ? 1 : 0;
    if (diag) { diag[0] = logr_u; diag[1] = logU; }
    if (*acc_u) memcpy(u, ustar, sizeof(int32_t) * (size_t)m);
    free(ustar);

    /* 2. theta | u: HMC with inverse mass matrix Sigma */
    double p[512], z[512] = {0}, g0[512], th1[512], v[512];
    for (int k = 0; k < d; ++k) z[k] = rng_normal(seed, 6, st, mv, ds, (uint64_t)i, (uint64_t)k);
    solve_upper_from_lower(d, K->Lchol, z, p); /* p ~ N(0, Sigma^{-1}) */
    orc_est e0, e1;
    double lt0 = log_target(D, cv, K, a, theta, u, g0, &e0);
    double H0 = -lt0 + kinetic(d, K->Sigma, p);
    for (int k = 0; k < d; ++k) { th1[k] = theta[k]; p[k] += 0.5 * eps * g0[k]; }
    double lt1 = lt0;
    e1 = e0;
    for (int32_t l = 1; l <= L; ++l) {
        for (int r = 0; r < d; ++r) {
            double s = 0;
            for (int c = 0; c < d; ++c) s += K->Sigma[(size_t)r * d + c] * p[c];
            v[r] = s;
        }
        for (int r = 0; r < d; ++r) th1[r] += eps * v[r];
        lt1 = log_target(D, cv, K, a, th1, u, g0, &e1);
        double h = (l < L) ? eps : 0.5 * eps;
        for (int r = 0; r < d; ++r) p[r] += h * g0[r];
    }
    double H1 = -lt1 + kinetic(d, K->Sigma, p);
    double logr = H0 - H1;
    double logU2 = log(rng_uniform_open0(orc_rng_word(seed, 7, st, mv, ds, (uint64_t)i, 0)));
    *acc_th = (isfinite(logr) && logU2 < logr) ? 1 : 0;
    if (diag) { diag[2] = logr; diag[3] = logU2; }
    if (*acc_th) {
        for (int r = 0; r < d; ++r) theta[r] = th1[r];
        *lhat_out = e1.lhat;
        *sig2_out = e1.sig2;
    } else {
        *lhat_out = e0.lhat;
        *sig2_out = e0.sig2;
    }
}

/*
 * One Markov move (index `mv` within the stage) for every particle, in place.
 * acc: M*2 flags (u accepted, theta accepted). lhat/sig2 receive the estimator
 * at the particle's final state.
 */
int orc_move(const orc_data *D, const orc_cv *cv, const orc_move_cfg *K, double a, double eps,
             int32_t L, uint32_t mv, double *theta, int32_t *u, int32_t *acc,
             double *lhat, double *sig2)
{
    if (D->d > 512) return ORC_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < K->M; ++i) {
        move_one(D, cv, K, a, eps, L, mv, i, theta + (size_t)i * D->d, u + (size_t)i * K->m,
                 &acc[2 * i], &acc[2 * i + 1], &lhat[i], &sig2[i], NULL);
    }
    return ORC_OK;
}

/*
 * Move a subset of particles [i0, i0+count) (bounded CPU timing, tests).
 * diag (count*4, nullable): log r and log U of the u-refresh and of the HMC step.
 */
int orc_move_range(const orc_data *D, const orc_cv *cv, const orc_move_cfg *K, double a,
                   double eps, int32_t L, uint32_t mv, int32_t i0, int32_t count, double *theta,
                   int32_t *u, int32_t *acc, double *lhat, double *sig2, double *diag)
{
    if (D->d > 512) return ORC_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < count; ++t) {
        int32_t i = i0 + t;
        move_one(D, cv, K, a, eps, L, mv, i, theta + (size_t)t * D->d, u + (size_t)t * K->m,
                 &acc[2 * t], &acc[2 * t + 1], &lhat[t], &sig2[t], diag ? diag + 4 * (size_t)t : NULL);
    }
    return ORC_OK;
}

/* Threads the parallel loops over particles use from now on (timing only). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
