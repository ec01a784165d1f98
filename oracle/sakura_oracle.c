/*
 * Sakura CPU oracle -- TEST INFRASTRUCTURE ONLY (see sakura_oracle.h).
 *
 * Plain, slow fp64 reference of the Keplerian-splitting integrator of
 * Goncalves Ferrari, Boekholt & Portegies Zwart (2014).  It follows the
 * paper's own order of operations: the half drifts of eqs. (27a, 27d), the
 * pair map of eq. (26) applied independently to every ordered pair as in
 * Listing 1, and the mass-weighted sums of eqs. (23, 27b, 27c).  The pair flow
 * of eq. (18) is a universal-variable Kepler solver driven by the Laguerre
 * iteration that the paper credits to Conway (1986), written here from the
 * textbook formulation (universal anomaly chi, Stumpff functions c2, c3),
 * safeguarded by bisection.
 *
 * Nothing here is blocked, fused or reordered for speed.  The only
 * concurrency is an OpenMP loop over the rows i of the pair sum; every row is
 * computed exactly as the serial loop would compute it.
 */
#include "sakura_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double EPS = 2.220446049250313e-16; /* 2^-52 */

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ------------------------------------------------------------------------ */
/* Stumpff functions.                                                        */
/*   c2(z) = (1 - cos sqrt z) / z,   c3(z) = (sqrt z - sin sqrt z) / z^{3/2} */
/* for z > 0, continued analytically by cosh / sinh for z < 0.  Both equal   */
/* the entire series c_k(z) = sum_m (-z)^m / (2m + k)!, which is used near   */
/* z = 0 where the closed forms lose digits to cancellation.                 */
/* ------------------------------------------------------------------------ */
static const double SERIES_LIMIT = 4.0;

static double stumpff_series(double z, int k)
{
    double term = 1.0;
    for (int i = 2; i <= k; ++i) term /= (double)i; /* 1/k! */
    double sum = term;
    for (int m = 1; m < 80; ++m) {
        term *= -z / ((2.0 * m + k - 1.0) * (2.0 * m + k));
        double next = sum + term;
        if (next == sum) break;
        sum = next;
    }
    return sum;
}

double sref_stumpff_c2(double z)
{
    if (fabs(z) < SERIES_LIMIT) return stumpff_series(z, 2);
    if (z > 0.0) {
        double s = sqrt(z);
        return (1.0 - cos(s)) / z;
    }
    double s = sqrt(-z);
    return (cosh(s) - 1.0) / (-z);
}

double sref_stumpff_c3(double z)
{
    if (fabs(z) < SERIES_LIMIT) return stumpff_series(z, 3);
    if (z > 0.0) {
        double s = sqrt(z);
        return (s - sin(s)) / (z * s);
    }
    double s = sqrt(-z);
    return (sinh(s) - s) / ((-z) * s);
}

/* ------------------------------------------------------------------------ */
/* Universal Kepler equation (eq. 18 solver).                               */
/* With r0 = |x0|, sig0 = x0.w0 / sqrt(mu), alpha = 2/r0 - w0.w0/mu,         */
/* q = 1 - alpha r0, z = alpha chi^2, C = c2(z), S = c3(z):                   */
/*   F(chi)   = sig0 chi^2 C + q chi^3 S + r0 chi - sqrt(mu) t               */
/*   F'(chi)  = sig0 chi (1 - z S) + q chi^2 C + r0     (the radius, > 0)    */
/*   F''(chi) = sig0 (1 - z C) + q chi (1 - z S)                             */
/* F is strictly increasing, so the root is unique.                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    double r0, sig0, alpha, q, T;
} kepeq_t;

static void kepeq_eval(const kepeq_t *k, double chi, double *F, double *dF,
                       double *d2F, double *Fnoise)
{
    double z = k->alpha * chi * chi;
    double C = sref_stumpff_c2(z), S = sref_stumpff_c3(z);
    double U1 = chi * (1.0 - z * S), U2 = chi * chi * C, U3 = chi * chi * chi * S;
    double U0 = 1.0 - z * C;
    *F = k->sig0 * U2 + k->q * U3 + k->r0 * chi - k->T;
    *dF = k->sig0 * U1 + k->q * U2 + k->r0;
    *d2F = k->sig0 * U0 + k->q * U1;
    /* size of the rounding error of F: eps times the sum of its terms */
    *Fnoise = EPS * (fabs(k->sig0 * U2) + fabs(k->q * U3) + fabs(k->r0 * chi) + fabs(k->T));
}

/* Root of F by the Laguerre iteration (order 5, as Conway uses for Kepler's
 * equation) inside a bracket that bisection falls back to whenever a Laguerre
 * step would leave it.  Converged when the step or the bracket is below
 * 4 eps |chi|, or when F is zero to within the rounding of its own terms (for
 * ill-conditioned orbits the iterates can otherwise bounce between points a
 * few ulps apart).  Returns 0 on convergence. */
static int kepeq_solve(const kepeq_t *k, double *chi_out, int *iters)
{
    const double nL = 5.0;
    if (k->T == 0.0) {
        *chi_out = 0.0;
        if (iters) *iters = 0;
        return 0;
    }
    /* Starter: invert the cubic Taylor series T = r0 chi + sig0 chi^2/2 + q chi^3/6. */
    double u = k->T / k->r0;
    double chi = u - k->sig0 * u * u / (2.0 * k->r0) +
                 (3.0 * k->sig0 * k->sig0 - k->q * k->r0) * u * u * u /
                     (6.0 * k->r0 * k->r0);
    /* Beyond the reach of the series (its corrections dominate) start from the
     * free-drift value u; the bracket search below doubles from there. */
    if (!isfinite(chi) || (chi > 0.0) != (k->T > 0.0) || fabs(chi - u) > 0.5 * fabs(u))
        chi = u;

    /* Bracket.  F(0) = -T, so the root has the sign of T. */
    double lo, hi, F, dF, d2F, Fn;
    int grow = 0;
    if (k->T > 0.0) {
        lo = 0.0;
        hi = chi;
        for (;;) {
            kepeq_eval(k, hi, &F, &dF, &d2F, &Fn);
            if (!(F < 0.0)) break; /* F >= 0, or overflow far beyond the root */
            lo = hi;
            hi *= 2.0;
            if (++grow > 2100) return SREF_ENOCONV;
        }
    } else {
        hi = 0.0;
        lo = chi;
        for (;;) {
            kepeq_eval(k, lo, &F, &dF, &d2F, &Fn);
            if (!(F > 0.0)) break;
            hi = lo;
            lo *= 2.0;
            if (++grow > 2100) return SREF_ENOCONV;
        }
    }
    if (!(chi >= lo && chi <= hi)) chi = 0.5 * (lo + hi);

    for (int it = 1; it <= 400; ++it) {
        kepeq_eval(k, chi, &F, &dF, &d2F, &Fn);
        if (!isfinite(F) || !isfinite(dF)) {
            /* The Stumpff functions overflow only far beyond the root: shrink
             * the bracket from that side and bisect. */
            if (k->T > 0.0) hi = chi;
            else lo = chi;
            chi = 0.5 * (lo + hi);
            continue;
        }
        if (fabs(F) <= 2.0 * Fn) {
            *chi_out = chi;
            if (iters) *iters = it;
            return 0;
        }
        if (F < 0.0) lo = chi;
        else hi = chi;
        double disc = (nL - 1.0) * (nL - 1.0) * dF * dF - nL * (nL - 1.0) * F * d2F;
        double den = dF + sqrt(fabs(disc)); /* dF = r > 0 */
        double next = chi - nL * F / den;
        if (!(next >= lo && next <= hi)) next = 0.5 * (lo + hi);
        double step = fabs(next - chi);
        chi = next;
        if (step <= 4.0 * EPS * fabs(chi) || hi - lo <= 4.0 * EPS * fabs(chi)) {
            *chi_out = chi;
            if (iters) *iters = it;
            return 0;
        }
    }
    return SREF_ENOCONV;
}

int sref_kepler(double tau, double mu, const double x0[3], const double w0[3],
                double x1[3], double w1[3], double coef[4], int *iters)
{
    double r0 = sqrt(dot3(x0, x0));
    if (!(r0 > 0.0)) return SREF_ECOLLIDE;
    double fm1 = 0.0, gmt = 0.0, fdot = 0.0, gdm1 = 0.0;
    int it = 0;
    if (mu != 0.0) {
        double sqmu = sqrt(mu);
        kepeq_t k;
        k.r0 = r0;
        k.sig0 = dot3(x0, w0) / sqmu;
        k.alpha = 2.0 / r0 - dot3(w0, w0) / mu;
        k.q = 1.0 - k.alpha * r0;
        /* A bound orbit repeats after P = 2 pi / (sqrt(mu) alpha^{3/2});
         * propagate over the remainder when tau spans more than half of it. */
        double t = tau;
        if (k.alpha > 0.0) {
            double P = 2.0 * M_PI / (sqmu * k.alpha * sqrt(k.alpha));
            if (fabs(t) > 0.5 * P) t -= P * nearbyint(t / P);
        }
        k.T = sqmu * t;
        double chi;
        int rc = kepeq_solve(&k, &chi, &it);
        if (rc) return rc;
        double z = k.alpha * chi * chi;
        double C = sref_stumpff_c2(z), S = sref_stumpff_c3(z);
        double U1 = chi * (1.0 - z * S), U2 = chi * chi * C, U3 = chi * chi * chi * S;
        double r = k.sig0 * U1 + k.q * U2 + r0;
        /* Lagrange coefficients f, g, fdot, gdot, kept as differences from the
         * free drift (f = 1, g = tau, fdot = 0, gdot = 1). */
        fm1 = -U2 / r0;
        gmt = (t - tau) - U3 / sqmu;
        fdot = -sqmu * U1 / (r * r0);
        gdm1 = -U2 / r;
    }
    for (int c = 0; c < 3; ++c) {
        x1[c] = x0[c] + fm1 * x0[c] + (tau + gmt) * w0[c];
        w1[c] = w0[c] + fdot * x0[c] + gdm1 * w0[c];
    }
    if (coef) {
        coef[0] = fm1;
        coef[1] = gmt;
        coef[2] = fdot;
        coef[3] = gdm1;
    }
    if (iters) *iters = it;
    return SREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Pair map of eq. (26): back-drift tau/2 (eq. 17), Kepler flow tau (eq. 18), */
/* back-drift tau/2; the increments are the result minus the input.          */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Learned Kepler starter: inputs, domain and target (an extension of the    */
/* method; the paper's solver only needs some starting value).               */
/* In units with r0 = 1 and mu = 1 the Kepler problem over time t depends on  */
/* three numbers only: tau' = |t| sqrt(mu / r0^3), e' = sgn(t) (x0.w0) /      */
/* sqrt(mu r0) (radial speed over circular speed, sign-flipped for t < 0 by  */
/* time reversal) and b' = alpha r0 = 2 - r0 |w0|^2 / mu.  The eight inputs   */
/* are functions of these; the target is y = log(chi r0 / (sqrt(mu) t)), the  */
/* log of the root over its free-drift value, which is even under time       */
/* reversal.  Bound orbits use the same period reduction of t as             */
/* sref_kepler.                                                             */
/* ------------------------------------------------------------------------ */
int sref_guess_sample(double tau, double mu, const double x0[3], const double w0[3],
                      const double domain[4], double feat[8], double *y, int *in_domain)
{
    if (!x0 || !w0 || !domain || !feat || !y || !in_domain) return SREF_EINVAL;
    *in_domain = 0;
    *y = 0.0;
    for (int k = 0; k < 8; ++k) feat[k] = 0.0;
    const double r0 = sqrt(dot3(x0, x0));
    if (!(r0 > 0.0)) return SREF_ECOLLIDE;
    if (!(mu > 0.0)) return SREF_OK; /* no Kepler problem: never in the domain */
    const double sqmu = sqrt(mu);
    const double alpha = 2.0 / r0 - dot3(w0, w0) / mu;
    double t = tau;
    if (alpha > 0.0) {
        double P = 2.0 * M_PI / (sqmu * alpha * sqrt(alpha));
        if (fabs(t) > 0.5 * P) t -= P * nearbyint(t / P);
    }
    const double sgn = (t > 0.0) ? 1.0 : ((t < 0.0) ? -1.0 : 0.0);
    const double taup = fabs(t) * sqrt(mu / (r0 * r0 * r0));
    const double ep = sgn * dot3(x0, w0) / sqrt(mu * r0);
    const double bp = alpha * r0;
    const double bpos = bp > 0.0 ? bp : 0.0;
    feat[0] = (taup > 0.0) ? log2(taup) : -1074.0;
    feat[1] = ep;
    feat[2] = bp;
    feat[3] = taup;
    feat[4] = ep * taup;
    feat[5] = taup * taup * (3.0 * ep * ep - 1.0 + bp) / 6.0;
    feat[6] = taup * bpos * sqrt(bpos);
    feat[7] = ep * sqrt(bpos);
    const int dom = taup >= domain[0] && taup <= domain[1] && bp >= domain[2] &&
                    fabs(ep) <= domain[3];
    if (!dom) return SREF_OK;
    kepeq_t k;
    k.r0 = r0;
    k.sig0 = dot3(x0, w0) / sqmu;
    k.alpha = alpha;
    k.q = 1.0 - alpha * r0;
    k.T = sqmu * t;
    double chi;
    int rc = kepeq_solve(&k, &chi, NULL);
    if (rc) return rc;
    *y = log(chi * r0 / (sqmu * t));
    *in_domain = 1;
    return SREF_OK;
}

int sref_pair_increment(double tau, double G, double mi, double mj,
                        const double ri[3], const double vi[3],
                        const double rj[3], const double vj[3], int solver,
                        double dr[3], double dv[3])
{
    double X[3], W[3], x0[3];
    double h = 0.5 * tau;
    for (int c = 0; c < 3; ++c) {
        X[c] = ri[c] - rj[c];
        W[c] = vi[c] - vj[c];
        x0[c] = X[c] - W[c] * h;
    }
    double mu = G * (mi + mj);

    if (solver == SREF_SOLVER_DKD) {
        /* eq. (28): the Kepler flow replaced by drift-kick-drift. */
        double r[3], v[3];
        for (int c = 0; c < 3; ++c) r[c] = x0[c] + W[c] * h; /* 28b */
        double d = sqrt(dot3(r, r));
        if (!(d > 0.0)) return SREF_ECOLLIDE;
        double s = -mu / (d * d * d);
        for (int c = 0; c < 3; ++c) v[c] = W[c] + tau * (s * r[c]); /* 28c */
        for (int c = 0; c < 3; ++c) r[c] = r[c] + v[c] * h;          /* 28d */
        for (int c = 0; c < 3; ++c) r[c] = r[c] - v[c] * h;          /* 28e */
        for (int c = 0; c < 3; ++c) {
            dr[c] = r[c] - X[c];
            dv[c] = v[c] - W[c];
        }
        return SREF_OK;
    }

    double x1[3], w1[3], k[4];
    int rc = sref_kepler(tau, mu, x0, W, x1, w1, k, NULL);
    if (rc) return rc;
    if (solver == SREF_SOLVER_KEPLER_LITERAL) {
        /* Listing 1: rr1 = r1 - v1 tau/2, then subtract the starting state. */
        for (int c = 0; c < 3; ++c) {
            dr[c] = (x1[c] - w1[c] * h) - X[c];
            dv[c] = w1[c] - W[c];
        }
        return SREF_OK;
    }
    /* The same increments written through the Lagrange coefficients, so the
     * free drift cancels exactly instead of in rounded subtractions:
     *   dr = (f - 1 - fdot tau/2) x0 + (g - tau - (gdot - 1) tau/2) W
     *   dv = fdot x0 + (gdot - 1) W                                       */
    double a = k[0] - h * k[2];
    double b = k[1] - h * k[3];
    for (int c = 0; c < 3; ++c) {
        dr[c] = a * x0[c] + b * W[c];
        dv[c] = k[2] * x0[c] + k[3] * W[c];
    }
    return SREF_OK;
}

/* The general pair map behind eqs. (19a, 19b, 26): back-drift the relative
 * position by cb (eq. 17), Kepler flow over t (eq. 18), back-drift by ca.
 * With x0 = X - cb W and k = {f-1, g-t, fdot, gdot-1} of the flow:
 *   X + dr = f x0 + g W - ca (fdot x0 + gdot W),   X = x0 + cb W,
 * so dr = (f - 1 - ca fdot) x0 + (g - ca gdot - cb) W
 *       = (k0 - ca k2) x0 + ((k1 - ca k3) + (t - ca - cb)) W,
 *    dv = fdot x0 + (gdot - 1) W.                                            */
int sref_pair_map(double t, double cb, double ca, double G, double mi, double mj,
                  const double ri[3], const double vi[3], const double rj[3],
                  const double vj[3], double dr[3], double dv[3])
{
    double X[3], W[3], x0[3];
    for (int c = 0; c < 3; ++c) {
        X[c] = ri[c] - rj[c];
        W[c] = vi[c] - vj[c];
        x0[c] = X[c] - W[c] * cb;
    }
    double x1[3], w1[3], k[4];
    int rc = sref_kepler(t, G * (mi + mj), x0, W, x1, w1, k, NULL);
    if (rc) return rc;
    double a = k[0] - ca * k[2];
    double b = (k[1] - ca * k[3]) + (t - ca - cb);
    for (int c = 0; c < 3; ++c) {
        dr[c] = a * x0[c] + b * W[c];
        dv[c] = k[2] * x0[c] + k[3] * W[c];
    }
    return SREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Full step, eqs. (27a-d).                                                  */
/* ------------------------------------------------------------------------ */
static int all_finite(const double *a, int64_t count)
{
    for (int64_t i = 0; i < count; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* New state of row i from the half-drifted positions rh (eq. 27a done). The
 * weight of pair (i, j) is mu_ij / m_i, written m_j / (m_i + m_j) so that a
 * massless particle is defined; pairs with m_i + m_j = 0 exert nothing. */
static int step_row(int64_t n, const double *m, const double *rh,
                    const double *v, double tau, double G, int solver, int64_t i,
                    double rn[3], double vn[3])
{
    long double ar[3] = {0.0L, 0.0L, 0.0L}, av[3] = {0.0L, 0.0L, 0.0L};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double mij = m[i] + m[j];
        if (mij == 0.0) continue;
        double w = m[j] / mij;
        double dr[3], dv[3];
        int rc = sref_pair_increment(tau, G, m[i], m[j], rh + 3 * i, v + 3 * i,
                                     rh + 3 * j, v + 3 * j, solver, dr, dv);
        if (rc) return rc;
        for (int c = 0; c < 3; ++c) {
            ar[c] += (long double)w * (long double)dr[c];
            av[c] += (long double)w * (long double)dv[c];
        }
    }
    double h = 0.5 * tau;
    for (int c = 0; c < 3; ++c) {
        double rt = (double)((long double)rh[3 * i + c] + ar[c]); /* 27b */
        vn[c] = (double)((long double)v[3 * i + c] + av[c]);      /* 27c */
        rn[c] = rt + h * vn[c];                                   /* 27d */
    }
    return SREF_OK;
}

static int check_args(int64_t n, const double *m, const double *r,
                      const double *v, double tau, double G);
static double *half_drift(int64_t n, const double *r, const double *v, double tau);

/* The weighted increments w_ij (dr_ij, dv_ij) that row i of eqs. (27b, c) sums,
 * one per partner j (zero for j = i and for massless pairs), in double. */
int sref_row_terms(int64_t n, const double *m, const double *r, const double *v, double tau,
                   double G, int64_t i, double *dr_terms, double *dv_terms)
{
    int rc = check_args(n, m, r, v, tau, G);
    if (rc) return rc;
    if (i < 0 || i >= n || !dr_terms || !dv_terms) return SREF_EINVAL;
    double *rh = half_drift(n, r, v, tau);
    if (!rh) return SREF_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        for (int c = 0; c < 3; ++c) dr_terms[3 * j + c] = dv_terms[3 * j + c] = 0.0;
        double mij = m[i] + m[j];
        if (j == i || mij == 0.0) continue;
        double w = m[j] / mij;
        double dr[3], dv[3];
        rc = sref_pair_increment(tau, G, m[i], m[j], rh + 3 * i, v + 3 * i, rh + 3 * j,
                                 v + 3 * j, SREF_SOLVER_KEPLER, dr, dv);
        if (rc) break;
        for (int c = 0; c < 3; ++c) {
            dr_terms[3 * j + c] = w * dr[c];
            dv_terms[3 * j + c] = w * dv[c];
        }
    }
    free(rh);
    return rc;
}

static int check_args(int64_t n, const double *m, const double *r,
                      const double *v, double tau, double G)
{
    if (n < 1 || !m || !r || !v) return SREF_EINVAL;
    if (!isfinite(tau) || !isfinite(G) || G < 0.0) return SREF_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!(m[i] >= 0.0)) return SREF_EINVAL;
    if (!all_finite(m, n) || !all_finite(r, 3 * n) || !all_finite(v, 3 * n))
        return SREF_ENONFINITE;
    return SREF_OK;
}

static double *half_drift(int64_t n, const double *r, const double *v, double tau)
{
    double *rh = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!rh) return NULL;
    double h = 0.5 * tau;
    for (int64_t i = 0; i < 3 * n; ++i) rh[i] = r[i] + h * v[i]; /* 27a */
    return rh;
}

int sref_step_rows(int64_t n, const double *m, const double *r, const double *v,
                   double tau, double G, int64_t nrows, const int64_t *rows,
                   double *r_out, double *v_out)
{
    int rc = check_args(n, m, r, v, tau, G);
    if (rc) return rc;
    for (int64_t k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= n) return SREF_EINVAL;
    double *rh = half_drift(n, r, v, tau);
    if (!rh) return SREF_EINVAL;
    int status = SREF_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int64_t k = 0; k < nrows; ++k) {
        int e = step_row(n, m, rh, v, tau, G, SREF_SOLVER_KEPLER, rows[k],
                         r_out + 3 * k, v_out + 3 * k);
        if (e < status) status = e;
    }
    free(rh);
    if (status) return status;
    if (!all_finite(r_out, 3 * nrows) || !all_finite(v_out, 3 * nrows))
        return SREF_ENONFINITE;
    return SREF_OK;
}

int sref_step(int64_t n, const double *m, double *r, double *v, double tau,
              double G, int solver)
{
    int rc = check_args(n, m, r, v, tau, G);
    if (rc) return rc;
    if (solver < SREF_SOLVER_KEPLER || solver > SREF_SOLVER_DKD) return SREF_EINVAL;
    double *rh = half_drift(n, r, v, tau);
    double *rn = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vn = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!rh || !rn || !vn) {
        free(rh);
        free(rn);
        free(vn);
        return SREF_EINVAL;
    }
    int status = SREF_OK;
#pragma omp parallel for schedule(dynamic, 4) reduction(min : status)
    for (int64_t i = 0; i < n; ++i) {
        int e = step_row(n, m, rh, v, tau, G, solver, i, rn + 3 * i, vn + 3 * i);
        if (e < status) status = e;
    }
    if (status == SREF_OK && (!all_finite(rn, 3 * n) || !all_finite(vn, 3 * n)))
        status = SREF_ENONFINITE;
    if (status == SREF_OK) {
        memcpy(r, rn, sizeof(double) * 3 * (size_t)n);
        memcpy(v, vn, sizeof(double) * 3 * (size_t)n);
    }
    free(rh);
    free(rn);
    free(vn);
    return status;
}

int sref_evolve(int64_t n, const double *m, double *r, double *v, double tau,
                int64_t nsteps, double G, int solver)
{
    if (nsteps < 0) return SREF_EINVAL;
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc = sref_step(n, m, r, v, tau, G, solver);
        if (rc) return rc;
    }
    return SREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Compositions of the step (Sec. 2.2): eq. (24) unmerged, and the triple    */
/* jump of eq. (25).                                                         */
/* ------------------------------------------------------------------------ */

/* Row i of a W stage: the eq. (23) sums with the pair map (t, cb, ca), from
 * the state (r, v) that every pair of the stage sees. */
static int stage_row(int64_t n, const double *m, const double *r, const double *v,
                     double t, double cb, double ca, double G, int64_t i, double rn[3],
                     double vn[3])
{
    long double ar[3] = {0.0L, 0.0L, 0.0L}, av[3] = {0.0L, 0.0L, 0.0L};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double mij = m[i] + m[j];
        if (mij == 0.0) continue;
        double w = m[j] / mij;
        double dr[3], dv[3];
        int rc = sref_pair_map(t, cb, ca, G, m[i], m[j], r + 3 * i, v + 3 * i, r + 3 * j,
                               v + 3 * j, dr, dv);
        if (rc) return rc;
        for (int c = 0; c < 3; ++c) {
            ar[c] += (long double)w * (long double)dr[c];
            av[c] += (long double)w * (long double)dv[c];
        }
    }
    for (int c = 0; c < 3; ++c) {
        rn[c] = (double)((long double)r[3 * i + c] + ar[c]);
        vn[c] = (double)((long double)v[3 * i + c] + av[c]);
    }
    return SREF_OK;
}

int sref_w_stage(int64_t n, const double *m, double *r, double *v, double t, double cb,
                 double ca, double G)
{
    int rc = check_args(n, m, r, v, t, G);
    if (rc) return rc;
    if (!isfinite(cb) || !isfinite(ca)) return SREF_EINVAL;
    double *rn = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vn = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!rn || !vn) {
        free(rn);
        free(vn);
        return SREF_EINVAL;
    }
    int status = SREF_OK;
#pragma omp parallel for schedule(dynamic, 4) reduction(min : status)
    for (int64_t i = 0; i < n; ++i) {
        int e = stage_row(n, m, r, v, t, cb, ca, G, i, rn + 3 * i, vn + 3 * i);
        if (e < status) status = e;
    }
    if (status == SREF_OK && (!all_finite(rn, 3 * n) || !all_finite(vn, 3 * n)))
        status = SREF_ENONFINITE;
    if (status == SREF_OK) {
        memcpy(r, rn, sizeof(double) * 3 * (size_t)n);
        memcpy(v, vn, sizeof(double) * 3 * (size_t)n);
    }
    free(rn);
    free(vn);
    return status;
}

/* Free drift of every particle by d (eqs. 27a, 27d). */
static void drift(int64_t n, double *r, const double *v, double d)
{
    for (int64_t i = 0; i < 3 * n; ++i) r[i] = r[i] + d * v[i];
}

/* eq. (24): drift tau/2, W(tau/2) with eq. (19b) pairs, W(tau/2) with eq.
 * (19a) pairs, drift tau/2.  On error r and v are left unchanged. */
static int unmerged_step(int64_t n, const double *m, double *r, double *v, double tau,
                         double G)
{
    double h = 0.5 * tau;
    double *r1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *v1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!r1 || !v1) {
        free(r1);
        free(v1);
        return SREF_EINVAL;
    }
    memcpy(r1, r, sizeof(double) * 3 * (size_t)n);
    memcpy(v1, v, sizeof(double) * 3 * (size_t)n);
    drift(n, r1, v1, h);
    int rc = sref_w_stage(n, m, r1, v1, h, h, 0.0, G);   /* eq. (19b) */
    if (!rc) rc = sref_w_stage(n, m, r1, v1, h, 0.0, h, G); /* eq. (19a) */
    if (!rc) {
        drift(n, r1, v1, h);
        if (!all_finite(r1, 3 * n)) rc = SREF_ENONFINITE;
    }
    if (!rc) {
        memcpy(r, r1, sizeof(double) * 3 * (size_t)n);
        memcpy(v, v1, sizeof(double) * 3 * (size_t)n);
    }
    free(r1);
    free(v1);
    return rc;
}

int sref_evolve_scheme(int64_t n, const double *m, double *r, double *v, double tau,
                       int64_t nsteps, double G, int scheme)
{
    if (nsteps < 0) return SREF_EINVAL;
    if (scheme < SREF_SCHEME_PSI || scheme > SREF_SCHEME_TRIPLE_JUMP) return SREF_EINVAL;
    int rc = check_args(n, m, r, v, tau, G);
    if (rc) return rc;
    /* Yoshida's triple jump: the outer weights g1 and the inner g0 sum to one
     * and cancel the third-order error of a symmetric second-order step,
     * 2 g1^3 + g0^3 = 0.  g1 = 1/(2 - 2^(1/3)) = 1.35120719195965763..., here
     * its correctly rounded double (the libm expression can be 1-2 ulps off);
     * g0 = 1 - 2 g1 is exact in double. */
    const double g1 = 0x1.59e8b6eb96338p+0;
    const double g0 = 1.0 - 2.0 * g1;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (scheme == SREF_SCHEME_PSI) {
            rc = sref_step(n, m, r, v, tau, G, SREF_SOLVER_KEPLER);
        } else if (scheme == SREF_SCHEME_UNMERGED) {
            rc = unmerged_step(n, m, r, v, tau, G);
        } else {
            rc = sref_step(n, m, r, v, g1 * tau, G, SREF_SOLVER_KEPLER);
            if (!rc) rc = sref_step(n, m, r, v, g0 * tau, G, SREF_SOLVER_KEPLER);
            if (!rc) rc = sref_step(n, m, r, v, g1 * tau, G, SREF_SOLVER_KEPLER);
        }
        if (rc) return rc;
    }
    return SREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Close-pair hybrid: the Kepler map of eq. (26) for close pairs, the eq. (28) */
/* drift-kick-drift map for the rest.                                        */
/* ------------------------------------------------------------------------ */
int sref_pair_is_close(double tau, double G, double mi, double mj, const double X[3],
                       const double W[3], double eta)
{
    double mu = G * (mi + mj);
    double r2 = fma(X[0], X[0], fma(X[1], X[1], X[2] * X[2]));
    double w2 = fma(W[0], W[0], fma(W[1], W[1], W[2] * W[2]));
    double t2 = tau * tau;
    double e2 = eta * eta;
    double e4 = e2 * e2;
    double A = t2 * mu;
    double r3 = (r2 * r2) * r2;
    /* tau sqrt(mu / r^3) > eta, squared twice */
    if (A * A > e4 * r3) return 1;
    /* tau |W| / r > eta, squared */
    if (t2 * w2 > e2 * r2) return 1;
    return 0;
}

/* Row i of the hybrid step from the half-drifted positions rh; *nk counts the
 * Kepler pairs (i, j) with j > i. */
static int hybrid_row(int64_t n, const double *m, const double *rh, const double *v,
                      double tau, double G, double eta, int64_t i, double rn[3],
                      double vn[3], int64_t *nk)
{
    long double ar[3] = {0.0L, 0.0L, 0.0L}, av[3] = {0.0L, 0.0L, 0.0L};
    int64_t kep = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double mij = m[i] + m[j];
        if (mij == 0.0) continue;
        double w = m[j] / mij;
        double X[3], W[3];
        for (int c = 0; c < 3; ++c) {
            X[c] = rh[3 * i + c] - rh[3 * j + c];
            W[c] = v[3 * i + c] - v[3 * j + c];
        }
        int close = sref_pair_is_close(tau, G, m[i], m[j], X, W, eta);
        if (close && j > i) ++kep;
        double dr[3], dv[3];
        int rc = sref_pair_increment(tau, G, m[i], m[j], rh + 3 * i, v + 3 * i, rh + 3 * j,
                                     v + 3 * j, close ? SREF_SOLVER_KEPLER : SREF_SOLVER_DKD,
                                     dr, dv);
        if (rc) return rc;
        for (int c = 0; c < 3; ++c) {
            ar[c] += (long double)w * (long double)dr[c];
            av[c] += (long double)w * (long double)dv[c];
        }
    }
    double h = 0.5 * tau;
    for (int c = 0; c < 3; ++c) {
        double rt = (double)((long double)rh[3 * i + c] + ar[c]); /* 27b */
        vn[c] = (double)((long double)v[3 * i + c] + av[c]);      /* 27c */
        rn[c] = rt + h * vn[c];                                   /* 27d */
    }
    if (nk) *nk = kep;
    return SREF_OK;
}

int sref_step_hybrid(int64_t n, const double *m, double *r, double *v, double tau,
                     double G, double eta, int64_t *n_kepler)
{
    int rc = check_args(n, m, r, v, tau, G);
    if (rc) return rc;
    if (!(eta > 0.0) || !isfinite(eta)) return SREF_EINVAL;
    double *rh = half_drift(n, r, v, tau);
    double *rn = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vn = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!rh || !rn || !vn) {
        free(rh);
        free(rn);
        free(vn);
        return SREF_EINVAL;
    }
    int status = SREF_OK;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(min : status) reduction(+ : total)
    for (int64_t i = 0; i < n; ++i) {
        int64_t nk = 0;
        int e = hybrid_row(n, m, rh, v, tau, G, eta, i, rn + 3 * i, vn + 3 * i, &nk);
        if (e < status) status = e;
        total += nk;
    }
    if (status == SREF_OK && (!all_finite(rn, 3 * n) || !all_finite(vn, 3 * n)))
        status = SREF_ENONFINITE;
    if (status == SREF_OK) {
        memcpy(r, rn, sizeof(double) * 3 * (size_t)n);
        memcpy(v, vn, sizeof(double) * 3 * (size_t)n);
        if (n_kepler) *n_kepler = total;
    }
    free(rh);
    free(rn);
    free(vn);
    return status;
}

int sref_step_rows_hybrid(int64_t n, const double *m, const double *r, const double *v,
                          double tau, double G, double eta, int64_t nrows,
                          const int64_t *rows, double *r_out, double *v_out)
{
    int rc = check_args(n, m, r, v, tau, G);
    if (rc) return rc;
    if (!(eta > 0.0) || !isfinite(eta)) return SREF_EINVAL;
    for (int64_t k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= n) return SREF_EINVAL;
    double *rh = half_drift(n, r, v, tau);
    if (!rh) return SREF_EINVAL;
    int status = SREF_OK;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
    for (int64_t k = 0; k < nrows; ++k) {
        int e = hybrid_row(n, m, rh, v, tau, G, eta, rows[k], r_out + 3 * k, v_out + 3 * k,
                           NULL);
        if (e < status) status = e;
    }
    free(rh);
    if (status) return status;
    if (!all_finite(r_out, 3 * nrows) || !all_finite(v_out, 3 * nrows))
        return SREF_ENONFINITE;
    return SREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics: H = H_T + H_U of eqs. (1-3), momentum, angular momentum and  */
/* centre of mass.  Row partial sums are combined serially for a result that */
/* does not depend on the thread count.                                      */
/* ------------------------------------------------------------------------ */
int sref_energy(int64_t n, const double *m, const double *r, const double *v,
                double G, double out[12])
{
    if (n < 1 || !m || !r || !v || !out) return SREF_EINVAL;
    long double *urow = (long double *)malloc(sizeof(long double) * (size_t)n);
    if (!urow) return SREF_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        long double u = 0.0L;
        for (int64_t j = i + 1; j < n; ++j) {
            long double dx = (long double)r[3 * i] - r[3 * j];
            long double dy = (long double)r[3 * i + 1] - r[3 * j + 1];
            long double dz = (long double)r[3 * i + 2] - r[3 * j + 2];
            u -= (long double)m[i] * m[j] / sqrtl(dx * dx + dy * dy + dz * dz);
        }
        urow[i] = u;
    }
    long double K = 0, U = 0, M = 0, P[3] = {0, 0, 0}, L[3] = {0, 0, 0},
                R[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double *ri = r + 3 * i, *vi = v + 3 * i;
        long double mi = m[i];
        U += urow[i];
        K += 0.5L * mi *
             ((long double)vi[0] * vi[0] + (long double)vi[1] * vi[1] +
              (long double)vi[2] * vi[2]);
        M += mi;
        for (int c = 0; c < 3; ++c) {
            P[c] += mi * vi[c];
            R[c] += mi * ri[c];
        }
        L[0] += mi * ((long double)ri[1] * vi[2] - (long double)ri[2] * vi[1]);
        L[1] += mi * ((long double)ri[2] * vi[0] - (long double)ri[0] * vi[2]);
        L[2] += mi * ((long double)ri[0] * vi[1] - (long double)ri[1] * vi[0]);
    }
    free(urow);
    U *= G;
    out[0] = (double)(K + U);
    out[1] = (double)K;
    out[2] = (double)U;
    for (int c = 0; c < 3; ++c) {
        out[3 + c] = (double)P[c];
        out[6 + c] = (double)L[c];
        out[9 + c] = M > 0 ? (double)(R[c] / M) : 0.0;
    }
    return SREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Learned-starter network reference: plain loops in fp64, written from the  */
/* definition of a two-hidden-layer perceptron and the chain rule.           */
/* ------------------------------------------------------------------------ */
enum { MLP_IN = 8, MLP_H = 64 };
#define MLP_OFF_W1 0
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_H * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_H)

static double mlp_one(const double *p, const double *x, double *z1, double *a1,
                      double *z2, double *a2)
{
    const double *W1 = p + MLP_OFF_W1, *b1 = p + MLP_OFF_B1;
    const double *W2 = p + MLP_OFF_W2, *b2 = p + MLP_OFF_B2;
    const double *W3 = p + MLP_OFF_W3, *b3 = p + MLP_OFF_B3;
    for (int i = 0; i < MLP_H; ++i) {
        double z = b1[i];
        for (int j = 0; j < MLP_IN; ++j) z += W1[i * MLP_IN + j] * x[j];
        z1[i] = z;
        a1[i] = z > 0.0 ? z : 0.0;
    }
    for (int i = 0; i < MLP_H; ++i) {
        double z = b2[i];
        for (int j = 0; j < MLP_H; ++j) z += W2[i * MLP_H + j] * a1[j];
        z2[i] = z;
        a2[i] = z > 0.0 ? z : 0.0;
    }
    double o = b3[0];
    for (int j = 0; j < MLP_H; ++j) o += W3[j] * a2[j];
    return o;
}

int sref_mlp_forward(const double *params, int64_t batch, const double *x, double *out)
{
    if (!params || !x || !out || batch < 0) return SREF_EINVAL;
    for (int64_t b = 0; b < batch; ++b) {
        double z1[MLP_H], a1[MLP_H], z2[MLP_H], a2[MLP_H];
        out[b] = mlp_one(params, x + MLP_IN * b, z1, a1, z2, a2);
    }
    return SREF_OK;
}

int sref_mlp_loss_grad(const double *params, int64_t batch, const double *x,
                       const double *y, double *loss, double *grad)
{
    if (!params || !x || !y || !loss || !grad || batch < 1) return SREF_EINVAL;
    const double *W2 = params + MLP_OFF_W2, *W3 = params + MLP_OFF_W3;
    memset(grad, 0, sizeof(double) * SREF_MLP_PARAMS);
    double L = 0.0;
    for (int64_t b = 0; b < batch; ++b) {
        const double *xb = x + MLP_IN * b;
        double z1[MLP_H], a1[MLP_H], z2[MLP_H], a2[MLP_H], d2[MLP_H], d1[MLP_H];
        const double o = mlp_one(params, xb, z1, a1, z2, a2);
        const double e = o - y[b];
        L += e * e;
        const double g = 2.0 * e / (double)batch; /* dL/do */
        grad[MLP_OFF_B3] += g;
        for (int j = 0; j < MLP_H; ++j) {
            grad[MLP_OFF_W3 + j] += g * a2[j];
            d2[j] = z2[j] > 0.0 ? g * W3[j] : 0.0; /* dL/dz2 */
        }
        for (int i = 0; i < MLP_H; ++i) {
            grad[MLP_OFF_B2 + i] += d2[i];
            for (int j = 0; j < MLP_H; ++j) grad[MLP_OFF_W2 + i * MLP_H + j] += d2[i] * a1[j];
        }
        for (int j = 0; j < MLP_H; ++j) {
            double s = 0.0;
            for (int i = 0; i < MLP_H; ++i) s += W2[i * MLP_H + j] * d2[i];
            d1[j] = z1[j] > 0.0 ? s : 0.0; /* dL/dz1 */
        }
        for (int i = 0; i < MLP_H; ++i) {
            grad[MLP_OFF_B1 + i] += d1[i];
            for (int j = 0; j < MLP_IN; ++j) grad[MLP_OFF_W1 + i * MLP_IN + j] += d1[i] * xb[j];
        }
    }
    *loss = L / (double)batch;
    return SREF_OK;
}

int sref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void sref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
