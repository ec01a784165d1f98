// Two-body (Kepler) flow of one pair for the Sakura pair map, in FP64.
//
// The paper evolves every pair with a universal-variable Kepler solver
// (Sec. 2.3, eq. 18) and then removes the free drift of the two half
// back-drifts of eq. (26).  This device routine writes the same flow through
// Stumpff's G-functions of the regularised time s (dt/ds = r):
//
//   G_k(s) = s^k c_k(beta s^2),  beta = 2 mu / r0 - |w0|^2,  eta = x0 . w0,
//   t(s)   = r0 G1 + eta G2 + mu G3 = r0 s + eta G2 + zeta G3,
//   r(s)   = dt/ds = r0 + eta G1 + zeta G2 > 0,   zeta = mu - beta r0,
//
// (the second forms use G1 = s - beta G3 and G0 = 1 - beta G2),
//
// and solves t(s) = tau with a Laguerre iteration (order 5, as Conway 1986
// does for Kepler's equation), safeguarded by a bracket on the monotone t(s).
// From the root it forms the Lagrange coefficients as differences from the
// free drift (f-1, g-tau, fdot, gdot-1), so that the pair increments
//
//   dr = (f-1 - fdot tau/2) x0 + (g-tau - (gdot-1) tau/2) w0
//   dv = fdot x0 + (gdot-1) w0
//
// carry no cancellation of the drift.  There is one code path for elliptic,
// parabolic and hyperbolic motion: the Stumpff functions come from a fixed
// seven-term series after quartering the argument, rebuilt with the doubling
// identities, so typical pairs (|beta s^2| << 1) take no data-dependent branch.
#pragma once

#ifndef SAKURA_HD
#define SAKURA_HD __device__
#endif

namespace kep {

struct KeplerParams {
    double tol;   // relative convergence tolerance on s
    int max_iter; // Laguerre iterations before the pair is declared unconverged
};
// The library's defaults (sakura_opts with zeros).
constexpr double DEFAULT_TOL = 0x1p-50;
constexpr int DEFAULT_MAX_ITER = 40;

// c2(z), c3(z) from sum_m (-z)^m / (2m+k)! for |z| <= 1/4 (seven terms leave a
// truncation below 0.05 ulp), extended to any z by c2(4z) = c1(z)^2 / 2 and
// c3(4z) = (c2(z) + c0(z) c3(z)) / 4 with c0 = 1 - z c2, c1 = 1 - z c3.
SAKURA_HD inline void stumpff23(double z, double &c2, double &c3)
{
    int k = 0;
    double zr = z;
    // exact scaling by powers of two; the bound keeps z = +-inf from looping
    // (1100 quarterings span the whole double range)
    while (fabs(zr) > 0.25 && k < 1100) {
        zr *= 0.25;
        ++k;
    }
    c2 = 1.0 / 87178291200.0;            // 1/14!
    c2 = fma(c2, -zr, 1.0 / 479001600.0); // 1/12!
    c2 = fma(c2, -zr, 1.0 / 3628800.0);   // 1/10!
    c2 = fma(c2, -zr, 1.0 / 40320.0);     // 1/8!
    c2 = fma(c2, -zr, 1.0 / 720.0);       // 1/6!
    c2 = fma(c2, -zr, 1.0 / 24.0);        // 1/4!
    c2 = fma(c2, -zr, 0.5);               // 1/2!
    c3 = 1.0 / 1307674368000.0;           // 1/15!
    c3 = fma(c3, -zr, 1.0 / 6227020800.0); // 1/13!
    c3 = fma(c3, -zr, 1.0 / 39916800.0);   // 1/11!
    c3 = fma(c3, -zr, 1.0 / 362880.0);     // 1/9!
    c3 = fma(c3, -zr, 1.0 / 5040.0);       // 1/7!
    c3 = fma(c3, -zr, 1.0 / 120.0);        // 1/5!
    c3 = fma(c3, -zr, 1.0 / 6.0);          // 1/3!
    for (; k > 0; --k) {
        double c0 = fma(-zr, c2, 1.0);
        double c1 = fma(-zr, c3, 1.0);
        c3 = 0.25 * fma(c0, c3, c2);
        c2 = 0.5 * c1 * c1;
        zr *= 4.0;
    }
}

// Reciprocal and reciprocal square root from the hardware estimates
// (v_rcp_f64 / v_rsq_f64, relative error e near 2^-23) refined by one step of
// third order: y (1 + e + e^2) resp. y (1 + e/2 + 3 e^2/8) leave an error of
// order e^3, below the rounding of the result.
SAKURA_HD inline double rcp_refined(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}
SAKURA_HD inline double rcp_step(double x) // about 2^-46
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}
SAKURA_HD inline double rsqrt_refined(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
SAKURA_HD inline double sqrt_step(double x) // about 2^-46, x >= 0
{
    if (!(x > 0.0)) return 0.0;
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return x * y;
}

// z + c and a b + c with the constant c read from a scalar register pair by
// the vector operation itself; left to the compiler, such a constant is moved
// into two vector registers first (as the accumulator of a v_fmac), which
// costs two vector instructions on the unit that bounds the pair kernels.
#ifndef SAKURA_NO_SCALAR_ASM
SAKURA_HD inline double add_sc(double z, double c)
{
    double r;
    asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(z), "s"(c));
    return r;
}
SAKURA_HD inline double fma_sc(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}
SAKURA_HD inline double vmov_sc(double c)
{
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "s"(c));
    return r;
}
SAKURA_HD inline double fma_v(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
#else
inline double add_sc(double z, double c) { return z + c; }
inline double fma_sc(double a, double b, double c) { return fma(a, b, c); }
inline double fma_v(double a, double b, double c) { return fma(a, b, c); }
inline double vmov_sc(double c) { return c; }
#endif

// The same functions for |z| <= 2^-6 only: five terms each leave a truncation
// below 4e-18 relative (the first term dropped, z^5/12! against 1/2 and
// z^5/13! against 1/6), without the argument reduction.
SAKURA_HD inline void stumpff23_small(double z, double &c2, double &c3)
{
    c2 = fma(fma(fma(fma(-z, 1.0 / 3628800.0, 1.0 / 40320.0), -z, 1.0 / 720.0), -z, 1.0 / 24.0),
             -z, 0.5);
    c3 = fma(fma(fma(fma(-z, 1.0 / 39916800.0, 1.0 / 362880.0), -z, 1.0 / 5040.0), -z,
                 1.0 / 120.0),
             -z, 1.0 / 6.0);
}

#ifndef SAKURA_WAVE_ALL
#define SAKURA_WAVE_ALL(pred) __all(pred) // every active lane of the wavefront
#endif

struct PairFlow {
    // Lagrange coefficients as differences from the free drift, per unit mu:
    // (f-1)/mu, (g-tau)/mu, fdot/mu, (gdot-1)/mu.  All four are proportional
    // to mu, so the caller's weights m_j/(m_i+m_j) become G m_j, with no
    // division per pair.
    double fm1, gmt, fdot, gdm1;
    int iters;
    bool converged;
    bool safeguarded; // a bisection or bracket-expansion step was needed
    bool restarted;   // the search was started again from the plain starter
    bool in_dom;      // kepler_flow_domain: the pair lies in the given domain
    double resid;     // |t(s) - t| / |t| at the accepted root (policies with resid; else 0)
};

// State of the root search on t(s) = tau.
struct KepIter {
    double s, lo, hi;       // iterate and bracket
    double ds_prev, F_prev; // for the stall tests
    double G1, G2, G3, r;   // G-functions and radius at the accepted root
    bool safeguarded;
};

// The quantities of one evaluation of t(s) - t at s, with c2(z), c3(z) of
// z = beta s^2 evaluated by the tier every lane of the wavefront qualifies
// for: 0 nothing; 1 |z| <= 2^-6 (five-term series); 2 |z| <= 2^-14, where
// three terms of each series leave a truncation below 2^-56.
struct KepEval {
    double G0, G1, G2, G3, F, r;
};
// F'' = t''(s) = eta G0 + zeta G1, formed where a step or test needs it (the
// Newton step of the common path does not)
SAKURA_HD inline double kepler_fpp(const KepEval &e, double eta, double zeta)
{
    return fma(eta, e.G0, zeta * e.G1);
}
template <int TIER>
SAKURA_HD inline KepEval kepler_eval(double s, double beta, double eta, double zeta, double r0,
                                     double t)
{
    const double s2 = s * s;
    const double z = beta * s2;
    double c2, c3;
    if (TIER == 2) {
        // 1/2 - z/24 + z^2/720 and 1/6 - z/120 + z^2/5040, written with one
        // non-trivial constant per operation (a VALU operation reads at most
        // one scalar), which saves the moves of constants into vector registers
        c2 = fma((1.0 / 720.0) * z, add_sc(z, -30.0), 0.5);
        c3 = fma_sc((1.0 / 5040.0) * z, add_sc(z, -42.0), 1.0 / 6.0);
    } else if (TIER == 1) {
        stumpff23_small(z, c2, c3);
    } else {
        stumpff23(z, c2, c3);
    }
    KepEval e;
    e.G1 = s * fma(-z, c3, 1.0);
    e.G2 = s2 * c2;
    e.G3 = s2 * s * c3;
    e.G0 = fma(-z, c2, 1.0);
    e.F = fma(r0, s, fma(eta, e.G2, fma(zeta, e.G3, -t)));
    e.r = fma(eta, e.G1, fma(zeta, e.G2, r0));
    return e;
}

// Laguerre step of order 5 at an evaluation, or the Halley step
// F r / (r^2 - F F''/2) where |F F''| is small against r^2.  HALLEY 1 (every
// lane has |z| <= 2^-14) takes it while |F F''| <= 2^-22 r^2, where the two
// agree to a relative q^2/10, q = 5 F F'' / 4 r^2, i.e. below 2^-42.  HALLEY 2
// (the first evaluation of the other tiers, whose acceptance test bounds the
// cubic error of either step) takes it while |F F''| <= 2^-8 r^2: near the
// root, where a step is accepted, q is small anyway (q ~ ds t''/r), and farther
// out Laguerre's step keeps its wider convergence.  HALLEY 0: Laguerre's.
template <int HALLEY>
SAKURA_HD inline double laguerre_step(const KepEval &e, double eta, double zeta)
{
    const double FFpp = e.F * kepler_fpp(e, eta, zeta);
    if (HALLEY != 0 && fabs(FFpp) <= (HALLEY == 1 ? 0x1p-22 : 0x1p-8) * (e.r * e.r))
        return e.F * e.r * rcp_step(fma(-0.5, FFpp, e.r * e.r));
    const double disc = fma(16.0 * e.r, e.r, -20.0 * FFpp);
    return 5.0 * e.F * rcp_step(e.r + sqrt_step(fabs(disc)));
}

// Acceptance of the root s - ds after a step from s: the step taken
// (Laguerre's, or Halley's) has a cubic error, e_new ~ C e^3 with
// |C| <= (t2 / r)^2 + |t3| / r for both (t2, t3 the second and third
// derivatives of t(s); Laguerre's order-5 constant differs from Halley's
// t2^2/4r^2 - t3/6r by 5 t2^2 / 32 r^2), so once the step is small
// (|ds| <= 2^-16 |s - ds|, where that expansion holds) the error left is
// bounded by (|t3| r + t2^2) |ds|^3 / r^2, and the step is accepted when that
// is below tol |s - ds| / 4 (tested without divisions).
SAKURA_HD inline bool step_accepted(const KepEval &e, double ds, double sn, double beta,
                                    double eta, double zeta, double tol)
{
    const double ads = fabs(ds), asn = fabs(sn);
    const double aFpp = fabs(kepler_fpp(e, eta, zeta));
    const double Fppp = fma(zeta, e.G0, -beta * eta * e.G1);
    const double err_r2 = ads * ads * ads * fma(fabs(Fppp), e.r, aFpp * aFpp);
    return ads <= 0x1p-16 * asn && err_r2 <= 0.25 * tol * asn * e.r * e.r;
}

// The G-functions carried from s to s + d by their Taylor series
// (dG_k/ds = G_{k-1}, dG_0/ds = -beta G_1), to third order, and r there.
SAKURA_HD inline void taylor_shift3(KepIter &st, const KepEval &e, double d, double beta,
                                    double eta, double zeta, double r0)
{
    const double d2 = 0.5 * d * d, d3 = d2 * d * (1.0 / 3.0);
    const double mbG1 = -beta * e.G1, mbG0 = -beta * e.G0;
    st.G3 = fma(d3, e.G0, fma(d2, e.G1, fma(d, e.G2, e.G3)));
    st.G2 = fma(d3, mbG1, fma(d2, e.G0, fma(d, e.G1, e.G2)));
    st.G1 = fma(d3, mbG0, fma(d2, mbG1, fma(d, e.G0, e.G1)));
    st.r = fma(eta, st.G1, fma(zeta, st.G2, r0));
}

// First evaluation, at the starter.  Returns 2 when s - ds is the root
// (st.s moved there, with the G-functions and r carried there by their Taylor
// series), else 0 with st.s kept and F and the step ds left (signed) in
// st.F_prev and st.ds_prev for kepler_search to go on from.  The root is taken
// when the step is below tol |s| (or F = 0), or when the step is accepted by
// its error bound; no bracket is consulted: t(s) increases strictly (r > 0),
// so the root is unique.  Every lane forms the carried G-functions (those that
// go on do not use them), so the common path has no divergent writes.  In
// tier 2 they are carried to first order when |ds| <= 2^-28 |s - ds| on every
// taking lane, to second order when |ds| <= 2^-18 |s - ds| (the dropped terms
// are then below 3 (ds/s)^2 resp. (ds/s)^3, i.e. below 2^-54 of each
// function), else, as in the other tiers, to third order.
//
// With EASY (tier 2, every lane of the wavefront started by the plain starter
// with corrections |corr1| + |corr2| = c <= 2^-9, and tol >= 2^-52) the error
// bound needs no evaluation: at such a starter |t2 s / r| <= 8.2 c and
// |t3| s^2 / r <= 6.2 c (t2 s ~ eta s + zeta s^2, whose terms the corrections
// bound through 2 |corr1| and 6 |A3 u^2| <= 6 (c + 2 c^2)), so
// C s^2 <= 6.2 c + 67 c^2 <= 0.0124, and a step with |ds| <= 2^-16 |s - ds|
// leaves an error below 2^-48 C s^2 |s - ds| <= tol |s - ds| / 4.
//
// With NEWTON as well (EASY and tol >= 2^-50) the step is Newton's,
// ds = F / r, when every lane of the wavefront has |ds| <= 2^-23 |s - ds|:
// its error is t2 ds^2 / (2 r) to leading order, and |t2 s / r| <= 8.2 c
// bounds it by 4.1 c (ds/s)^2 |s| <= 2^-52.96 |s|, below tol |s| / 4 (the
// starter's own error, about the square of its corrections times u, is below
// 2^-23 for 99.9 % of a star cluster's easy wavefronts).  Otherwise the
// Halley step is taken as before.  The two agree to a relative F F'' / 2 r^2
// of the step, below the rounding of the root here.
template <int TIER>
SAKURA_HD inline int kepler_first(KepIter &st, double beta, double eta, double zeta, double r0,
                                  double t, double tol, bool easy, bool newton)
{
    const double s = st.s;
    const KepEval e = kepler_eval<TIER>(s, beta, eta, zeta, r0, t);
    double ds;
    if (TIER == 2 && newton) {
        const double dn = e.F * rcp_step(e.r);
        if (SAKURA_WAVE_ALL(fabs(dn) <= 0x1p-23 * fabs(s - dn))) {
            // every lane takes the root s - dn (the shift of the general
            // path below, with done on every lane: to first order where it
            // suffices on every lane, else to second)
            const double sn = s - dn, d = -dn;
            double G3 = fma(d, e.G2, e.G3);
            double G2 = fma(d, e.G1, e.G2);
            double G1 = fma(d, e.G0, e.G1);
            if (!SAKURA_WAVE_ALL(0x1p28 * fabs(dn) <= fabs(sn))) {
                // (a branch, not both orders formed and one selected: the
                // empty statement cannot be executed speculatively)
                asm volatile("");
                const double d2 = 0.5 * d * d;
                G3 = fma(d2, e.G1, G3);
                G2 = fma(d2, e.G0, G2);
                G1 = fma(d2, -beta * e.G1, G1);
            }
            st.G1 = G1;
            st.G2 = G2;
            st.G3 = G3;
            st.r = fma(eta, G1, fma(zeta, G2, r0));
            st.s = sn;
            // (not read after a root is taken; written, the compiler keeps this
            // path apart from the Halley step's instead of joining the two
            // with moves of the iteration state's initial values)
            st.F_prev = e.F;
            st.ds_prev = dn;
            return 2;
        }
        ds = laguerre_step<1>(e, eta, zeta);
    } else {
        ds = laguerre_step<TIER == 2 ? 1 : 2>(e, eta, zeta);
    }
    const double ads = fabs(ds);
    const double sn = s - ds;
    const double asn = fabs(sn);
    bool done;
    if (TIER == 2 && easy)
        done = ads <= tol * fabs(s) || e.F == 0.0 || ads <= 0x1p-16 * asn;
    else
        done = ads <= tol * fabs(s) || e.F == 0.0 ||
               step_accepted(e, ds, sn, beta, eta, zeta, tol);
    const double d = -ds;
    double G3 = fma(d, e.G2, e.G3);
    double G2 = fma(d, e.G1, e.G2);
    double G1 = fma(d, e.G0, e.G1);
    // order of the shift that suffices on every lane that takes the root: the
    // first, else the second, else the third (after a Newton step on every
    // lane, above, |ds| <= 2^-23 |s - ds| and the second always does)
    bool first = false, second = false;
    if (TIER == 2) {
        first = SAKURA_WAVE_ALL(!done || ads <= 0x1p-28 * asn);
        second = first || SAKURA_WAVE_ALL(!done || ads <= 0x1p-18 * asn);
    }
    if (!first) {
        const double d2 = 0.5 * d * d;
        const double mbG1 = -beta * e.G1;
        G3 = fma(d2, e.G1, G3);
        G2 = fma(d2, e.G0, G2);
        G1 = fma(d2, mbG1, G1);
        if (!second) {
            const double d3 = d2 * d * (1.0 / 3.0);
            G3 = fma(d3, e.G0, G3);
            G2 = fma(d3, mbG1, G2);
            G1 = fma(d3, -beta * e.G0, G1);
        }
    }
    st.G1 = G1;
    st.G2 = G2;
    st.G3 = G3;
    st.r = fma(eta, G1, fma(zeta, G2, r0));
    st.s = done ? sn : s;
    st.F_prev = e.F;
    st.ds_prev = ds;
    return done ? 2 : 0;
}

// A later evaluation (general tier), inside the bracket [st.lo, st.hi].
// Returns 1 / 2 as kepler_first, or 0 with st.s moved to the next iterate.
SAKURA_HD inline int kepler_iterate(KepIter &st, double beta, double eta, double zeta,
                                    double r0, double t, double tol)
{
    const double s = st.s;
    const KepEval e = kepler_eval<0>(s, beta, eta, zeta, r0, t);
    if (e.F < 0.0) st.lo = s;
    else st.hi = s;
    const double ds = laguerre_step<0>(e, eta, zeta);
    const double ads = fabs(ds), as = fabs(s);
    // Converged at s: the correction is below tol |s|, or it sits at the
    // rounding floor of F (tiny and no longer shrinking).
    if (ads <= tol * as || e.F == 0.0 || (ads <= 1e-10 * as && ads >= 0.5 * st.ds_prev)) {
        st.G1 = e.G1;
        st.G2 = e.G2;
        st.G3 = e.G3;
        st.r = e.r;
        return 1;
    }
    const double sn = s - ds;
    if (step_accepted(e, ds, sn, beta, eta, zeta, tol) && sn >= st.lo && sn <= st.hi) {
        taylor_shift3(st, e, -ds, beta, eta, zeta, r0);
        st.s = sn;
        return 2;
    }
    // Safeguard when the step leaves the bracket, or when the search crawls:
    // the residual fails to halve, or a large step fails to halve (linear
    // progress down an exponential).  A crawl inside a bracket much wider
    // than the step doubles the step; otherwise bisect, and an open bracket
    // is expanded.
    const bool stall = (fabs(e.F) > 0.5 * st.F_prev && ads > 1e-6 * as) ||
                       (ads > 0.5 * st.ds_prev && ads > 1e-3 * as);
    double next = sn;
    const bool inside = next >= st.lo && next <= st.hi;
    if (!inside || stall) {
        const double ext = s - 2.0 * ds;
        if (inside && ext > st.lo && ext < st.hi && 8.0 * ads < st.hi - st.lo)
            next = ext;
        else
            next = (st.hi - st.lo < 1e299) ? 0.5 * (st.lo + st.hi) : 2.0 * s;
        st.safeguarded = true;
    }
    st.ds_prev = ads;
    st.F_prev = fabs(e.F);
    st.s = next;
    return 0;
}

// Period reduction: for a bound orbit (beta > 0) sqrt(beta) s is the change
// of eccentric anomaly, so one period P = 2 pi mu / beta^(3/2) spans
// s = 2 pi / sqrt(beta), and with |t| <= P/2 the root lies inside that span.
// Returns the reduced time t; s_half bounds |s| (1e300 for unbound motion)
// and tshift_mu = (t - tau) / mu.
SAKURA_HD inline double reduce_time(double tau, double mu, double beta, double &s_half,
                                    double &tshift_mu)
{
    double t = tau;
    s_half = vmov_sc(1e300); // one vector move from a scalar pair, where a literal takes two
    tshift_mu = 0.0;
    if (beta > 0.0) {
        const double ib = rsqrt_refined(beta);
        s_half = 6.3 * ib; // just above 2 pi / sqrt(beta)
        const double P_mu = 6.283185307179586 * ib * ib * ib;
        const double P = P_mu * mu;
        if (fabs(t) > 0.5 * P) {
            const double k = rint(t * rcp_refined(P));
            t -= P * k;
            tshift_mu = -P_mu * k;
        }
    }
    return t;
}

// Plain starter of the root search on t(s) = t: the reversion of the Taylor
// series of t(s) = r0 s + eta s^2/2 + zeta s^3/6 - beta eta s^4/24
// - beta zeta s^5/120 + ..., i.e. with u = t / r0 and A_k = t^(k)(0) / (k! r0),
//   s = u - A2 u^2 + (2 A2^2 - A3) u^3 + (5 A2 A3 - A4 - 5 A2^3) u^4
//         + (6 A2 A4 + 3 A3^2 + 14 A2^4 - A5 - 21 A2^2 A3) u^5,
// to third order where the corrections are below 2^-9 (the reversion error is
// then about their square, which the first evaluation accepts) and to fifth
// order otherwise.  When its corrections dominate the series is no
// guide: start from the free drift u instead, or, deep in the hyperbolic
// regime (-beta u^2 > 1), from the inversion of
// t ~ exp(k|s|) (r0 k^2 + eta k sgn t + mu) / (2 k^3), k = sqrt(-beta).
// A starter beyond |s| <= s_half or of the wrong sign is replaced by u,
// clamped to that bound.
SAKURA_HD inline double starter_bounded(double s, double u, double s_half)
{
    if (!(fabs(s) <= s_half) || (s > 0.0) != (u > 0.0)) s = fmin(fmax(u, -s_half), s_half);
    return s;
}
SAKURA_HD inline double plain_starter(double t, double u, double r0, double r0inv, double eta,
                                      double zeta, double beta, double mu, double s_half,
                                      double &csum_out, bool &all_small)
{
    const double p = eta * r0inv; // 2 A2
    const double A2 = 0.5 * p;
    const double A3 = (1.0 / 6.0) * (zeta * r0inv);
    const double corr1 = -0.5 * (p * u);          // -A2 u
    const double uu = u * u;
    const double corr2 = fma(A2, p, -A3) * uu; // (2 A2^2 - A3) u^2
    const double csum = fabs(corr1) + fabs(corr2);
    csum_out = csum;
    double corr = corr1 + corr2;
    all_small = SAKURA_WAVE_ALL(csum <= 0x1p-9);
    if (all_small) {
        // third order on every lane of the wavefront: s = u (1 + corr) with
        // |corr| <= 2^-9 has the sign of u (or is zero with it), so of the
        // replacement's conditions only the bound can hold
        const double s = fma(u, corr, u);
        return SAKURA_WAVE_ALL(fabs(s) <= s_half) ? s : starter_bounded(s, u, s_half);
    }
    if (csum > 0x1p-9) {
        const double A4 = (-1.0 / 24.0) * beta * eta * r0inv;
        const double A5 = (-1.0 / 120.0) * beta * zeta * r0inv;
        const double A22 = A2 * A2;
        const double k4 = fma(5.0 * A2, A3 - A22, -A4);
        const double k5 = fma(A2, fma(6.0, A4, A2 * fma(14.0, A22, -21.0 * A3)),
                              fma(3.0 * A3, A3, -A5));
        corr += uu * u * fma(k5, u, k4);
    }
    double s = fma(u, corr, u);
    if (csum > 0.5) {
        s = u;
        if (beta < 0.0 && -beta * uu > 1.0) {
            const double k = sqrt(-beta);
            const double D = fmax(fma(r0 * k, k, fma(eta * k, copysign(1.0, t), mu)), 1e-300);
            s = copysign(log1p(2.0 * k * k * k * fabs(t) / D) / k, t);
        }
    }
    return starter_bounded(s, u, s_half);
}

// Bracket of the root: it has the sign of t since t(0) = 0 and t(s)
// increases.  For unbound motion the far end stays open (+-1e300), except
// that an unbound pair moving apart (eta sgn t >= 0) only grows in r, so
// t(s) >= r0 s and the root lies within |u|.
SAKURA_HD inline void initial_bracket(double t, double u, double beta, double eta,
                                      double s_half, double &lo, double &hi)
{
    lo = (t > 0.0) ? 0.0 : -s_half;
    hi = (t > 0.0) ? s_half : 0.0;
    if (beta <= 0.0 && eta * t >= 0.0) {
        if (t > 0.0) hi = fmin(hi, u);
        else lo = fmax(lo, u);
    }
}

// A starter policy sees every pair between the plain starter and the root
// search (all lanes of the wavefront together) and again after the search.
// start() returns START_PLAIN (keep the plain starter), START_REPLACED (it
// replaced s) or START_SKIP (the pair is solved elsewhere: the flow returns
// zero coefficients at once).  NoGuess keeps the plain starter.
enum { START_PLAIN = 0, START_REPLACED = 1, START_SKIP = 2 };
// A policy with resid = true also has the flow evaluate t(s) once more at the
// accepted root (general tier) and report the relative residual.
struct NoGuess {
    static constexpr bool active = false;
    static constexpr bool resid = false;
    SAKURA_HD int start(double, double, double, double, double, double, double, double,
                        double, double &) { return START_PLAIN; }
    SAKURA_HD void done(double, double, double, double, double, double, double, int) {}
};

// Root search from st.s until convergence or kp.max_iter evaluations.  The
// first evaluation takes the cheapest tier every lane of the wavefront
// qualifies for (almost every pair of a star cluster converges there, in
// tier 2); the pairs that go on set up the bracket and continue in the
// general tier.
SAKURA_HD inline int kepler_search(KepIter &st, double beta, double eta, double zeta, double r0,
                                   double t, double u, double s_half, const KeplerParams &kp,
                                   bool easy, int &it, bool newton = false)
{
    const double z0 = fabs(beta * (st.s * st.s)); // z as the evaluation forms it
    int res;
    if (SAKURA_WAVE_ALL(z0 <= 0x1p-14))
        res = kepler_first<2>(st, beta, eta, zeta, r0, t, kp.tol, easy, newton);
    else if (SAKURA_WAVE_ALL(z0 <= 0x1p-6))
        res = kepler_first<1>(st, beta, eta, zeta, r0, t, kp.tol, false, false);
    else
        res = kepler_first<0>(st, beta, eta, zeta, r0, t, kp.tol, false, false);
    it = 1;
    if (res == 0) {
        initial_bracket(t, u, beta, eta, s_half, st.lo, st.hi);
        const double s = st.s, F = st.F_prev, ds = st.ds_prev;
        if (F < 0.0) st.lo = s;
        else st.hi = s;
        double next = s - ds;
        if (!(next >= st.lo && next <= st.hi)) {
            next = (st.hi - st.lo < 1e299) ? 0.5 * (st.lo + st.hi) : 2.0 * s;
            st.safeguarded = true;
        }
        st.ds_prev = fabs(ds);
        st.F_prev = fabs(F);
        st.s = next;
        while (res == 0 && it < kp.max_iter) {
            ++it;
            res = kepler_iterate(st, beta, eta, zeta, r0, t, kp.tol);
        }
    }
    return res;
}

// Kepler flow over tau of the relative state (x0, w0) with parameter mu >= 0
// and r0^2 = |x0|^2 > 0 (callers substitute a trivial problem otherwise).
// With a starter policy that replaced the plain starter, a search that fails
// to converge is started again from the plain starter (PairFlow::restarted).
template <class Guess>
SAKURA_HD __attribute__((always_inline)) inline PairFlow kepler_flow(double tau, double mu,
                                                                     double x0, double x1,
                                                                     double x2,
                                      double w0, double w1, double w2, double r0sq,
                                      const KeplerParams &kp, Guess &guess)
{
    const double r0inv = rsqrt_refined(r0sq);
    const double r0 = r0sq * r0inv;
    const double eta = fma(x0, w0, fma(x1, w1, x2 * w2));
    const double vsq = fma(w0, w0, fma(w1, w1, w2 * w2));
    const double beta = fma(2.0 * mu, r0inv, -vsq);
    const double zeta = fma(-beta, r0, mu); // mu - beta r0 = d^2 r / ds^2 at s = 0

    double s_half, tshift_mu;
    const double t = reduce_time(tau, mu, beta, s_half, tshift_mu);
    const double u = t * r0inv;
    double csum;
    bool all_small; // csum <= 2^-9 on every lane
    double s = plain_starter(t, u, r0, r0inv, eta, zeta, beta, mu, s_half, csum, all_small);
    bool replaced = false;
    if (Guess::active) {
        double lo, hi;
        initial_bracket(t, u, beta, eta, s_half, lo, hi);
        const int how = guess.start(t, mu, r0, r0inv, eta, beta, u, lo, hi, s);
        if (how == START_SKIP) {
            PairFlow z;
            z.fm1 = z.gmt = z.fdot = z.gdm1 = 0.0;
            z.iters = 0;
            z.converged = true;
            z.safeguarded = z.restarted = false;
            z.in_dom = false;
            return z;
        }
        replaced = how == START_REPLACED;
    }

    // the simplified acceptance of kepler_first (uniform over the wavefront)
    const bool easy =
        kp.tol >= 0x1p-52 && all_small && (!Guess::active || SAKURA_WAVE_ALL(!replaced));
    KepIter st{s, 0.0, 0.0, 1e300, 1e300, 0.0, 0.0, 0.0, r0, false};
    int it = 0;
    int res = kepler_search(st, beta, eta, zeta, r0, t, u, s_half, kp, easy, it,
                            easy && kp.tol >= 0x1p-50);
    bool restarted = false;
    if (Guess::active && res == 0 && replaced) {
        restarted = true;
        s = plain_starter(t, u, r0, r0inv, eta, zeta, beta, mu, s_half, csum, all_small);
        st = KepIter{s, 0.0, 0.0, 1e300, 1e300, 0.0, 0.0, 0.0, r0, false};
        int it2 = 0;
        res = kepler_search(st, beta, eta, zeta, r0, t, u, s_half, kp, false, it2);
        it += it2;
    }
    PairFlow out;
    out.converged = res != 0;
    out.safeguarded = st.safeguarded;
    out.restarted = restarted;
    out.in_dom = false;
    out.resid = 0.0;
    if constexpr (Guess::resid) {
        if (t != 0.0) {
            const KepEval e = kepler_eval<0>(st.s, beta, eta, zeta, r0, t);
            out.resid = fabs(e.F) / fabs(t);
        }
    }
    const double G1 = st.G1, G2 = st.G2, G3 = st.G3, r = st.r;
    out.iters = it;
    if (Guess::active) guess.done(st.s, t, mu, r0, r0inv, eta, beta, it);
    // Lagrange coefficients at the converged s, per unit mu.
    const double rinv = rcp_refined(r);
    out.fm1 = -G2 * r0inv;
    out.gmt = tshift_mu - G3;
    out.fdot = -G1 * rinv * r0inv;
    out.gdm1 = -G2 * rinv;
    return out;
}

// The plain flow is kept out of line on purpose: the call boundary splits the
// register allocation of the pair loop from that of the solver, which
// measured about 3 % faster in the tile kernel than the inlined form (which
// keeps more state live across the solve and spills inside the loop).
// Its result: the coefficients of PairFlow, the evaluations, and the status
// bits of pack_info (0x100 safeguarded, 1 not converged).
struct PairCoef {
    double fm1, gmt, fdot, gdm1;
    int iters;
    unsigned status;
};
SAKURA_HD __attribute__((noinline)) PairCoef kepler_flow(double tau, double mu, double x0,
                                                         double x1, double x2, double w0,
                                                         double w1, double w2, double r0sq,
                                                         const KeplerParams &kp)
{
    NoGuess g;
    const PairFlow f = kepler_flow(tau, mu, x0, x1, x2, w0, w1, w2, r0sq, kp, g);
    return PairCoef{f.fm1, f.gmt, f.fdot, f.gdm1, f.iters,
                    (f.safeguarded ? 0x100u : 0u) | (f.converged ? 0u : 1u)};
}
// The plain flow for the diagnostic kernels: also the relative residual of
// the Kepler equation at the accepted root.
struct NoGuessResid : NoGuess {
    static constexpr bool resid = true;
};
struct PairCoefDiag {
    double fm1, gmt, fdot, gdm1;
    int iters;
    unsigned status;
    double resid;
};
SAKURA_HD __attribute__((noinline)) PairCoefDiag kepler_flow_diag(double tau, double mu,
                                                                  double x0, double x1,
                                                                  double x2, double w0,
                                                                  double w1, double w2,
                                                                  double r0sq,
                                                                  const KeplerParams &kp)
{
    NoGuessResid g;
    const PairFlow f = kepler_flow(tau, mu, x0, x1, x2, w0, w1, w2, r0sq, kp, g);
    return PairCoefDiag{f.fm1, f.gmt, f.fdot, f.gdm1, f.iters,
                        (f.safeguarded ? 0x100u : 0u) | (f.converged ? 0u : 1u), f.resid};
}
// The same with the default parameters built in: three fewer argument
// registers to fill per call, and the tolerance folded into the tests.
SAKURA_HD __attribute__((noinline)) PairCoef kepler_flow_default(double tau, double mu,
                                                                 double x0, double x1,
                                                                 double x2, double w0,
                                                                 double w1, double w2,
                                                                 double r0sq)
{
    constexpr KeplerParams kp{DEFAULT_TOL, DEFAULT_MAX_ITER};
    NoGuess g;
    const PairFlow f = kepler_flow(tau, mu, x0, x1, x2, w0, w1, w2, r0sq, kp, g);
    return PairCoef{f.fm1, f.gmt, f.fdot, f.gdm1, f.iters,
                    (f.safeguarded ? 0x100u : 0u) | (f.converged ? 0u : 1u)};
}

// The whole pair map of eq. (26) with the default parameters, for the split
// of the step's drifts about the Kepler flow into two halves (cb = ca =
// tau/2): the relative state (x, w) after the back-drift cb, the solve, and
// the increments of the relative position and velocity less their starting
// values, per unit mu, d = ((f - 1 - ca fdot) x + (g - tau - ca (gdot - 1)) w,
// fdot x + (gdot - 1) w).  Formed here, the caller keeps nothing live across
// the call (its copies of x and w in the callee-saved registers cost twelve
// register moves per pair).  info as pack_info.  The arithmetic is that of
// the caller's own form of the increments with ca = tau/2, which is exact.
struct PairMap {
    // position and velocity increments interleaved by component: (d0, d3),
    // (d1, d4), (d2, d5), each pair formed from x_c and w_c alone, so that
    // every result can take the return registers of the arguments it used
    double dx0, dv0, dx1, dv1, dx2, dv2;
    unsigned info;
};
SAKURA_HD __attribute__((noinline)) PairMap kepler_map_halves(double tau, double mu, double x0,
                                                              double x1, double x2, double w0,
                                                              double w1, double w2, double r0sq)
{
    constexpr KeplerParams kp{DEFAULT_TOL, DEFAULT_MAX_ITER};
    NoGuess g;
    // -ca = -tau/2 formed first (kept there by the empty statement): tau then
    // ends where the flow takes it, and the flow's time can take its register
    double mca = -0.5 * tau;
    asm volatile("" : "+v"(mca));
    const PairFlow f = kepler_flow(tau, mu, x0, x1, x2, w0, w1, w2, r0sq, kp, g);
    PairMap m;
    m.info = ((unsigned)f.iters << 16) | (f.safeguarded ? 0x100u : 0u) | (f.converged ? 0u : 1u);
    const double a = fma(mca, f.fdot, f.fm1);
    const double b = fma(mca, f.gdm1, f.gmt);
    m.dx0 = fma(a, x0, b * w0);
    m.dv0 = fma(f.fdot, x0, f.gdm1 * w0);
    m.dx1 = fma(a, x1, b * w1);
    m.dv1 = fma_v(f.fdot, x1, f.gdm1 * w1);
    m.dv2 = fma(f.fdot, x2, f.gdm1 * w2);
    m.dx2 = fma_v(a, x2, b * w2);
    return m;
}

// Outcome of one pair's search packed for cheap accumulation: evaluations in
// bits 16-31, a safeguarded step in bit 8, no convergence in bit 0.  Sums of
// up to 64 of them keep the fields apart while every count of evaluations
// stays below 1024 (a limit on KeplerParams::max_iter), and the maximum of
// them carries the largest count of evaluations.
SAKURA_HD inline unsigned pack_info(int iters, bool converged, bool safeguarded)
{
    return ((unsigned)iters << 16) | (safeguarded ? 0x100u : 0u) | (converged ? 0u : 1u);
}

} // namespace kep
