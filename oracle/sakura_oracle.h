/*
 * Sakura CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, fp64 reference of the Keplerian Hamiltonian splitting step
 * (Goncalves Ferrari, Boekholt & Portegies Zwart 2014, Sec. 2).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no source with the HIP library under
 * paper_1402_3325_amd/csrc and must never be used as a compute fallback.
 *
 * All arrays are host memory.  Positions and velocities are [n][3] row-major
 * doubles, masses [n] doubles.  Return codes: 0 ok, <0 error (values below).
 */
#ifndef SAKURA_ORACLE_H
#define SAKURA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SREF_OK          0
#define SREF_EINVAL     -1
#define SREF_ENONFINITE -2
#define SREF_ECOLLIDE   -3
#define SREF_ENOCONV    -4

/* Pair solvers usable inside the eq. (26) map. */
#define SREF_SOLVER_KEPLER        0 /* universal-variable Kepler flow, increments in difference form */
#define SREF_SOLVER_KEPLER_LITERAL 1 /* same flow, increments by the literal subtraction of Listing 1 */
#define SREF_SOLVER_DKD           2 /* drift-kick-drift two-body map of eq. (28) */

/* Stumpff functions c2(z), c3(z) of the universal-variable formulation. */
double sref_stumpff_c2(double z);
double sref_stumpff_c3(double z);

/* Kepler flow of eq. (18): propagate the relative state (x0, w0) of a two-body
 * problem with gravitational parameter mu over time tau.
 * Outputs x1, w1 and coef = {f-1, g-tau, fdot, gdot-1} (Lagrange coefficients
 * written as differences from the free-drift values).  iters may be NULL. */
int sref_kepler(double tau, double mu, const double x0[3], const double w0[3],
                double x1[3], double w1[3], double coef[4], int *iters);

/* Relative increments (dr_ij, dv_ij) of one pair from the second-order pair map
 * of eq. (26): back-drift by tau/2, pair flow over tau, back-drift by tau/2,
 * minus the starting relative state.  ri, vi, rj, vj are the absolute
 * (half-drifted) states. */
int sref_pair_increment(double tau, double G, double mi, double mj,
                        const double ri[3], const double vi[3],
                        const double rj[3], const double vj[3], int solver,
                        double dr[3], double dv[3]);

/* One step Psi(tau) = T(tau/2) W(tau) T(tau/2), eqs. (27a-d), over ordered
 * pairs as in Listing 1.  r and v are updated in place (left unchanged on
 * error). */
int sref_step(int64_t n, const double *m, double *r, double *v, double tau,
              double G, int solver);

/* The state after one step for the listed particles only (r, v unchanged). */
int sref_step_rows(int64_t n, const double *m, const double *r, const double *v,
                   double tau, double G, int64_t nrows, const int64_t *rows,
                   double *r_out, double *v_out);

/* The terms row i of eqs. (27b, 27c) sums: w_ij dr_ij and w_ij dv_ij for every
 * partner j ([n][3] each, zero for j = i and massless pairs). */
int sref_row_terms(int64_t n, const double *m, const double *r, const double *v, double tau,
                   double G, int64_t i, double *dr_terms, double *dv_terms);

/* nsteps calls of sref_step. */
int sref_evolve(int64_t n, const double *m, double *r, double *v, double tau,
                int64_t nsteps, double G, int solver);

/* Compositions of the step over tau (Sec. 2.2).
 *  PSI          eq. (25) with the pair map of eq. (26): sref_step.
 *  UNMERGED     eq. (24) as written: drift tau/2; a W stage over tau/2 whose
 *               pair increments come from eq. (19b) (back-drift, then Kepler
 *               flow); a W stage over tau/2 from eq. (19a) (Kepler flow, then
 *               back-drift); drift tau/2.  Either reading of the operator order
 *               gives this one sequence of maps in time.
 *  TRIPLE_JUMP  the symmetric composition Psi(g1 tau) Psi(g0 tau) Psi(g1 tau)
 *               suggested in Sec. 2.2 for higher order (Yoshida 1990),
 *               g1 = 1 / (2 - 2^(1/3)), g0 = 1 - 2 g1.                        */
#define SREF_SCHEME_PSI         0
#define SREF_SCHEME_UNMERGED    1
#define SREF_SCHEME_TRIPLE_JUMP 2

/* Relative increments of one pair under the map: back-drift the relative
 * position by cb, Kepler flow over t, back-drift by ca (eqs. 17, 18); minus
 * the starting relative state.  eq. (26): (t, cb, ca) = (tau, tau/2, tau/2);
 * eq. (19b): (tau, tau, 0); eq. (19a): (tau, 0, tau). */
int sref_pair_map(double t, double cb, double ca, double G, double mi, double mj,
                  const double ri[3], const double vi[3], const double rj[3],
                  const double vj[3], double dr[3], double dv[3]);

/* One W stage, eq. (23) with the pair map (t, cb, ca) of sref_pair_map and no
 * drifts: r_i += sum_j mu_ij/m_i dr_ij, v_i += sum_j mu_ij/m_i dv_ij.  In
 * place; unchanged on error. */
int sref_w_stage(int64_t n, const double *m, double *r, double *v, double t, double cb,
                 double ca, double G);

/* nsteps steps of the given composition scheme. */
int sref_evolve_scheme(int64_t n, const double *m, double *r, double *v, double tau,
                       int64_t nsteps, double G, int scheme);

/* Close-pair hybrid.  Sec. 1 names applying the Kepler solver only to a few
 * close pairs as a possible optimisation, without a criterion.  A pair is
 * close when the step is not small against its own time scales: with X, W the
 * relative position and velocity after the half drift of eq. (27a), r2 = X.X,
 * w2 = W.W, mu = G (mi + mj),
 *     tau sqrt(mu / r^3) > eta   or   tau |W| / r > eta,
 * evaluated without square roots as
 *     (tau^2 mu)^2 > eta^4 r2^3   or   tau^2 w2 > eta^2 r2,
 * every product rounded in the order written (t2 = tau*tau, e2 = eta*eta,
 * e4 = e2*e2), r2 and w2 formed as fma(x, x, fma(y, y, z*z)).
 * Close pairs take the Kepler map of eq. (26); the others the drift-kick-drift
 * map of eq. (28), whose increments are dr = 0 and dv = tau a_ij in exact
 * arithmetic.  eta > 0. */
int sref_pair_is_close(double tau, double G, double mi, double mj, const double X[3],
                       const double W[3], double eta);

/* One step, eqs. (27a-d), with the hybrid pair maps.  *n_kepler (may be NULL)
 * receives the number of unordered pairs solved by the Kepler map. */
int sref_step_hybrid(int64_t n, const double *m, double *r, double *v, double tau,
                     double G, double eta, int64_t *n_kepler);

/* The hybrid step's state for the listed particles only (r, v unchanged). */
int sref_step_rows_hybrid(int64_t n, const double *m, const double *r, const double *v,
                          double tau, double G, double eta, int64_t nrows,
                          const int64_t *rows, double *r_out, double *v_out);

/* out[12] = {E, K, U, P[3], L[3], Rcm[3]} with long-double accumulation. */
int sref_energy(int64_t n, const double *m, const double *r, const double *v,
                double G, double out[12]);

/* Reference of the learned Kepler starter network (an extension of the
 * method, not in the paper): 8 -> 64 -> 64 -> 1, ReLU, parameters packed as
 * W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 (4801 values).
 * sref_mlp_forward: out[b] for inputs x[b][8].
 * sref_mlp_loss_grad: mean squared error over the batch and its gradient
 * with respect to every parameter (same packing). */
#define SREF_MLP_PARAMS 4801
int sref_mlp_forward(const double *params, int64_t batch, const double *x, double *out);
int sref_mlp_loss_grad(const double *params, int64_t batch, const double *x,
                       const double *y, double *loss, double *grad);

/* Inputs and target of the learned Kepler starter for one pair (an extension
 * of the method, not in the paper).  With t the time after the bound-orbit
 * period reduction, tau' = |t| sqrt(mu/r0^3), e' = sgn(t) x0.w0 / sqrt(mu r0),
 * b' = alpha r0:
 *   feat = {log2 tau', e', b', tau', e' tau', tau'^2 (3 e'^2 - 1 + b') / 6,
 *           tau' max(b',0)^(3/2), e' max(b',0)^(1/2)}.
 * domain = {tau_lo, tau_hi, b_lo, e_hi}: the pair is in the domain when
 * mu > 0, tau_lo <= tau' <= tau_hi, b' >= b_lo and |e'| <= e_hi; only then is
 * *y = log(chi r0 / (sqrt(mu) t)) computed (chi the converged root). */
int sref_guess_sample(double tau, double mu, const double x0[3], const double w0[3],
                      const double domain[4], double feat[8], double *y, int *in_domain);

/* Number of OpenMP threads the row loops use. */
int sref_num_threads(void);

/* Threads of later row loops (n > 0); the results do not depend on it. */
void sref_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
