/*
 * sakura.h -- C ABI of the MI355X (gfx950) implementation of the Keplerian
 * Hamiltonian splitting of Goncalves Ferrari, Boekholt & Portegies Zwart (2014).
 *
 * One step is the map Psi(tau) = T(tau/2) W(tau) T(tau/2) of eq. (25), written
 * out as eqs. (27a-d):
 *   (27a)  r_i <- r_i + tau/2 v_i
 *   (27b)  r_i <- r_i + sum_{j != i} (mu_ij / m_i) dr_ij
 *   (27c)  v_i <- v_i + sum_{j != i} (mu_ij / m_i) dv_ij
 *   (27d)  r_i <- r_i + tau/2 v_i
 * where (dr_ij, dv_ij) come from the pair map of eq. (26): a back-drift by
 * tau/2 (eq. 17), the two-body Kepler flow over tau with parameter
 * G (m_i + m_j) (eq. 18), and a second back-drift by tau/2, minus the starting
 * relative state.  Each unordered pair is solved once (Newton's third law,
 * Sec. 2.1): (dr_ji, dv_ji) = -(dr_ij, dv_ij).  The weight mu_ij / m_i is
 * evaluated as m_j / (m_i + m_j), which also defines massless particles.
 *
 * Conventions shared by every entry point:
 *   - m, r, v are DEVICE pointers (hipMalloc'd or torch CUDA tensors), float64,
 *     contiguous: m[n], r[n][3], v[n][3] row-major (the layout of Listing 1).
 *     The caller owns them.  r and v are updated in place.
 *   - stream is a hipStream_t (NULL = the default stream).  Work is ordered on
 *     it; each call returns after that work has completed (one device-to-host
 *     status read per call, not per step).
 *   - On any error the positions and velocities are left exactly as they were
 *     (results are staged in library memory and copied out only on success),
 *     and the stats' failed_step names the first failing step.
 *   - Masses must be >= 0; a pair with m_i + m_j = 0 exerts nothing.  There is
 *     no softening: coincident particles are an error (SAKURA_ECOLLIDE).
 *   - dt may be negative (the pair map is time-symmetric).
 *   - A handle is used by one host thread at a time.
 */
#ifndef SAKURA_H
#define SAKURA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SAKURA_OK = 0,
    SAKURA_EINVAL = -1,     /* bad argument: n < 2, dt not finite, G not finite or G <= 0, m < 0,
                               bad offsets, n beyond what one device's partial sums hold */
    SAKURA_ENONFINITE = -2, /* NaN/Inf in the input, or produced by a step */
    SAKURA_ECOLLIDE = -3,   /* two particles (after the pair back-drift) at zero separation */
    SAKURA_ENOCONV = -4,    /* a Kepler solve did not converge within max_iter */
    SAKURA_EHIP = -5,       /* a HIP runtime call failed (message in sakura_last_error) */
    SAKURA_ENOMEM = -6,     /* device allocation failed */
    SAKURA_ENOMODEL = -7    /* learned guess requested without a loaded model */
};

enum { SAKURA_GUESS_ANALYTIC = 0, SAKURA_GUESS_LEARNED = 1 };

typedef struct sakura sakura_t;

#define SAKURA_MAX_ITER 1000 /* largest accepted sakura_opts.max_iter */

typedef struct {
    int guess;          /* SAKURA_GUESS_ANALYTIC or SAKURA_GUESS_LEARNED */
    double kepler_rtol; /* relative tolerance on the Kepler root; 0 selects 2^-50 */
    int max_iter;       /* Kepler iterations before ENOCONV; 0 selects 40; at most
                           SAKURA_MAX_ITER (sakura_create fails with EINVAL above) */
    int histogram;      /* nonzero: diagnostic pair kernels that fill sakura_stats.hist (one
                           LDS atomic per pair) and max_rel_residual (one more evaluation of
                           the Kepler equation per pair) */
    int tile_override;  /* batched ensembles: 0 packs each system size as the handle's table
                           says (sakura_autotune_batch, sakura_batch_set_policy/_group);
                           L in [1, 64] gives every system of n <= L particles L lanes (a
                           64-lane tile is one wavefront per system).  The single-system
                           pair kernel has one tile, 64 x 64 particles (the wavefront
                           width), and ignores it.  EINVAL outside [0, 64]. */
    int row_strip;      /* single-system pair kernel of the plain starter (Sec. 2.2, the sum
                           over pairs of eq. 23): tiles per work item along a row of the upper
                           triangle of 64 x 64 tiles, whose i-side partial sums are written
                           once per item.  0 picks strips of 4 tiles in the rows before a
                           last triangle of at least two tiles per wavefront slot, whose rows
                           stay single tiles (none where a small system's tiles are split
                           over wavefronts); S = 1, 2, 4, ..., 64 asks for S in every row,
                           with one wavefront per tile (S is capped at the number of
                           64-particle blocks).  The close-pair hybrid, a loaded starter
                           network and the harvest of training rows take one tile per item.
                           The partial sums are stored compactly, one block of 64 x 6 doubles
                           per slot k_apply reads: nb^2 blocks with one tile per item (nb the
                           number of 64-particle blocks), 0.72 nb^2 at nb = 256 by default.
                           The partial sums are added in another grouping for each S, so the
                           results agree to rounding, not bit for bit, across S.  EINVAL
                           for S outside [0, 64] or not a power of two. */
} sakura_opts;

typedef struct {
    uint64_t pair_solves;  /* Kepler pair solves performed */
    uint64_t iters_total;  /* Kepler iterations summed over those solves */
    uint64_t fallbacks;    /* solves that needed a bisection or bracket-expansion step */
    uint32_t iters_max;    /* largest iteration count of one solve */
    uint32_t hist[32];     /* solves by iteration count (bin 31 holds >= 31); opts.histogram */
    double pair_kernel_ms; /* summed duration of the pair-kernel launches (HIP events; a
                              call holds at most 256 launches' events: each pair is read
                              back, waiting for its launch, before it is reused) */
    double call_ms;        /* duration of the whole call on the stream (HIP events) */
    int64_t pair_launches; /* number of pair-kernel launches */
    int64_t failed_step;   /* first failing step, -1 if none */
    /* Learned starter (zero unless a model is loaded or a harvest is running): */
    uint64_t guess_domain_pairs; /* solves whose pair lies in the network's domain */
    uint64_t guess_domain_iters; /* Kepler evaluations of those solves */
    uint64_t guess_learned;      /* solves started from the network's value */
    uint64_t guess_restarts;     /* of those, searches restarted from the plain starter */
    /* Close-pair hybrid (zero unless sakura_set_hybrid is on): */
    uint64_t pair_kicks; /* pairs given the eq. (28) kick instead of a Kepler solve */
    /* Largest relative residual |t(s) - t| / |t| of the Kepler equation at the accepted
     * roots (t the flight time after the bound-orbit period reduction, t(s) evaluated
     * once more at the root in FP64, stored in single precision).  Filled for every
     * solve of the single-system paths when opts.histogram is set (except during a
     * harvest), and for the pairs the learned starter solves in any mode; 0 otherwise
     * (and for batched ensembles). */
    double max_rel_residual;
} sakura_stats;

/* Create a handle on HIP device `device`; opts may be NULL (defaults).
 * Returns SAKURA_OK and *h, or an error code and *h = NULL. */
int sakura_create(sakura_t **h, int device, const sakura_opts *opts);

/* Release the handle and all library-owned device memory.  NULL is a no-op. */
void sakura_destroy(sakura_t *h);

/* One step Psi(dt), eqs. (27a-d), over all N(N-1)/2 pairs.
 * n >= 2 particles; G > 0 the gravitational constant (the paper sets G = 1).
 * The library keeps 0.75 n^2 bytes of partial sums (a block of 6 x 64 doubles
 * for each side of each 64 x 64 tile, n rounded up to a multiple of 64); n
 * whose partial sums exceed the device's memory is EINVAL, and ENOMEM is
 * returned when an allocation fails.  stats may be NULL (no counters, no timing). */
int sakura_step(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                double dt, double G, void *stream, sakura_stats *stats);

/* nsteps consecutive steps of sakura_step (fixed dt, Sec. 3), with the state
 * kept in library memory between steps.  nsteps = 0 is a no-op. */
int sakura_evolve(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                  double dt, int64_t nsteps, double G, void *stream,
                  sakura_stats *stats);

/* Allocation-free variant of sakura_evolve, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It runs the same kernels on a static device array of
 * the library (12.4 MB: state, partial sums and counters for up to
 * SAKURA_NOALLOC_MAX_N particles) instead of handle-owned buffers, and calls
 * no allocating routine.  Each device the library runs on holds one copy of
 * that array until the process ends; every call on a device shares it and it
 * keeps the last call's contents (the kernels clear what must start at zero),
 * so calls that overlap on one device -- from several threads, handles or
 * streams -- race, and the caller must serialise them.  Runs the merged step
 * (eq. 25) with the plain starter, or the close-pair hybrid when it is on;
 * stats get the counters but no timings.  Arguments, ownership and errors as
 * sakura_evolve; EINVAL also for n > SAKURA_NOALLOC_MAX_N, the learned
 * starter and a running harvest. */
#define SAKURA_NOALLOC_MAX_N 4096
int sakura_evolve_noalloc(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                          double dt, int64_t nsteps, double G, void *stream,
                          sakura_stats *stats);

/* Compositions of the step (Sec. 2.2).  A W stage applies eqs. (27b, 27c)
 * with a pair map made of a back-drift cb of the relative position, the Kepler
 * flow over t and a back-drift ca (t = cb + ca); stages are separated by free
 * drifts of every particle.  One step over dt is:
 *   SAKURA_SCHEME_PSI          eq. (25) with the pair map of eq. (26): drift
 *                              dt/2, stage (dt; dt/2, dt/2), drift dt/2
 *                              (= sakura_evolve).
 *   SAKURA_SCHEME_UNMERGED     eq. (24): drift dt/2, stage (dt/2; dt/2, 0)
 *                              (pairs by eq. 19b), stage (dt/2; 0, dt/2) (pairs
 *                              by eq. 19a), drift dt/2.  Two pair launches.
 *   SAKURA_SCHEME_TRIPLE_JUMP  Psi(g1 dt) Psi(g0 dt) Psi(g1 dt),
 *                              g1 = 1/(2 - 2^(1/3)), g0 = 1 - 2 g1 < 0 (the
 *                              higher-order composition the paper proposes,
 *                              after Yoshida 1990).  Three pair launches.
 * In exact arithmetic the unmerged step over dt equals two merged steps over
 * dt/2 (a drift moves through a stage by shifting its back-drifts), and since
 * the merged step is time-symmetric only up to a fourth-order defect for
 * N > 2, the triple jump is third order, not fourth.
 * stats count every pair launch (pair_launches = nsteps x stages) and
 * failed_step names the step, not the stage.  Other arguments, errors and
 * ownership as sakura_evolve; an unknown scheme is SAKURA_EINVAL. */
enum { SAKURA_SCHEME_PSI = 0, SAKURA_SCHEME_UNMERGED = 1, SAKURA_SCHEME_TRIPLE_JUMP = 2 };

int sakura_evolve_scheme(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                         double dt, int64_t nsteps, double G, int scheme, void *stream,
                         sakura_stats *stats);

/* Close-pair hybrid.  Sec. 1 names applying the Kepler solver only to a few
 * close pairs as a possible optimisation; the criterion is this library's.
 * With eta > 0, the merged step (sakura_step, sakura_evolve,
 * sakura_evolve_scheme with SAKURA_SCHEME_PSI) solves a pair by the Kepler map
 * of eq. (26) only when the step is not small against the pair's own time
 * scales,
 *     tau sqrt(mu / r^3) > eta   or   tau |W| / r > eta,
 * with X, W the relative position and velocity after the half drift of
 * eq. (27a), r = |X|, mu = G (m_i + m_j); evaluated without square roots as
 * (tau^2 mu)^2 > eta^4 r^6 or tau^2 |W|^2 > eta^2 r^2, every product rounded
 * in that order and |X|^2, |W|^2 formed as fma(x, x, fma(y, y, z*z)).  Every
 * other pair takes the drift-kick-drift map of eq. (28), whose increments are
 * dr = 0 and dv = tau a_ij, a_ij = -mu X / r^3.  The step stays second order
 * for any fixed eta; eta = 0 (the default) solves every pair by Kepler.
 * stats: pair_solves counts the Kepler pairs, pair_kicks the kicked ones.
 * While eta > 0, the learned starter, harvests and the other composition
 * schemes are SAKURA_EINVAL.  EINVAL for eta < 0 or not finite. */
int sakura_set_hybrid(sakura_t *h, double eta);

/* Batched ensembles: nsys independent systems, each of 1..64 particles, stored
 * back to back (CSR): system s owns particles offsets[s] .. offsets[s+1]-1 of
 * m, r, v.  offsets is a HOST array of nsys + 1 entries with offsets[0] = 0;
 * dt is a DEVICE array of nsys per-system steps.  Every system takes nsteps
 * steps of eqs. (27a-d) inside one persistent kernel (the launch sequence is
 * captured in a hipGraph and replayed while the pointers, the counts of
 * systems, particles, steps and work items and the solver settings are
 * unchanged; any other call captures it again).  Systems do not interact.
 * On any error no system is updated. */
int sakura_batch_evolve(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m,
                        double *r, double *v, const double *dt, int64_t nsteps, double G,
                        void *stream, sakura_stats *stats);

/* Packing of batched systems: policy 0 gives a system of n particles n lanes
 * (dense), 1 rounds n up to even, 2 to a power of two; waves_per_cu sizes the
 * persistent grid; use_graph = 0 launches the kernels directly (the three
 * launch widths on three streams).  Resets the wavefronts per item to their
 * default (sakura_batch_set_width).  A new handle packs with policy 0, 16
 * wavefronts per compute unit and the graph. */
int sakura_batch_set_policy(sakura_t *h, int policy, int waves_per_cu, int use_graph);

/* Lanes used by systems of exactly n particles (n <= lanes <= 64). */
int sakura_batch_set_group(sakura_t *h, int n, int lanes);

/* Wavefronts per work item (1, 2 or 4) for systems of exactly n particles:
 * the wavefronts of an item hold the same systems and take every first,
 * second or fourth sub-step of the pair schedule, which shortens the item's
 * sequential chain.  The default (also after sakura_batch_set_policy) is 4.
 * EINVAL for n outside [1, 64] or another count. */
int sakura_batch_set_width(sakura_t *h, int n, int waves);

/* Tune the packing on this ensemble (scratch copies; r and v are not
 * modified): the grid size (4, 8 or 16 wavefronts per compute unit), then for
 * each size bucket the ensemble has systems in (1-8, 9-16, 17-32, 33-64
 * particles) the lane policy of sakura_batch_set_policy and then the
 * wavefronts per item (1, 2 or 4), one coordinate at a time.  Each probe runs
 * probe_steps steps with direct launches (no graph; the three launch widths
 * side by side on three streams, as in the graph) and takes the least of two
 * timed calls after a warm-up call.  The best settings stay on the handle and are recorded in
 * its packing table under (gfx architecture, compute units, bucket); the
 * least probe time goes to *best_ms (may be NULL).  If a probe fails, its
 * error is returned and the handle keeps the settings it had. */
int sakura_autotune_batch(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m,
                          const double *r, const double *v, const double *dt,
                          int64_t probe_steps, double G, void *stream, double *best_ms);

/* The packing table as a text file (one line per entry: arch, compute units,
 * bucket 0-3, policy 0-2, wavefronts per compute unit, wavefronts per item
 * 1/2/4; '#' lines are comments).  Load merges the file's entries into the handle's table and
 * applies those of the handle's device; EINVAL for an unreadable or malformed
 * file (the table is then unchanged). */
int sakura_batch_table_save(const sakura_t *h, const char *path);
int sakura_batch_table_load(sakura_t *h, const char *path);

/* ---------------------------------------------------------------------------
 * Learned Kepler starter (an extension of the method; the paper's solver
 * needs only some starting value of the universal variable).
 *
 * A pair's Kepler problem over time t (after the bound-orbit period
 * reduction) is fixed, up to scale, by tau' = |t| sqrt(mu/r0^3),
 * e' = sgn(t) x0.w0 / sqrt(mu r0) and b' = 2 - r0 |w0|^2 / mu.  Pairs with
 *   domain[0] <= tau' <= domain[1],  b' >= domain[2],  |e'| <= domain[3]
 * (and mu > 0) are in the network's domain.  The network 8 -> 64 -> 64 -> 1
 * (ReLU) maps the inputs
 *   f = {log2 tau', e', b', tau', e' tau', tau'^2 (3 e'^2 - 1 + b') / 6,
 *        tau' max(b',0)^(3/2), e' max(b',0)^(1/2)},
 * each as (f[k] - in_shift[k]) * in_scale[k], to y = out_shift + out_scale *
 * output, and the starter is s = (t / r0) exp(y) in the regularised time
 * (dt/ds = r); y approximates log(s r0 / t) at the root.  Inference is fused
 * into the pair kernels on MFMA with bf16 weights and activations and fp32
 * accumulation, only for wavefronts holding a pair in the domain.  The root
 * search that follows is the plain one (same stopping rule, same results to
 * the solver tolerance); a search that fails to converge from the network's
 * value is restarted from the plain starter.
 * ------------------------------------------------------------------------- */

#define SAKURA_MLP_PARAMS 4801 /* W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 */
#define SAKURA_HARVEST_ROW 12  /* floats per harvest row */

typedef struct {
    float params[SAKURA_MLP_PARAMS]; /* fp32, packed as listed above (row-major W[out][in]) */
    float in_shift[8], in_scale[8];
    float out_shift, out_scale;
    double domain[4];                /* tau_lo, tau_hi, b_lo, e_hi */
} sakura_guess_model;

/* Load or, with blob = NULL, unload the network.  blob is a HOST pointer to
 * one sakura_guess_model, whose size bytes must equal; the library copies it
 * and derives the bf16 inference fragments on the device from it.  While a model is loaded, plain-starter runs also count
 * the solves in its domain (sakura_stats.guess_domain_*).  EINVAL for a wrong
 * size, non-finite values or an empty domain. */
int sakura_set_guess_model(sakura_t *h, const void *blob, size_t bytes);

/* Starter of later calls: SAKURA_GUESS_ANALYTIC or SAKURA_GUESS_LEARNED (the
 * latter makes steps fail with ENOMODEL while no model is loaded). */
int sakura_set_guess(sakura_t *h, int guess);

/* Harvest: until sakura_harvest_end, every step (sakura_step, sakura_evolve,
 * sakura_batch_evolve) uses the plain starter and appends, for every solved
 * pair in `domain` (HOST, 4 doubles as above), one row of SAKURA_HARVEST_ROW
 * floats to `rows` (DEVICE, cap rows): the eight raw inputs f, the target
 * y = log(s r0 / t) at the converged root, then the particle indices i and j
 * and the number of Kepler evaluations, those three as int32 bit patterns.
 * Row order is unspecified.  Rows beyond cap are dropped (but counted). */
int sakura_harvest_begin(sakura_t *h, float *rows, int64_t cap, const double domain[4]);

/* End the harvest; *offered (HOST, may be NULL) = rows produced, including
 * those dropped beyond cap. */
int sakura_harvest_end(sakura_t *h, int64_t *offered);

/* The Kepler root search of the pair kernels on n independent problems
 * (DEVICE arrays): propagate (x0[k], w0[k]) ([n][3]) with parameter mu[k] over
 * tau[k], with the handle's starter.  Outputs (DEVICE, [n]): s_start the
 * starting value, s_root the converged root (regularised time s of t(s)),
 * info bit 0 in the domain, bit 1 network starter used, bit 2 restarted,
 * bit 3 converged, bits 8-15 Kepler evaluations.  |x0[k]| must be > 0. */
int sakura_guess_eval(sakura_t *h, int64_t n, const double *tau, const double *mu,
                      const double *x0, const double *w0, double *s_start, double *s_root,
                      int32_t *info, void *stream);

/* Network training kernels (fp32; DEVICE pointers unless noted).
 * sakura_mlp_forward: out[b] = network output for inputs x[b][8] (already
 *   shifted and scaled), parameters params[SAKURA_MLP_PARAMS].
 * sakura_mlp_loss_grad: mean over the batch of (output - y)^2 in *loss (HOST)
 *   and its gradient in grad[SAKURA_MLP_PARAMS] (same packing as params);
 *   the per-parameter sums are taken in a fixed order (deterministic). */
int sakura_mlp_forward(sakura_t *h, const float *params, int64_t batch, const float *x,
                       float *out, void *stream);
int sakura_mlp_loss_grad(sakura_t *h, const float *params, int64_t batch, const float *x,
                         const float *y, float *grad, double *loss, void *stream);

typedef struct {
    int epochs;          /* passes over the training rows; 0 selects 20 */
    int batch;           /* minibatch size; 0 selects 4096 */
    float lr, lr_final;  /* Adam step size, cosine-annealed from lr to lr_final; 0 selects 3e-3, 3e-5 */
    uint64_t seed;       /* initial weights and minibatch sampling */
    double val_fraction; /* trailing fraction of the rows held out; 0 selects 0.05 */
} sakura_fit_opts;

/* Train the starter network on n harvested rows (DEVICE, SAKURA_HARVEST_ROW
 * floats each) with the kernels above and Adam.  Input and output scaling
 * come from the training rows' means and standard deviations.  Fills *model
 * (HOST) including `domain` (HOST, 4 doubles); val_loss (HOST, epochs floats,
 * may be NULL) receives the held-out mean squared error of the scaled target
 * after each epoch.  n >= 64 rows. */
int sakura_mlp_fit(sakura_t *h, const float *rows, int64_t n, const double domain[4],
                   const sakura_fit_opts *opts, sakura_guess_model *model, float *val_loss,
                   void *stream);

/* Energy diagnostics of eqs. (1-3) with compensated sums:
 * out[12] (HOST) = {E, K, U, P[3], L[3], Rcm[3]}: total, kinetic and potential
 * energy, linear and angular momentum, centre of mass. */
int sakura_energy(sakura_t *h, int64_t n, const double *m, const double *r,
                  const double *v, double G, double out[12], void *stream);

/* Message for the last error on this handle ("" if none).  Owned by the handle. */
const char *sakura_last_error(const sakura_t *h);

#ifdef __cplusplus
}
#endif
#endif
