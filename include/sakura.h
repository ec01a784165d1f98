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
    SAKURA_EINVAL = -1,     /* bad argument: n < 1, dt or G not finite, G < 0, m < 0, bad offsets */
    SAKURA_ENONFINITE = -2, /* NaN/Inf in the input, or produced by a step */
    SAKURA_ECOLLIDE = -3,   /* two particles (after the pair back-drift) at zero separation */
    SAKURA_ENOCONV = -4,    /* a Kepler solve did not converge within max_iter */
    SAKURA_EHIP = -5,       /* a HIP runtime call failed (message in sakura_last_error) */
    SAKURA_ENOMEM = -6,     /* device allocation failed */
    SAKURA_ENOMODEL = -7    /* learned guess requested without a loaded model */
};

enum { SAKURA_GUESS_ANALYTIC = 0, SAKURA_GUESS_LEARNED = 1 };

typedef struct sakura sakura_t;

typedef struct {
    int guess;          /* SAKURA_GUESS_ANALYTIC or SAKURA_GUESS_LEARNED */
    double kepler_rtol; /* relative tolerance on the Kepler root; 0 selects 2^-50 */
    int max_iter;       /* Kepler iterations before ENOCONV; 0 selects 40 */
    int histogram;      /* nonzero: fill sakura_stats.hist (one LDS atomic per pair) */
} sakura_opts;

typedef struct {
    uint64_t pair_solves;  /* Kepler pair solves performed */
    uint64_t iters_total;  /* Kepler iterations summed over those solves */
    uint64_t fallbacks;    /* solves that needed a bisection or bracket-expansion step */
    uint32_t iters_max;    /* largest iteration count of one solve */
    uint32_t hist[32];     /* solves by iteration count (bin 31 holds >= 31); opts.histogram */
    double pair_kernel_ms; /* summed duration of the pair-kernel launches (HIP events) */
    double call_ms;        /* duration of the whole call on the stream (HIP events) */
    int64_t pair_launches; /* number of pair-kernel launches */
    int64_t failed_step;   /* first failing step, -1 if none */
} sakura_stats;

/* Create a handle on HIP device `device`; opts may be NULL (defaults).
 * Returns SAKURA_OK and *h, or an error code and *h = NULL. */
int sakura_create(sakura_t **h, int device, const sakura_opts *opts);

/* Release the handle and all library-owned device memory.  NULL is a no-op. */
void sakura_destroy(sakura_t *h);

/* One step Psi(dt), eqs. (27a-d), over all N(N-1)/2 pairs.
 * n >= 1 particles; G >= 0 the gravitational constant (the paper sets G = 1).
 * stats may be NULL (no counters, no timing). */
int sakura_step(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                double dt, double G, void *stream, sakura_stats *stats);

/* nsteps consecutive steps of sakura_step (fixed dt, Sec. 3), with the state
 * kept in library memory between steps.  nsteps = 0 is a no-op. */
int sakura_evolve(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                  double dt, int64_t nsteps, double G, void *stream,
                  sakura_stats *stats);

/* Batched ensembles: nsys independent systems, each of 1..64 particles, stored
 * back to back (CSR): system s owns particles offsets[s] .. offsets[s+1]-1 of
 * m, r, v.  offsets is a HOST array of nsys + 1 entries with offsets[0] = 0;
 * dt is a DEVICE array of nsys per-system steps.  Every system takes nsteps
 * steps of eqs. (27a-d) inside one persistent kernel (the launch sequence is
 * captured in a hipGraph and replayed while the arguments are unchanged).
 * Systems do not interact.  On any error no system is updated. */
int sakura_batch_evolve(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m,
                        double *r, double *v, const double *dt, int64_t nsteps, double G,
                        void *stream, sakura_stats *stats);

/* Packing of batched systems: policy 0 gives a system of n particles n lanes
 * (dense), 1 rounds n up to even, 2 to a power of two; waves_per_cu sizes the
 * persistent grid; use_graph = 0 launches the kernels directly. */
int sakura_batch_set_policy(sakura_t *h, int policy, int waves_per_cu, int use_graph);

/* Lanes used by systems of exactly n particles (n <= lanes <= 64). */
int sakura_batch_set_group(sakura_t *h, int n, int lanes);

/* Time every packing policy and grid size on this ensemble for probe_steps
 * steps (on scratch copies; r and v are not modified), keep the fastest on the
 * handle and report its time in *best_ms (may be NULL). */
int sakura_autotune_batch(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m,
                          const double *r, const double *v, const double *dt,
                          int64_t probe_steps, double G, void *stream, double *best_ms);

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
