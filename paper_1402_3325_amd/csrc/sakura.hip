// Sakura step on MI355X (gfx950): kernels and the C ABI of include/sakura.h.
//
// Data layout in HBM (library-owned, per handle):
//   state[10][np] float64 structure-of-arrays, np = 64 * ceil(n / 64):
//     row 0 m, rows 1-3 r (after the step), rows 4-6 v, rows 7-9 r half-drifted
//   partial sums, float64 blocks [6][64]: slot k of block K holds, for
//     component c (dr xyz, dv xyz) and particle 64 K + l, the sum of the
//     weighted increments it receives from one tile's or one row strip's pairs
//     (tiles.hpp: slots k < K the j sides of tiles (k, K), then the i sides of
//     row K's work items); block K's slots follow one another from
//     apply_offset(K), nb^2 slots with one tile per work item.
// Per step: k_pairs (eqs. 26, 23 over all unordered pairs) then k_apply
// (eqs. 27b-d and the next step's 27a); a composition of the step (Sec. 2.2)
// runs one such pair of launches per stage.  k_import / k_export convert
// between the caller's [n][3] arrays and the internal layout once per call.
#include "common.hpp"
#include "tiles.hpp"

#include <algorithm>
#include <mutex>

__global__ void sk::k_clear(DevCounters *c, SlotStats *slots)
{
    const int t = threadIdx.x; // NSLOT threads
    slots[t].pair_solves = 0;
    slots[t].iters_total = 0;
    slots[t].fallbacks = 0;
    slots[t].iters_max = 0;
    slots[t].learned = 0;
    slots[t].restarts = 0;
    slots[t].dom_pairs = 0;
    slots[t].dom_iters = 0;
    slots[t].kicks = 0;
    slots[t].resid_bits = 0;
    if (t == 0) {
        c->status = 0;
        c->iters_max = 0;
        c->pair_solves = 0;
        c->iters_total = 0;
        c->fallbacks = 0;
        c->failed_step = LLONG_MAX;
        c->work_next = 0;
        c->work_next2 = 0;
        c->work_next4 = 0;
        c->dom_pairs = 0;
        c->dom_iters = 0;
        c->learned = 0;
        c->restarts = 0;
        c->defer_ntiles = 0;
        c->defer_next = 0;
        c->kicks = 0;
        c->resid_bits = 0;
    }
    if (t < 32) c->hist[t] = 0;
}

namespace {
// Sum (or maximum) over the NSLOT threads of one workgroup, fixed order.
__device__ unsigned long long fold_slots(unsigned long long *a, unsigned long long x, bool is_max)
{
    const int t = threadIdx.x;
    __syncthreads();
    a[t] = x;
    __syncthreads();
    for (int w = sk::NSLOT / 2; w > 0; w >>= 1) {
        if (t < w) a[t] = is_max ? max(a[t], a[t + w]) : a[t] + a[t + w];
        __syncthreads();
    }
    return a[0];
}
} // namespace

// Sum of the counter slots (one workgroup of NSLOT threads).
__global__ void sk::k_fold_stats(const SlotStats *slots, DevCounters *c)
{
    __shared__ unsigned long long a[NSLOT];
    const int t = threadIdx.x;
    const SlotStats sl = slots[t];
    const unsigned long long solves = fold_slots(a, sl.pair_solves, false);
    const unsigned long long iters = fold_slots(a, sl.iters_total, false);
    const unsigned long long fb = fold_slots(a, sl.fallbacks, false);
    const unsigned long long mx = fold_slots(a, sl.iters_max, true);
    const unsigned long long dom = fold_slots(a, sl.dom_pairs, false);
    const unsigned long long dit = fold_slots(a, sl.dom_iters, false);
    const unsigned long long lrn = fold_slots(a, sl.learned, false);
    const unsigned long long rst = fold_slots(a, sl.restarts, false);
    const unsigned long long kick = fold_slots(a, sl.kicks, false);
    const unsigned long long rb = fold_slots(a, sl.resid_bits, true);
    if (t == 0) {
        c->pair_solves = solves;
        c->iters_total = iters;
        c->fallbacks = fb;
        c->iters_max = (unsigned)mx;
        c->dom_pairs = dom;
        c->dom_iters = dit;
        c->learned = lrn;
        c->restarts = rst;
        c->kicks = kick;
        c->resid_bits = (unsigned)rb;
    }
}

namespace {
using namespace sk;

// Caller layout -> SoA, with the half drift of eq. (27a) into the row r_half.
__global__ void k_import(int n, int np, const double *__restrict__ m,
                         const double *__restrict__ r, const double *__restrict__ v,
                         double h, double *__restrict__ S, DevCounters *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double mi = 0.0, p[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        mi = m[i];
        for (int c = 0; c < 3; ++c) {
            p[c] = r[3 * i + c];
            q[c] = v[3 * i + c];
        }
        bool fin = isfinite(mi);
        for (int c = 0; c < 3; ++c) fin = fin && isfinite(p[c]) && isfinite(q[c]);
        if (!fin) record_error(cnt, ST_NONFINITE, 0);
        else if (!(mi >= 0.0)) record_error(cnt, ST_INVAL, 0);
    }
    S[i] = mi;
    for (int c = 0; c < 3; ++c) {
        S[(1 + c) * (size_t)np + i] = p[c];
        S[(4 + c) * (size_t)np + i] = q[c];
        S[(7 + c) * (size_t)np + i] = p[c] + h * q[c];
    }
}

// The plain solve of one pair: with HIST the diagnostic copy that also
// evaluates the Kepler equation once more at the root (relative residual);
// otherwise the copy with the default parameters built in (DEFKP) or the
// general one (resid 0).
template <bool HIST, bool DEFKP>
__device__ __forceinline__ kep::PairCoefDiag solve_pair(double t, double mu, double x0, double x1,
                                                        double x2, double w0, double w1,
                                                        double w2, double r0sq,
                                                        const kep::KeplerParams &kp)
{
    if constexpr (HIST) {
        return kep::kepler_flow_diag(t, mu, x0, x1, x2, w0, w1, w2, r0sq, kp);
    } else {
        const kep::PairCoef c =
            DEFKP ? kep::kepler_flow_default(t, mu, x0, x1, x2, w0, w1, w2, r0sq)
                  : kep::kepler_flow(t, mu, x0, x1, x2, w0, w1, w2, r0sq, kp);
        return kep::PairCoefDiag{c.fm1, c.gmt, c.fdot, c.gdm1, c.iters, c.status, 0.0};
    }
}

// Close-pair test of the hybrid step: the step is not small against the pair's
// own time scales, t sqrt(mu / r^3) > eta or t |W| / r > eta, evaluated without
// square roots as (t^2 mu)^2 > eta^4 r2^3 or t^2 w2 > eta^2 r2, with r2 and w2
// formed as fma(x, x, fma(y, y, z z)) and every product rounded in the order
// written, so the decision is a fixed function of X, W, t, mu and eta.
__device__ inline bool hybrid_close(double t2, double mu, double r2, double w2, double e2,
                                    double e4)
{
    const double A = t2 * mu;
    return (A * A > e4 * ((r2 * r2) * r2)) | (t2 * w2 > e2 * r2);
}

// All unordered pairs of one 64 x 64 tile (I, J), I <= J, by one wavefront;
// in the plain kernels of one wavefront per tile a work item may be a strip of
// tiles (I, J0), ..., (I, J0 + len - 1) along a row (tiles.hpp), taken one
// after the other with block I's particles and i-side sums kept.
//
// Lane l holds particle i = 64 I + l and its i-side sums in registers; block
// J sits in LDS.  In sub-step s lane l takes the pair
// (i, 64 J + ((l + s) mod 64)), so within a sub-step every lane touches a
// different j, and the j-side sums (Newton's third law) are added in LDS, one
// slot per j, with no atomics and no barrier: the wavefront's LDS operations
// complete in order, so a sub-step reads what the previous one wrote.  (Kept
// in registers and rotated by one lane per sub-step instead, they cost twelve
// DPP moves per pair on the vector ALU, which bounds this kernel.)  The
// diagonal tile runs s = 1..32 (s = 32 on half the lanes), which visits each
// pair i < j once.  Partial sums go to slot I of block J (j side) and to
// the work item's slot of block I (i side).
// The pair map is the back-drift cb of the relative position, the Kepler flow
// over tau and the back-drift ca (eq. 26: cb = ca = tau/2; eq. 19b: cb = tau,
// ca = 0; eq. 19a: cb = 0, ca = tau), with tau = cb + ca, which every
// composition of the step satisfies exactly; the increments below are written
// for that case.
// MODE selects the starter: 0 plain; with a loaded network 1 plain with
// domain statistics, 3 plain with harvest rows, 4 pairs that may lie in the
// network's domain listed for k_deferred (which starts those in the domain
// from the network) and the rest solved plainly.  MODE 5 is the close-pair
// hybrid: close pairs (hybrid_close, thresholds e2 = eta^2, e4 = eta^4) take
// the plain Kepler solve, the others the drift-kick-drift map of eq. (28),
// dr = 0 and dv = tau a_ij, and the solve runs only in sub-steps where some
// lane of the wavefront has a close pair.
// DEFKP: the solver copy with the default parameters built in; HALVES (with
// DEFKP, modes 0 and 4, cb = ca = tau/2): the copy that also forms the
// increments (kepler_map_halves), so that nothing stays live across the call.
// SPLIT (every mode but 4, whose deferred-pair list belongs to one
// wavefront): a workgroup of SPLIT wavefronts per
// tile, all holding block I, wavefront w taking the sub-steps s = s0 + w,
// s0 + w + SPLIT, ... with j-side slots of its own; at the end the
// wavefronts' i-side and j-side sums are added in wavefront order.  For small
// N, where the tiles alone would leave most of the SIMDs' wave slots empty.
template <bool B> struct BoolTag {
    static constexpr bool value = B;
};

template <bool HIST, int MODE, bool DEFKP = false, bool HALVES = false, int SPLIT = 1>
__global__ __launch_bounds__(TILE * SPLIT, 4) void k_pairs(int n, int nb, int np,
                                                StripLayout strips, double tau,
                                                double cb, double ca, double G,
                                                double e2, double e4,
                                                const double *__restrict__ S,
                                                double *__restrict__ part,
                                                DevCounters *cnt, SlotStats *slots,
                                                kep::KeplerParams kp, long long step,
                                                const kep::GuessNet net)
{
    // an earlier failure: the call will report it (with SPLIT the workgroup
    // takes one decision, as other workgroups may record a failure meanwhile)
    if constexpr (SPLIT == 1) {
        if (cnt->status) return;
    } else {
        __shared__ unsigned s_stop;
        if (threadIdx.x == 0) s_stop = cnt->status;
        __syncthreads();
        if (s_stop) return;
    }
    // the work item: tiles (I, J0), ..., (I, J0 + len - 1).  Strips of several
    // tiles are built into the plain modes' kernels of one wavefront per tile
    // only: with SPLIT > 1 the wavefronts combine their i-side sums in LDS per
    // tile, mode 4's deferred-pair list belongs to one tile, and the loop over
    // a strip's tiles costs the other modes' kernels, which hold more state,
    // registers they do not have (the hybrid's spilled).
    constexpr bool STRIPS = SPLIT == 1 && MODE == 0;
    const StripLayout lay = STRIPS ? strips : StripLayout{1, 0}; // of the partial sums
    int I, J0, len = 1;
    if constexpr (STRIPS) {
        layout_item(blockIdx.x, nb, strips, I, J0, len);
        // uniform: the decoding's divisions and square root run on the vector
        // ALU, and values left there would keep the sub-step counter there too
        I = __builtin_amdgcn_readfirstlane(I);
        J0 = __builtin_amdgcn_readfirstlane(J0);
        len = __builtin_amdgcn_readfirstlane(len);
    } else {
        tile_blocks(blockIdx.x, nb, I, J0);
    }
    static_assert(SPLIT == 1 || MODE != 4, "the deferred-pair list is one wavefront's");
    const int lane = SPLIT == 1 ? (int)threadIdx.x : (int)threadIdx.x % TILE;
    const int wv = SPLIT == 1 ? 0 : (int)threadIdx.x / TILE;

    const double *M = S;
    const double *V = S + 4 * (size_t)np;
    const double *XH = S + 7 * (size_t)np;

    __shared__ double sj[7][TILE];          // x y z vx vy vz G m of block J (read only)
    __shared__ double sjs[SPLIT][6][TILE];  // j-side sums, by wavefront and slot of block J
    // i-side sums of wavefronts 1.. (SPLIT > 1); with SPLIT 1 the i-side sums of
    // a strip's earlier tiles, each lane its own slots
    __shared__ double sacc[SPLIT > 1 ? SPLIT - 1 : 1][6][TILE];
    __shared__ unsigned shist[HIST ? 32 : 1];

    const int ig = I * TILE + lane;
    // particle i and its sums stay in registers.  The masses are held as G m:
    // mu = G m_i + G m_j (G (m_i + m_j) up to its rounding, equal for G = 1)
    // and the weights G m_j, G m_i of the increments per unit mu are read as
    // they are.
    const double xi[7] = {XH[ig], XH[np + ig], XH[2 * (size_t)np + ig], V[ig], V[np + ig],
                          V[2 * (size_t)np + ig], G * M[ig]};
    if (HIST && wv == 0 && lane < 32) shist[lane] = 0;

    const bool valid_i = ig < n;
    const double wgt_j = xi[6];
    const double q4 = MODE == 4 ? kep::may_qualify_scale(net, tau) : 0.0;
    const double t2 = tau * tau, mtau = -tau; // MODE 5
    const int lane8 = 8 * lane;

    // Every lane solves a pair in every sub-step (lanes without one solve
    // tau = 0: one evaluation, converged, never safeguarded), so the outcomes
    // are summed over all lanes and the trivial ones taken off at the end.
    unsigned info_sum = 0, info_max = 0; // per lane: sum and maximum of kep::pack_info
    unsigned long long n_solve = 0;      // per wave: pairs solved (ballot counts)
    unsigned long long n_kick = 0;       // per wave, MODE 5
    GuessCount gc;                       // per wave
    unsigned dom_it = 0;                 // per lane
    int room = kep::DEFER_CAP;           // MODE 4: list slots left
    unsigned long long coll_bits = 0;    // per wave: lanes that met a zero separation
    bool coll_lane = false;              // HALVES: per lane, a zero separation met
    float rmax = 0.0f;                   // per lane, HIST: largest relative Kepler residual
    int nsub_w = 0;                      // sub-steps this wavefront took, over the item
    // tau held in a vector register, where the selection of the time passed to
    // the solver reads it (from a scalar register it is moved there first, two
    // more vector operations per pair)
    double tau_v = tau;
    asm volatile("" : "+v"(tau_v));

    // the partial-sum slots (tiles.hpp; fewer than 2^31): the item's i side in
    // block I, and the first slot of the current tile's block J
    const int slot_i = (int)(apply_offset(I, nb, lay) + item_slot(I, J0, nb, lay));
    int slot_j = (int)apply_offset(J0, nb, lay);
    for (int J = J0; J < J0 + len; ++J) {
        const bool diag = (I == J);
        const int jg = J * TILE + lane;
        if (J != J0) __syncthreads(); // the previous tile's reads of sj and sjs are done
        if (wv == 0) {
            sj[0][lane] = XH[jg];
            sj[1][lane] = XH[np + jg];
            sj[2][lane] = XH[2 * (size_t)np + jg];
            sj[3][lane] = V[jg];
            sj[4][lane] = V[np + jg];
            sj[5][lane] = V[2 * (size_t)np + jg];
            sj[6][lane] = G * M[jg];
        }
        double ai[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 6; ++c) sjs[wv][c][lane] = 0.0;
        const int nj = n - J * TILE; // valid j slots in this block
        const int nj8 = 8 * nj;
        __syncthreads();

        const int s0 = diag ? 1 : 0, s1 = diag ? (TILE / 2 + 1) : TILE;
        // The sub-step loop in two copies: FULL for tiles whose 64 i and 64 j
        // slots all hold particles of positive mass (every tile but those of the
        // last block, in a system without massless particles), which need no test
        // of the slots or of mu > 0.
        const bool full_tile = (I + 1) * TILE <= n && (J + 1) * TILE <= n &&
                               __all(xi[6] > 0.0 && sj[6][lane] > 0.0);
        auto sweep = [&](auto full_tag) __attribute__((always_inline)) {
        constexpr bool FULL = decltype(full_tag)::value;
        int p8 = lane8 + 8 * (s0 + wv); // lane8 + 8 s, stepped with s
        for (int s = s0 + wv; s < s1; s += SPLIT, p8 += 8 * SPLIT) {
            // q scaled by 8 (the byte offset of slot q in a row of doubles) is
            // formed and tested directly: one vector operation less than q itself.
            // p8 is kept opaque, so that q8 stays one mask of it (left to itself
            // the compiler forms ((lane + s) & 63) << 3 where q8 is not tested).
            asm volatile("" : "+v"(p8));
            const int q8 = p8 & (8 * (TILE - 1));
            const int q = q8 >> 3;
            // slot q of a row of block J and of this wavefront's j-side sums, by
            // its byte offset (indexing by q has the compiler form q, then q8 again)
#define SJ(c) (*(const double *)((const char *)sj[c] + q8))
#define SJS(c) (*(double *)((char *)sjs[wv][c] + q8))
            // In harvest mode the particle data are read from LDS at every use and
            // the relative state is formed again after the solve (compiler-only
            // fences): its inlined policy's extra live state would otherwise push
            // the loop past 128 VGPRs.  The other modes keep it.
            if (MODE == 3) asm volatile("" ::: "memory");
            const double gmj = SJ(6);
            const double mu = xi[6] + gmj;
            const bool act = (FULL || (valid_i && (q8 < nj8) && (mu > 0.0))) &&
                             !(diag && s == TILE / 2 && lane >= TILE / 2);
            if constexpr (MODE == 5) {
                const double X0 = xi[0] - SJ(0), X1 = xi[1] - SJ(1), X2 = xi[2] - SJ(2);
                const double w0 = xi[3] - SJ(3), w1 = xi[4] - SJ(4), w2 = xi[5] - SJ(5);
                const double r2 = fma(X0, X0, fma(X1, X1, X2 * X2));
                const double ws = fma(w0, w0, fma(w1, w1, w2 * w2));
                const bool close = act & hybrid_close(t2, mu, r2, ws, e2, e4);
                // eq. (28): the relative velocity changes by tau a_ij at X and the
                // position increment vanishes; per unit mu, dv = -tau X / r^3
                const bool kick = act & !close & (r2 > 0.0);
                bool collide = act & !close & !(r2 > 0.0);
                const double rinv = kep::rsqrt_refined(r2); // used only where kick holds
                const double kf = kick ? mtau * (rinv * rinv * rinv) : 0.0;
                const double wgt_i = gmj;
                if (!__builtin_amdgcn_ballot_w64(close)) {
                    // no close pair in this sub-step: velocity sums only, weights
                    // folded into the kick
                    const double ki = wgt_i * kf, kj = -wgt_j * kf;
                    ai[3] = fma(ki, X0, ai[3]);
                    ai[4] = fma(ki, X1, ai[4]);
                    ai[5] = fma(ki, X2, ai[5]);
                    SJS(3) = fma(kj, X0, SJS(3));
                    SJS(4) = fma(kj, X1, SJS(4));
                    SJS(5) = fma(kj, X2, SJS(5));
                } else {
                    // the Kepler map of eq. (26), as in MODE 0, for the close lanes
                    double d[6] = {0.0, 0.0, 0.0, kf * X0, kf * X1, kf * X2};
                    const double x0 = fma(-cb, w0, X0), x1 = fma(-cb, w1, X1),
                                 x2 = fma(-cb, w2, X2);
                    const double r0sq = fma(x0, x0, fma(x1, x1, x2 * x2));
                    const bool kl = close && (r0sq > 0.0);
                    collide = collide || (close && !(r0sq > 0.0));
                    const kep::PairCoefDiag f = solve_pair<HIST, DEFKP>(
                        kl ? tau : 0.0, mu, x0, x1, x2, w0, w1, w2, kl ? r0sq : 1.0, kp);
                    if (HIST && kl) rmax = fmaxf(rmax, (float)f.resid);
                    if (kl) {
                        const double a = fma(-ca, f.fdot, f.fm1);
                        const double b = fma(-ca, f.gdm1, f.gmt);
                        d[0] = fma(a, x0, b * w0);
                        d[1] = fma(a, x1, b * w1);
                        d[2] = fma(a, x2, b * w2);
                        d[3] = fma(f.fdot, x0, f.gdm1 * w0);
                        d[4] = fma(f.fdot, x1, f.gdm1 * w1);
                        d[5] = fma(f.fdot, x2, f.gdm1 * w2);
                    }
                    const unsigned info = kl ? (((unsigned)f.iters << 16) | f.status) : 0u;
                    info_sum += info;
                    info_max = max(info_max, info);
                    n_solve += __popcll(__builtin_amdgcn_ballot_w64(kl));
                    if (HIST && kl) atomicAdd(&shist[min(info >> 16, 31u)], 1u);
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        ai[c] = fma(wgt_i, d[c], ai[c]);
                        SJS(c) = fma(-wgt_j, d[c], SJS(c));
                    }
                }
                n_kick += __popcll(__builtin_amdgcn_ballot_w64(kick));
                coll_bits |= __builtin_amdgcn_ballot_w64(collide);
                continue;
            }
            // relative state and the pair back-drift of eq. (17) by cb
            double w0 = xi[3] - SJ(3), w1 = xi[4] - SJ(4),
                   w2 = xi[5] - SJ(5);
            double x0 = fma(-cb, w0, xi[0] - SJ(0));
            double x1 = fma(-cb, w1, xi[1] - SJ(1));
            double x2 = fma(-cb, w2, xi[2] - SJ(2));
            const double r0sq = fma(x0, x0, fma(x1, x1, x2 * x2));
            const bool collide = act && !(r0sq > 0.0);
            bool live = act && !collide;
            // lanes without a pair solve a trivial problem (tau = 0, |x0| = 1; any
            // finite mu): the starter is s = 0, where t(s) = 0 holds at once
            double d[6]; // increment of the pair map less the starting relative state, per unit mu
            unsigned info;
            if constexpr (MODE == 4) {
                // Pairs that may lie in the network's domain (a necessary condition
                // from the unreduced tau) are listed for k_deferred while the tile's
                // list has room, and skipped here; the rest take the plain solve.
                const bool cand = live & kep::pair_may_qualify_q(q4, mu, r0sq);
                const unsigned long long mask = __builtin_amdgcn_ballot_w64(cand);
                if (mask) {
                    const unsigned long long below =
                        lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
                    const int rank = (int)__popcll(below), total = (int)__popcll(mask);
                    if (cand && rank < room) {
                        net.defer_pairs[(size_t)blockIdx.x * kep::DEFER_CAP +
                                        (kep::DEFER_CAP - room) + rank] =
                            make_int2(ig, J * TILE + q);
                        live = false; // solved, and counted, by k_deferred
                    }
                    room = room > total ? room - total : 0;
                }
            }
            if constexpr (HALVES && !HIST && (MODE == 0 || MODE == 4)) {
                // The pairs solved are counted by a ballot of the time passed on
                // (tau where a pair is solved, 0 elsewhere; tau != 0 is a condition
                // of this path): the compiler forms a ballot of the combined lane
                // predicate through two vector operations, of the comparison
                // through one.  The collisions are tallied per lane.
                double tsel = live ? tau_v : 0.0;
                asm volatile("" : "+v"(tsel)); // keeps the comparison on tsel
                n_solve += __popcll(__builtin_amdgcn_ballot_w64(tsel != 0.0));
                coll_lane = coll_lane | collide;
                // Lanes without a pair pass their own r0^2 with tau = 0, which the
                // solve takes at s = 0 to zero increments for any finite positive
                // r0^2; the floor keeps r0^2 = 0 (a collision, or a pair of
                // coincident massless particles) finite in the solve.
                const kep::PairMap pm = kep::kepler_map_halves(tsel, mu, x0, x1, x2, w0, w1, w2,
                                                               fmax(r0sq, 0x1p-1022));
                d[0] = pm.dx0;
                d[1] = pm.dx1;
                d[2] = pm.dx2;
                d[3] = pm.dv0;
                d[4] = pm.dv1;
                d[5] = pm.dv2;
                info = pm.info;
            } else if constexpr (MODE == 0 || MODE == 4 || MODE == 5) { // (MODE 5 never gets here)
                const kep::PairCoefDiag f = solve_pair<HIST, DEFKP>(
                    live ? tau : 0.0, mu, x0, x1, x2, w0, w1, w2, live ? r0sq : 1.0, kp);
                if (HIST && live) rmax = fmaxf(rmax, (float)f.resid);
                const double a = fma(-ca, f.fdot, f.fm1);
                const double b = fma(-ca, f.gdm1, f.gmt);
                d[0] = fma(a, x0, b * w0);
                d[1] = fma(a, x1, b * w1);
                d[2] = fma(a, x2, b * w2);
                d[3] = fma(f.fdot, x0, f.gdm1 * w0);
                d[4] = fma(f.fdot, x1, f.gdm1 * w1);
                d[5] = fma(f.fdot, x2, f.gdm1 * w2);
                info = ((unsigned)f.iters << 16) | f.status;
            } else {
                kep::PairFlow f;
                if constexpr (MODE == 1) {
                    f = kep::kepler_flow_domain<HIST>(live ? tau : 0.0, mu, x0, x1, x2,
                                                      w0, w1, w2, live ? r0sq : 1.0, kp,
                                                      net.tau2_lo, net.tau2_hi, net.b_lo,
                                                      net.e2_hi);
                    if (HIST && live) rmax = fmaxf(rmax, (float)f.resid);
                    const bool dom = live && f.in_dom;
                    gc.dom += __popcll(__ballot(dom));
                    dom_it += dom ? (unsigned)f.iters : 0u;
                } else { // harvest
                    kep::NetGuess<MODE> gp(net, ig, J * TILE + q);
                    f = kep::kepler_flow(live ? tau : 0.0, mu, x0, x1, x2, w0, w1,
                                         w2, live ? r0sq : 1.0, kp, gp);
                    const bool dom = live && gp.in_dom;
                    gc.dom += __popcll(__ballot(dom));
                    dom_it += dom ? (unsigned)f.iters : 0u;
                }
                if (MODE == 3) { // the same relative state again, bitwise
                    asm volatile("" ::: "memory");
                    w0 = xi[3] - SJ(3);
                    w1 = xi[4] - SJ(4);
                    w2 = xi[5] - SJ(5);
                    x0 = fma(-cb, w0, xi[0] - SJ(0));
                    x1 = fma(-cb, w1, xi[1] - SJ(1));
                    x2 = fma(-cb, w2, xi[2] - SJ(2));
                }
                const double a = fma(-ca, f.fdot, f.fm1);
                const double b = fma(-ca, f.gdm1, f.gmt);
                d[0] = fma(a, x0, b * w0);
                d[1] = fma(a, x1, b * w1);
                d[2] = fma(a, x2, b * w2);
                d[3] = fma(f.fdot, x0, f.gdm1 * w0);
                d[4] = fma(f.fdot, x1, f.gdm1 * w1);
                d[5] = fma(f.fdot, x2, f.gdm1 * w2);
                info = kep::pack_info(f.iters, f.converged, f.safeguarded);
            }
            // weights mu_ij / m_i = m_j / (m_i + m_j) and mu_ij / m_j = m_i / (m_i + m_j),
            // times mu = G (m_i + m_j) that the increments are divided by; lanes
            // without a pair have zero increments (they solve tau = 0)
            const double wgt_i = gmj;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                ai[c] = fma(wgt_i, d[c], ai[c]);
                SJS(c) = fma(-wgt_j, d[c], SJS(c));
            }
            info_sum += info;
            info_max = max(info_max, info);
            if constexpr (!(HALVES && !HIST && (MODE == 0 || MODE == 4))) {
                n_solve += __popcll(__builtin_amdgcn_ballot_w64(live));
                coll_bits |= __builtin_amdgcn_ballot_w64(collide);
            }
            if (HIST && live) atomicAdd(&shist[min(info >> 16, 31u)], 1u);
        }
        };
        if (full_tile) sweep(BoolTag<true>{});
        else sweep(BoolTag<false>{});
#undef SJ
#undef SJS

        if constexpr (SPLIT > 1) {
            if (wv > 0)
                for (int c = 0; c < 6; ++c) sacc[wv - 1][c][lane] = ai[c];
        }
        __syncthreads();
        if (wv == 0) {
            // the wavefronts' sums in wavefront order (SPLIT 1: the sums as they are)
            double aj[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                aj[c] = sjs[0][c][lane];
#pragma unroll
                for (int w = 1; w < SPLIT; ++w) {
                    ai[c] += sacc[w - 1][c][lane];
                    aj[c] += sjs[w][c][lane];
                }
            }
            const size_t cs = TILE; // component stride inside a partial
            // slot I of block J (the j side)
            if (!diag) {
                double *pji = part + (size_t)(slot_j + I) * 6 * cs + lane;
                for (int c = 0; c < 6; ++c) pji[c * cs] = aj[c];
            }
            // the tile's i side (on the diagonal both sides are block I's): an item
            // of one tile writes it; a strip adds it to its earlier tiles' sums, in
            // tile order, and writes the total after its last tile
            double *pij = part + (size_t)slot_i * 6 * cs + lane;
            for (int c = 0; c < 6; ++c) {
                const double o = diag ? ai[c] + aj[c] : ai[c];
                if (len == 1) {
                    pij[c * cs] = o;
                } else {
                    const double acc = J == J0 ? o : sacc[0][c][lane] + o;
                    if (J == J0 + len - 1) pij[c * cs] = acc;
                    else sacc[0][c][lane] = acc;
                }
            }
        }
        slot_j += apply_slots(J, nb, lay); // block J + 1 starts after block J's slots
        // with SPLIT each wavefront counts the sub-steps it took
        nsub_w += SPLIT == 1 ? s1 - s0 : (s1 - s0 - wv + SPLIT - 1) / SPLIT;
    } // tiles of the item

    if constexpr (HALVES && !HIST && (MODE == 0 || MODE == 4))
        coll_bits = __builtin_amdgcn_ballot_w64(coll_lane);
    // MODE 5 counts only the close lanes' solves
    const unsigned trivial = MODE == 5 ? 0u : (unsigned)(TILE * nsub_w) - (unsigned)n_solve;
    const unsigned it_sum = wave_sum(info_sum >> 16) - trivial;
    const unsigned it_max = n_solve ? wave_max(info_max >> 16) : 0u;
    const unsigned n_fb = wave_sum((info_sum >> 8) & 0xffu);
    const bool any_noconv = wave_sum(info_sum & 0xffu) != 0;
    if (MODE != 0 && MODE != 5) gc.dom_iters = wave_sum(dom_it);
    const unsigned flags = (any_noconv ? ST_NOCONV : 0u) | (coll_bits ? ST_COLLIDE : 0u);
    const unsigned rbits = HIST ? wave_max(__float_as_uint(rmax)) : 0u;
    if (lane == 0) {
        slot_add(slots, blockIdx.x, n_solve, it_sum, n_fb, it_max);
        if (HIST) slot_max_resid(slots, blockIdx.x, rbits);
        if (MODE != 0 && MODE != 5) slot_add_guess(slots, blockIdx.x, gc);
        if (MODE == 5) slot_add_kicks(slots, blockIdx.x, n_kick);
        if (flags) record_error(cnt, flags, step);
        if (MODE == 4 && room < kep::DEFER_CAP) {
            net.defer_count[blockIdx.x] = kep::DEFER_CAP - room;
            net.defer_tiles[atomicAdd(&cnt->defer_ntiles, 1u)] = blockIdx.x;
        }
    }
    if (HIST && wv == 0 && lane < 32) atomicAdd(&cnt->hist[lane], shist[lane]);
}

// The pairs that k_pairs listed (MODE 4): the list of one tile per wavefront;
// those in the network's domain are started from its value (fused MFMA
// evaluation), the others from the plain starter, and all take the same root
// search; their weighted increments
// are added to the tile's partial sums in list order, one lane per component,
// so the result does not depend on the order in which tiles are taken.
// Persistent: every wave leaves once the list is exhausted.
__global__ __launch_bounds__(TILE) void k_deferred(int nb, int np, double tau, double cb,
                                                   double ca, double G,
                                                   const double *__restrict__ S,
                                                   double *__restrict__ part, DevCounters *cnt,
                                                   SlotStats *slots, kep::KeplerParams kp,
                                                   long long step, const kep::GuessNet net)
{
    if (cnt->status) return;
    __shared__ double sc[TILE][12]; // weighted increments of the listed pairs
    __shared__ int sidx[TILE][2];   // their slots in blocks I and J
    const int lane = threadIdx.x;
    const double *M = S;
    const double *V = S + 4 * (size_t)np;
    const double *XH = S + 7 * (size_t)np;
    unsigned long long n_solve = 0, n_fb = 0;
    unsigned it_sum = 0, it_max = 0;
    GuessCount gc;
    bool any_noconv = false;
    float rmax = 0.0f; // per lane: largest relative Kepler residual
    const unsigned ntl = cnt->defer_ntiles;
    for (;;) {
        unsigned item = 0;
        if (lane == 0) item = atomicAdd(&cnt->defer_next, 1u);
        item = __shfl(item, 0, 64);
        if (item >= ntl) break;
        const int tile = net.defer_tiles[item];
        const int count = net.defer_count[tile];
        int I, J;
        tile_blocks(tile, nb, I, J);
        const bool has = lane < count;
        int i = I * TILE, j = J * TILE + 1;
        if (has) {
            const int2 p = net.defer_pairs[(size_t)tile * kep::DEFER_CAP + lane];
            i = p.x;
            j = p.y;
        }
        // the relative state exactly as k_pairs forms it
        const double gmi = G * M[i], gmj = G * M[j];
        const double w0 = V[i] - V[j], w1 = V[np + i] - V[np + j],
                     w2 = V[2 * (size_t)np + i] - V[2 * (size_t)np + j];
        const double x0 = fma(-cb, w0, XH[i] - XH[j]);
        const double x1 = fma(-cb, w1, XH[np + i] - XH[np + j]);
        const double x2 = fma(-cb, w2, XH[2 * (size_t)np + i] - XH[2 * (size_t)np + j]);
        const double r0sq = fma(x0, x0, fma(x1, x1, x2 * x2));
        const double mu = has ? gmi + gmj : 0.0;
        const double s_net = kep::net_starter(net, tau, mu, x0, x1, x2, w0, w1, w2, r0sq);
        kep::NetGuess<2> gp(net, i, j, s_net);
        const kep::PairFlow f = kep::kepler_flow(has ? tau : 0.0, mu, x0, x1, x2, w0, w1, w2,
                                                 has ? r0sq : 1.0, kp, gp);
        const double a = fma(-ca, f.fdot, f.fm1);
        const double b = fma(-ca, f.gdm1, f.gmt);
        const double d[6] = {fma(a, x0, b * w0), fma(a, x1, b * w1), fma(a, x2, b * w2),
                             fma(f.fdot, x0, f.gdm1 * w0), fma(f.fdot, x1, f.gdm1 * w1),
                             fma(f.fdot, x2, f.gdm1 * w2)};
        // the weights of k_pairs (the flow's coefficients are per unit mu)
        const double wgt_i = gmj, wgt_j = gmi;
        __syncthreads(); // the previous item's readers of sc are done
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            sc[lane][c] = wgt_i * d[c];
            sc[lane][6 + c] = -wgt_j * d[c];
        }
        sidx[lane][0] = i - I * TILE;
        sidx[lane][1] = j - J * TILE;
        __syncthreads();
        // list order: lane c < 6 adds component c of every listed pair, i side to
        // slot J of block I, j side to slot I of block J (the listing kernel runs
        // one tile per work item: block K's slots are its tiles' columns, nb per
        // block; no two lanes touch one address)
        if (lane < 6) {
            double *pi = part + (((size_t)I * nb + J) * 6 + lane) * TILE;
            double *pj = part + (((size_t)J * nb + I) * 6 + lane) * TILE;
            for (int k = 0; k < count; ++k) {
                pi[sidx[k][0]] += sc[k][lane];
                pj[sidx[k][1]] += sc[k][6 + lane];
            }
        }
        n_solve += __popcll(__ballot(has));
        n_fb += __popcll(__ballot(has && f.safeguarded));
        it_sum += has ? f.iters : 0;
        it_max = max(it_max, has ? (unsigned)f.iters : 0u);
        gc.dom += __popcll(__ballot(has && gp.in_dom));
        gc.dom_iters += wave_sum(has && gp.in_dom ? (unsigned)f.iters : 0u);
        gc.learned += __popcll(__ballot(has && gp.used));
        gc.restarts += __popcll(__ballot(has && f.restarted));
        any_noconv = any_noconv || __ballot(has && !f.converged) != 0;
        if (has) rmax = fmaxf(rmax, (float)f.resid);
    }
    it_sum = wave_sum(it_sum);
    it_max = wave_max(it_max);
    const unsigned rbits = wave_max(__float_as_uint(rmax));
    if (lane == 0) {
        slot_add(slots, blockIdx.x, n_solve, it_sum, n_fb, it_max);
        slot_max_resid(slots, blockIdx.x, rbits);
        slot_add_guess(slots, blockIdx.x, gc);
        if (any_noconv) record_error(cnt, ST_NOCONV, step);
    }
}

// TwoSum of the nslot partial-sum slots of one component (stride apart) into
// (s, e), in slot order, B loads in flight per round.
template <int B>
__device__ inline void reduce_slots(const double *__restrict__ p, size_t stride, int nslot,
                                    double &s, double &e)
{
    int k0 = 0;
    for (; k0 + B <= nslot; k0 += B) {
        double x[B];
#pragma unroll
        for (int k = 0; k < B; ++k) x[k] = p[(size_t)(k0 + k) * stride];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const double t = s + x[k];
            const double bp = t - s;
            e += (s - (t - bp)) + (x[k] - bp);
            s = t;
        }
    }
    for (; k0 < nslot; ++k0) {
        const double x = p[(size_t)k0 * stride];
        const double t = s + x;
        const double bp = t - s;
        e += (s - (t - bp)) + (x - bp);
        s = t;
    }
}

// Deterministic compensated reduction of the partial sums of one block K
// (fixed order: the j sides L = 0..K-1, then the i sides of row K in tile
// order, one per work item of the pair launch with the layout `strips`;
// L = 0..nb-1 with one tile per item; TwoSum), then eqs. (27b-d): the drift h_after
// that ends the stage, and the drift h_next that begins the next one (27a of
// the next step; both tau/2 for eq. 25).  Wave c of the workgroup reduces
// component c.
__global__ __launch_bounds__(6 * TILE) void k_apply(int n, int nb, int np, StripLayout strips,
                                                    double h_after,
                                                    double h_next,
                                                    double *__restrict__ S,
                                                    const double *__restrict__ part,
                                                    DevCounters *cnt, long long step)
{
    const int K = blockIdx.x;
    const int c = threadIdx.x / TILE, lane = threadIdx.x % TILE;
    if (K == 0 && threadIdx.x == 0) { // the deferred-pair list of this step is consumed
        cnt->defer_ntiles = 0;
        cnt->defer_next = 0;
    }
    __shared__ double dsum[6][TILE];
    // block K's slots, stored one after the other in reduction order
    const double *p = part + ((size_t)apply_offset(K, nb, strips) * 6 + c) * TILE + lane;
    const size_t stride = 6 * TILE;
    double s = 0.0, e = 0.0;
    const int nslot = apply_slots(K, nb, strips);
    // With strips the blocks of the strip rows read fewer slots than those of
    // the single-tile rows, which set the launch's length: 16 loads in flight
    // shorten them (with every block reading nb slots the launch is bound by
    // the memory, and 8 do better).
    if (strips_on(strips)) reduce_slots<16>(p, stride, nslot, s, e);
    else reduce_slots<8>(p, stride, nslot, s, e);
    dsum[c][lane] = s + e;
    __syncthreads();
    if (c != 0) return;
    const int i = K * TILE + lane;
    if (i >= n) return;
    double *X = S + (size_t)np, *V = S + 4 * (size_t)np, *XH = S + 7 * (size_t)np;
    bool fin = true;
    for (int k = 0; k < 3; ++k) {
        const size_t o = (size_t)k * np + i;
        const double rt = XH[o] + dsum[k][lane];    // (27b)
        const double v1 = V[o] + dsum[3 + k][lane]; // (27c)
        const double x1 = rt + h_after * v1;        // (27d)
        X[o] = x1;
        V[o] = v1;
        XH[o] = x1 + h_next * v1; // (27a) of the next stage
        fin = fin && isfinite(x1) && isfinite(v1);
    }
    if (!fin) record_error(cnt, ST_NONFINITE, step);
}

// SoA -> caller layout, only when every step succeeded.
__global__ void k_export(int n, int np, const double *__restrict__ S, double *__restrict__ r,
                         double *__restrict__ v, const DevCounters *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || cnt->status) return;
    for (int c = 0; c < 3; ++c) {
        r[3 * i + c] = S[(1 + c) * (size_t)np + i];
        v[3 * i + c] = S[(4 + c) * (size_t)np + i];
    }
}

// --- energy diagnostics -----------------------------------------------------
// U: the same triangle of tiles; each tile writes sum_{pairs} m_i m_j / r_ij.
__global__ __launch_bounds__(TILE) void k_energy_pairs(int n, int nb, const double *__restrict__ m,
                                                       const double *__restrict__ r,
                                                       double *__restrict__ tile_u)
{
    const int t = blockIdx.x;
    const int noff = nb * (nb - 1) / 2;
    int I, J;
    if (t < noff) {
        int j = (int)((1.0 + sqrt(1.0 + 8.0 * (double)t)) * 0.5);
        while (j * (j - 1) / 2 > t) --j;
        while ((j + 1) * j / 2 <= t) ++j;
        J = j;
        I = t - j * (j - 1) / 2;
    } else {
        I = J = t - noff;
    }
    const int lane = threadIdx.x;
    __shared__ double sj[4][TILE];
    const int jg = J * TILE + lane;
    const bool vj = jg < n;
    sj[0][lane] = vj ? r[3 * jg] : 0.0;
    sj[1][lane] = vj ? r[3 * jg + 1] : 0.0;
    sj[2][lane] = vj ? r[3 * jg + 2] : 0.0;
    sj[3][lane] = vj ? m[jg] : 0.0;
    const int ig = I * TILE + lane;
    const bool vi = ig < n;
    const double xi = vi ? r[3 * ig] : 0.0, yi = vi ? r[3 * ig + 1] : 0.0,
                 zi = vi ? r[3 * ig + 2] : 0.0, mi = vi ? m[ig] : 0.0;
    __syncthreads();
    double u = 0.0;
    for (int q = 0; q < TILE; ++q) {
        const int j = J * TILE + q;
        const bool act = vi && j < n && (I != J || q > lane);
        const double dx = xi - sj[0][q], dy = yi - sj[1][q], dz = zi - sj[2][q];
        const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double term = act ? sj[3][q] / sqrt(d2) : 0.0;
        u += term;
    }
    u = wave_sum_d(mi * u);
    if (lane == 0) tile_u[t] = u;
}

// Per-block sums of K, M, P, L, M r (11 values) for the one-body terms.
__global__ __launch_bounds__(TILE) void k_energy_bodies(int n, const double *__restrict__ m,
                                                        const double *__restrict__ r,
                                                        const double *__restrict__ v,
                                                        double *__restrict__ blk)
{
    const int i = blockIdx.x * TILE + threadIdx.x;
    double q[11];
    for (int k = 0; k < 11; ++k) q[k] = 0.0;
    if (i < n) {
        const double mi = m[i];
        const double x = r[3 * i], y = r[3 * i + 1], z = r[3 * i + 2];
        const double a = v[3 * i], b = v[3 * i + 1], c = v[3 * i + 2];
        q[0] = 0.5 * mi * (a * a + b * b + c * c);
        q[1] = mi;
        q[2] = mi * a;
        q[3] = mi * b;
        q[4] = mi * c;
        q[5] = mi * (y * c - z * b);
        q[6] = mi * (z * a - x * c);
        q[7] = mi * (x * b - y * a);
        q[8] = mi * x;
        q[9] = mi * y;
        q[10] = mi * z;
    }
    for (int k = 0; k < 11; ++k) {
        const double s = wave_sum_d(q[k]);
        if (threadIdx.x == 0) blk[(size_t)blockIdx.x * 11 + k] = s;
    }
}

// compensated sum (s, e) of a sequence: TwoSum of each term into s, its
// rounding error into e
__device__ __forceinline__ void two_sum_add(double &s, double &e, double x)
{
    const double y = s + x;
    const double bp = y - s;
    e += (s - (y - bp)) + (x - bp);
    s = y;
}

// Compensated, fixed-order totals: out = {E, K, U, P[3], L[3], Rcm[3]}.
// Final sums of the energy diagnostics: the tile potentials (component 0) and
// the 11 per-block body sums (components 1..11).  Each of the 256 threads
// takes a strided share of a component with TwoSum, and the 256 (s, e) pairs
// are combined in a fixed binary tree, so the result is deterministic.
__global__ __launch_bounds__(256) void k_energy_final(int ntiles, int nblk, double G,
                                                      const double *__restrict__ tile_u,
                                                      const double *__restrict__ blk,
                                                      double *__restrict__ out)
{
    __shared__ double ps[256], pe[256];
    __shared__ double tot[12];
    const int k = threadIdx.x;
    for (int c = 0; c < 12; ++c) {
        const int cnt = c == 0 ? ntiles : nblk;
        double s = 0.0, e = 0.0;
        for (int t = k; t < cnt; t += 256)
            two_sum_add(s, e, c == 0 ? tile_u[t] : blk[(size_t)t * 11 + (c - 1)]);
        ps[k] = s;
        pe[k] = e;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (k < w) {
                double s2 = ps[k], e2 = pe[k] + pe[k + w];
                two_sum_add(s2, e2, ps[k + w]);
                ps[k] = s2;
                pe[k] = e2;
            }
            __syncthreads();
        }
        if (k == 0) tot[c] = ps[0] + pe[0];
        __syncthreads();
    }
    if (k == 0) {
        const double U = -G * tot[0], K = tot[1], M = tot[2];
        out[0] = K + U;
        out[1] = K;
        out[2] = U;
        for (int c = 0; c < 3; ++c) {
            out[3 + c] = tot[3 + c];
            out[6 + c] = tot[6 + c];
            out[9 + c] = M > 0.0 ? tot[9 + c] / M : 0.0;
        }
    }
}

// Wavefronts per tile for the plain mode: the tile kernel holds four
// wavefronts per SIMD, and a launch of fewer than two rounds of tiles over all
// of them leaves SIMDs idle or the last round ragged; splitting a tile's
// sub-steps over 2 or 4 wavefronts fills them (at the cost of one combination
// of the partial sums per tile).
int pair_split(int ntiles, int cus)
{
    const int64_t slots = (int64_t)cus * 16; // 4 SIMDs x 4 wavefronts per CU
    int split = 1;
    while (split < 4 && (int64_t)ntiles * split < 2 * slots) split *= 2;
    return split;
}

// One tile-kernel launch with SPLIT wavefronts per tile (mode 4 always one);
// with SPLIT 1 one wavefront per work item of the layout `strips`
// (choose_strips in tiles.hpp).
template <bool HIST, int MODE, bool DEFKP = false, bool HALVES = false>
void launch_tiles(int split, StripLayout strips, int ntiles, hipStream_t st, int n, int nb,
                  int np, double dt, double cb, double ca, double G, double e2, double e4, const double *S,
                  double *part, DevCounters *cnt, SlotStats *slots, kep::KeplerParams kp,
                  long long step, const kep::GuessNet &net)
{
#define SAKURA_PAIR_ARGS n, nb, np, strips, dt, cb, ca, G, e2, e4, S, part, cnt, slots, kp, step, \
                         net
    if constexpr (MODE != 4) {
        if (split == 4) {
            k_pairs<HIST, MODE, DEFKP, HALVES, 4><<<ntiles, 4 * TILE, 0, st>>>(SAKURA_PAIR_ARGS);
            return;
        }
        if (split == 2) {
            k_pairs<HIST, MODE, DEFKP, HALVES, 2><<<ntiles, 2 * TILE, 0, st>>>(SAKURA_PAIR_ARGS);
            return;
        }
    }
    const int nitems = (int)layout_items(nb, strips);
    k_pairs<HIST, MODE, DEFKP, HALVES, 1><<<nitems, TILE, 0, st>>>(SAKURA_PAIR_ARGS);
#undef SAKURA_PAIR_ARGS
}

template <bool HIST>
void launch_pairs_h(int mode, int split, StripLayout strips, int ntiles, hipStream_t st, int n, int nb,
                    int np,
                    double dt, double cb, double ca, double G, double e2, double e4,
                    const double *S, double *part, DevCounters *cnt, SlotStats *slots,
                    kep::KeplerParams kp, long long step, const kep::GuessNet &net)
{
    // the plain solve with the default parameters built in, where they apply,
    // and with the increments formed in the solver's copy where the drifts
    // split into halves of a step that is not zero (that kernel counts the
    // pairs it solves from the time it passes to the solver)
    const bool defkp = kp.tol == kep::DEFAULT_TOL && kp.max_iter == kep::DEFAULT_MAX_ITER;
    const bool halves = !HIST && defkp && cb == ca && ca == 0.5 * dt && dt != 0.0;
#define SAKURA_TILE_ARGS split, strips, ntiles, st, n, nb, np, dt, cb, ca, G, e2, e4, S, part, cnt, \
                         slots, \
                         kp, step, net
    switch (mode) {
    case 1:
        launch_tiles<HIST, 1>(SAKURA_TILE_ARGS);
        break;
    case 2: // the network's starter: pairs of its domain go through k_deferred
        if (halves) launch_tiles<HIST, 4, true, true>(SAKURA_TILE_ARGS);
        else if (defkp) launch_tiles<HIST, 4, true>(SAKURA_TILE_ARGS);
        else launch_tiles<HIST, 4>(SAKURA_TILE_ARGS);
        k_deferred<<<std::min(ntiles, 1024), TILE, 0, st>>>(nb, np, dt, cb, ca, G, S, part, cnt,
                                                          slots, kp, step, net);
        break;
    case 3:
        launch_tiles<HIST, 3>(SAKURA_TILE_ARGS);
        break;
    case 5: // close-pair hybrid
        if (defkp) launch_tiles<HIST, 5, true>(SAKURA_TILE_ARGS);
        else launch_tiles<HIST, 5>(SAKURA_TILE_ARGS);
        break;
    default:
        if constexpr (!HIST) {
            if (halves) {
                launch_tiles<false, 0, true, true>(SAKURA_TILE_ARGS);
                break;
            }
        }
        if (defkp) launch_tiles<HIST, 0, true>(SAKURA_TILE_ARGS);
        else launch_tiles<HIST, 0>(SAKURA_TILE_ARGS);
    }
#undef SAKURA_TILE_ARGS
}

void launch_pairs(bool hist, int mode, int split, StripLayout strips, int ntiles, hipStream_t st, int n,
                  int nb, int np,
                  double dt, double cb, double ca, double G, double e2, double e4,
                  const double *S, double *part,
                  DevCounters *cnt, SlotStats *slots, kep::KeplerParams kp, long long step,
                  const kep::GuessNet &net)
{
    if (hist)
        launch_pairs_h<true>(mode, split, strips, ntiles, st, n, nb, np, dt, cb, ca, G, e2, e4, S,
                             part, cnt,
                             slots, kp, step, net);
    else
        launch_pairs_h<false>(mode, split, strips, ntiles, st, n, nb, np, dt, cb, ca, G, e2, e4, S,
                              part, cnt,
                              slots, kp, step, net);
}

// One W stage of a composition of the step (Sec. 2.2): the pair map (flow
// time t, back-drifts cb before and ca after, t = cb + ca), the drift that
// ends the stage and the drift that begins the next one.
struct Stage {
    double t, cb, ca, after, next;
};

// The stages of one step over dt and the drift that begins the first.
//  eq. (25) with the pair map of eq. (26): one stage.
//  eq. (24): a stage over dt/2 with eq. (19b) pairs (back-drift first) and one
//    with eq. (19a) pairs (back-drift last), no drift between them.
//  triple jump of eq. (25): steps over g1 dt, g0 dt, g1 dt (Yoshida 1990).
int scheme_stages(int scheme, double dt, Stage st[3], int &count, double &first)
{
    const double h = 0.5 * dt;
    switch (scheme) {
    case SAKURA_SCHEME_PSI:
        st[0] = {dt, h, h, h, h};
        count = 1;
        first = h;
        return SAKURA_OK;
    case SAKURA_SCHEME_UNMERGED:
        st[0] = {h, h, 0.0, 0.0, 0.0};
        st[1] = {h, 0.0, h, h, h};
        count = 2;
        first = h;
        return SAKURA_OK;
    case SAKURA_SCHEME_TRIPLE_JUMP: {
        // g1 = 1/(2 - 2^(1/3)) correctly rounded; g0 = 1 - 2 g1 (exact in double)
        const double g1 = 0x1.59e8b6eb96338p+0, g0 = 1.0 - 2.0 * g1;
        const double t1 = g1 * dt, t0 = g0 * dt, h1 = 0.5 * t1, h0 = 0.5 * t0;
        st[0] = {t1, h1, h1, h1, h0};
        st[1] = {t0, h0, h0, h0, h1};
        st[2] = {t1, h1, h1, h1, h1};
        count = 3;
        first = h1;
        return SAKURA_OK;
    }
    default:
        return SAKURA_EINVAL;
    }
}

// event pairs that time the pair launches of one evolve call
constexpr int64_t TIMING_RING = 256;

// adds the duration of the launch bracketed by event pair `slot` (waits for it)
int read_pair_timing(sakura_t *h, size_t slot, double *total_ms)
{
    float ms = 0.0f;
    SAKURA_HIP(h, hipEventSynchronize(h->events[3 + 2 * slot]));
    SAKURA_HIP(h, hipEventElapsedTime(&ms, h->events[2 + 2 * slot], h->events[3 + 2 * slot]));
    *total_ms += ms;
    return SAKURA_OK;
}

int need_events(sakura_t *h, size_t count)
{
    while (h->events.size() < count) {
        hipEvent_t e;
        SAKURA_HIP(h, hipEventCreate(&e));
        h->events.push_back(e);
    }
    return SAKURA_OK;
}

} // namespace

// ---------------------------------------------------------------------------
// Static scratch of sakura_evolve_noalloc: state, tile partial sums, counter
// slots and counters for up to NOALLOC_MAX_N particles (12.4 MB), one copy on
// every device the library runs on, held until the process ends.  Host code
// never hands `scratch` itself to a kernel (in host code the name is only a
// stand-in): its device address comes from hipGetSymbolAddress, once per
// device, with that device current (sakura_create), and only that address is
// used.
namespace {
constexpr int NOALLOC_MAX_N = SAKURA_NOALLOC_MAX_N;
constexpr size_t NOALLOC_NB = NOALLOC_MAX_N / sk::TILE;
constexpr size_t NOALLOC_STATE = 10 * (size_t)NOALLOC_MAX_N;            // doubles
constexpr size_t NOALLOC_PART = NOALLOC_NB * NOALLOC_NB * 6 * sk::TILE; // doubles
constexpr size_t NOALLOC_SLOTS = sk::NSLOT * sizeof(sk::SlotStats) / sizeof(double);
constexpr size_t NOALLOC_CNT = (sizeof(sk::DevCounters) + 255) / 256 * 256 / sizeof(double);
constexpr size_t NOALLOC_DOUBLES = NOALLOC_STATE + NOALLOC_PART + NOALLOC_SLOTS + NOALLOC_CNT;
static_assert(NOALLOC_MAX_N % sk::TILE == 0, "whole tiles");
static_assert((NOALLOC_STATE * sizeof(double)) % 256 == 0 &&
                  (NOALLOC_PART * sizeof(double)) % 256 == 0 &&
                  (NOALLOC_SLOTS * sizeof(double)) % 256 == 0,
              "256-byte aligned sub-buffers");
} // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[NOALLOC_MAX_DEVICES] = {}; // device address of `scratch`, per device

// The device address of `scratch` on `device` (current), resolved once per
// device; hipSuccess or the error of hipGetSymbolAddress.
hipError_t scratch_address(int device, void **addr)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *addr = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *addr = g_scratch_addr[device];
    return hipSuccess;
}
} // namespace

extern "C" {

int sakura_create(sakura_t **out, int device, const sakura_opts *opts)
{
    if (!out) return SAKURA_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return SAKURA_EINVAL;
    sakura_t *h = new sakura();
    h->device = device;
    if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        h->cus < 1)
        h->cus = 256;
    if (opts) h->opts = *opts;
    if (h->opts.kepler_rtol <= 0.0) h->opts.kepler_rtol = kep::DEFAULT_TOL;
    if (h->opts.max_iter <= 0) h->opts.max_iter = kep::DEFAULT_MAX_ITER;
    if (h->opts.max_iter > SAKURA_MAX_ITER || h->opts.tile_override < 0 ||
        h->opts.tile_override > sk::TILE || h->opts.row_strip < 0 || h->opts.row_strip > 64 ||
        (h->opts.row_strip & (h->opts.row_strip - 1)) != 0 ||
        (h->opts.guess != SAKURA_GUESS_ANALYTIC && h->opts.guess != SAKURA_GUESS_LEARNED)) {
        delete h;
        return SAKURA_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc((void **)&h->cnt, sizeof(sk::DevCounters)) != hipSuccess ||
        hipMalloc((void **)&h->slots, sk::NSLOT * sizeof(sk::SlotStats)) != hipSuccess ||
        hipHostMalloc((void **)&h->host_cnt, sizeof(sk::DevCounters), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&h->host_out, 12 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        sakura_destroy(h);
        return SAKURA_EHIP;
    }
    // the allocation-free entry point's scratch on this device (a failure is
    // reported by that entry point; the others do not need it)
    const hipError_t se = scratch_address(device, &h->noalloc_scratch);
    if (se != hipSuccess)
        h->noalloc_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(se);
    *out = h;
    return SAKURA_OK;
}

void sakura_destroy(sakura_t *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->state) (void)hipFree(h->state);
    if (h->part) (void)hipFree(h->part);
    if (h->scratch_e) (void)hipFree(h->scratch_e);
    if (h->cnt) (void)hipFree(h->cnt);
    if (h->slots) (void)hipFree(h->slots);
    if (h->host_cnt) (void)hipHostFree(h->host_cnt);
    if (h->host_out) (void)hipHostFree(h->host_out);
    if (h->batch_state) (void)hipFree(h->batch_state);
    if (h->batch_work) (void)hipFree(h->batch_work);
    if (h->batch_offsets) (void)hipFree(h->batch_offsets);
    if (h->tune_rv) (void)hipFree(h->tune_rv);
    if (h->net_buf) (void)hipFree(h->net_buf);
    if (h->defer_pairs) (void)hipFree(h->defer_pairs);
    if (h->defer_idx) (void)hipFree(h->defer_idx);
    if (h->row_count) (void)hipFree(h->row_count);
    if (h->mlp_buf) (void)hipFree(h->mlp_buf);
    if (h->mlp_part) (void)hipFree(h->mlp_part);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    if (h->capture_stream2) (void)hipStreamDestroy(h->capture_stream2);
    if (h->capture_stream3) (void)hipStreamDestroy(h->capture_stream3);
    if (h->graph_fork) (void)hipEventDestroy(h->graph_fork);
    if (h->graph_join) (void)hipEventDestroy(h->graph_join);
    if (h->graph_join2) (void)hipEventDestroy(h->graph_join2);
    delete h;
}

const char *sakura_last_error(const sakura_t *h) { return h ? h->err.c_str() : "null handle"; }

} // extern "C"

namespace {

// Device buffers of one evolve call: the state, the tile partial sums and the
// counters.  `fixed` marks buffers the caller provides (the allocation-free
// entry point); otherwise the handle's own buffers are grown as needed.
struct EvolveBuffers {
    double *state, *part;
    sk::DevCounters *cnt;
    sk::SlotStats *slots;
    bool fixed;
};

int evolve_run(sakura_t *h, int64_t n, const double *m, double *r, double *v, double dt,
               int64_t nsteps, double G, int scheme, void *stream, sakura_stats *stats,
               EvolveBuffers buf)
{
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->failed_step = -1;
    }
    if (n < 2 || !m || !r || !v) return sk::fail(h, SAKURA_EINVAL, "n < 2 or null pointer");
    if (!std::isfinite(dt) || !std::isfinite(G) || !(G > 0.0))
        return sk::fail(h, SAKURA_EINVAL, "dt and G must be finite and G > 0");
    int rc;
    if (!buf.fixed && (rc = sk::check_size(h, n))) return rc;
    if (nsteps < 0) return sk::fail(h, SAKURA_EINVAL, "nsteps < 0");
    Stage stages[3];
    int nstage = 0;
    double first = 0.0;
    if (scheme_stages(scheme, dt, stages, nstage, first))
        return sk::fail(h, SAKURA_EINVAL, "unknown composition scheme");
    if (nsteps == 0) return SAKURA_OK;

    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)((n + sk::TILE - 1) / sk::TILE);
    const int np = nb * sk::TILE;
    const int ntiles = nb * (nb + 1) / 2;
    const kep::KeplerParams kp{h->opts.kepler_rtol, h->opts.max_iter};
    kep::GuessNet net{};
    int mode = sk::guess_mode(h, &net);
    if (mode < 0) return sk::fail(h, SAKURA_ENOMODEL, "learned starter requested but no model is loaded");
    const double e2 = h->hybrid_eta * h->hybrid_eta, e4 = e2 * e2;
    if (h->hybrid_eta > 0.0) {
        if (scheme != SAKURA_SCHEME_PSI)
            return sk::fail(h, SAKURA_EINVAL, "the close-pair hybrid runs the merged step only");
        if (mode == 2 || mode == 3)
            return sk::fail(h, SAKURA_EINVAL,
                            "the close-pair hybrid runs with the analytic starter only "
                            "(no learned starter, no harvest)");
        mode = 5;
    }
    if (buf.fixed && (mode == 2 || mode == 3))
        return sk::fail(h, SAKURA_EINVAL,
                        "the allocation-free entry point runs the plain starter only "
                        "(no learned starter, no harvest)");
    // a requested strip length runs one wavefront per tile; the pair launches
    // and k_apply share the layout of the partial sums, stored compactly
    const int split = h->opts.row_strip > 0 && mode == 0 ? 1 : pair_split(ntiles, h->cus);
    // wavefront slots: 4 SIMDs x 4 wavefronts per CU
    const StripLayout strips =
        choose_strips(h->opts.row_strip, split == 1 && mode == 0, nb, 16 * (long long)h->cus);
    if (strips.S < 1 || (strips.S & (strips.S - 1)) != 0 || strips.kc < 0 || strips.kc > nb)
        return sk::fail(h, SAKURA_EINVAL, "internal: strip layout out of range");
    const int64_t part_doubles = apply_offset(nb, nb, strips) * 6 * sk::TILE;
    if (!buf.fixed) {
        if ((rc = sk::check_capacity(h, n, part_doubles))) return rc;
        if ((rc = sk::grow(h, &h->state, &h->cap_np, 10 * (int64_t)np))) return rc;
        if ((rc = sk::grow(h, &h->part, &h->cap_part, part_doubles))) return rc;
        buf.state = h->state;
        buf.part = h->part;
    }
    // the allocation-free path creates no events: it reports no timings
    const bool timing = stats != nullptr && !buf.fixed;
    const int64_t nlaunch = nsteps * nstage;
    // pair launches are timed with a ring of event pairs: a pair is read back
    // (waiting for the launch it bracketed) before it is recorded again, so a
    // long evolve holds at most TIMING_RING launches' events
    const int64_t ring = std::min<int64_t>(nlaunch, TIMING_RING);
    if (timing && (rc = need_events(h, 2 + 2 * (size_t)ring))) return rc;
    double pair_ms = 0.0;
    if (mode == 2) { // lists of deferred pairs
        if ((rc = sk::grow(h, &h->defer_pairs, &h->cap_defer, (int64_t)ntiles * kep::DEFER_CAP)))
            return rc;
        if ((rc = sk::grow(h, &h->defer_idx, &h->cap_defer_idx, 2 * (int64_t)ntiles))) return rc;
        net.defer_pairs = h->defer_pairs;
        net.defer_count = h->defer_idx;
        net.defer_tiles = h->defer_idx + ntiles;
    }

    if (timing) SAKURA_HIP(h, hipEventRecord(h->events[0], st));
    sk::k_clear<<<1, sk::NSLOT, 0, st>>>(buf.cnt, buf.slots);
    k_import<<<(np + 255) / 256, 256, 0, st>>>((int)n, np, m, r, v, first, buf.state, buf.cnt);
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int k = 0; k < nstage; ++k) {
            const Stage &g = stages[k];
            const int64_t e = s * nstage + k;
            const size_t slot = timing ? (size_t)(e % ring) : 0;
            if (timing && e >= ring && (rc = read_pair_timing(h, slot, &pair_ms))) return rc;
            if (timing) SAKURA_HIP(h, hipEventRecord(h->events[2 + 2 * slot], st));
            launch_pairs(h->opts.histogram != 0, mode, split, strips, ntiles, st, (int)n, nb, np,
                         g.t, g.cb, g.ca, G, e2, e4, buf.state, buf.part, buf.cnt, buf.slots, kp,
                         s, net);
            if (timing) SAKURA_HIP(h, hipEventRecord(h->events[3 + 2 * slot], st));
            k_apply<<<nb, 6 * sk::TILE, 0, st>>>((int)n, nb, np, strips, g.after, g.next,
                                                 buf.state, buf.part, buf.cnt, s);
        }
    }
    k_export<<<(n + 255) / 256, 256, 0, st>>>((int)n, np, buf.state, r, v, buf.cnt);
    sk::k_fold_stats<<<1, sk::NSLOT, 0, st>>>(buf.slots, buf.cnt);
    SAKURA_HIP(h, hipGetLastError());
    if (timing) SAKURA_HIP(h, hipEventRecord(h->events[1], st));
    SAKURA_HIP(h, hipMemcpyAsync(h->host_cnt, buf.cnt, sizeof(sk::DevCounters), hipMemcpyDeviceToHost, st));
    SAKURA_HIP(h, hipStreamSynchronize(st));

    const sk::DevCounters &c = *h->host_cnt;
    if (stats) {
        stats->pair_solves = c.pair_solves;
        stats->iters_total = c.iters_total;
        stats->fallbacks = c.fallbacks;
        stats->iters_max = c.iters_max;
        sk::guess_stats(c, stats);
        for (int k = 0; k < 32; ++k) stats->hist[k] = c.hist[k];
        stats->pair_launches = nlaunch;
        stats->failed_step = c.status ? c.failed_step : -1;
        if (timing) {
            for (int64_t k = 0; k < ring; ++k)
                if ((rc = read_pair_timing(h, (size_t)k, &pair_ms))) return rc;
            stats->pair_kernel_ms = pair_ms;
            float ms = 0.0f;
            SAKURA_HIP(h, hipEventElapsedTime(&ms, h->events[0], h->events[1]));
            stats->call_ms = ms;
        }
    }
    const int code = sk::status_code(c.status);
    if (code) return sk::fail(h, code, std::string(sk::status_text(code)) + " at step " +
                                       std::to_string(c.failed_step));
    return SAKURA_OK;
}

} // namespace

extern "C" {

int sakura_evolve_scheme(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                         double dt, int64_t nsteps, double G, int scheme, void *stream,
                         sakura_stats *stats)
{
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    return evolve_run(h, n, m, r, v, dt, nsteps, G, scheme, stream, stats,
                      EvolveBuffers{nullptr, nullptr, h->cnt, h->slots, false});
}

int sakura_evolve(sakura_t *h, int64_t n, const double *m, double *r, double *v, double dt,
                  int64_t nsteps, double G, void *stream, sakura_stats *stats)
{
    return sakura_evolve_scheme(h, n, m, r, v, dt, nsteps, G, SAKURA_SCHEME_PSI, stream, stats);
}

int sakura_evolve_noalloc(sakura_t *h, int64_t n, const double *m, double *r, double *v,
                          double dt, int64_t nsteps, double G, void *stream,
                          sakura_stats *stats)
{
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (n > NOALLOC_MAX_N) {
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->failed_step = -1;
        }
        return sk::fail(h, SAKURA_EINVAL,
                        "n = " + std::to_string(n) + " exceeds the " +
                            std::to_string(NOALLOC_MAX_N) +
                            " particles of the allocation-free entry point's static scratch");
    }
    if (!h->noalloc_scratch)
        return sk::fail(h, SAKURA_EHIP, "no device address for the static scratch: " +
                                            h->noalloc_err);
    double *base = static_cast<double *>(h->noalloc_scratch);
    EvolveBuffers buf{base, base + NOALLOC_STATE,
                      reinterpret_cast<sk::DevCounters *>(base + NOALLOC_STATE + NOALLOC_PART +
                                                          NOALLOC_SLOTS),
                      reinterpret_cast<sk::SlotStats *>(base + NOALLOC_STATE + NOALLOC_PART),
                      true};
    return evolve_run(h, n, m, r, v, dt, nsteps, G, SAKURA_SCHEME_PSI, stream, stats, buf);
}

int sakura_set_hybrid(sakura_t *h, double eta)
{
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (!(eta >= 0.0) || !std::isfinite(eta))
        return sk::fail(h, SAKURA_EINVAL, "eta must be finite and >= 0");
    h->hybrid_eta = eta;
    return SAKURA_OK;
}

int sakura_step(sakura_t *h, int64_t n, const double *m, double *r, double *v, double dt,
                double G, void *stream, sakura_stats *stats)
{
    return sakura_evolve(h, n, m, r, v, dt, 1, G, stream, stats);
}

int sakura_energy(sakura_t *h, int64_t n, const double *m, const double *r, const double *v,
                  double G, double out[12], void *stream)
{
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (n < 2 || !m || !r || !v || !out) return sk::fail(h, SAKURA_EINVAL, "n < 2 or null pointer");
    if (n > ((int64_t)1 << 21)) return sk::fail(h, SAKURA_EINVAL, "n > 2^21 exceeds the tile grid");
    if (!std::isfinite(G) || !(G > 0.0)) return sk::fail(h, SAKURA_EINVAL, "G must be finite and > 0");
    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)((n + sk::TILE - 1) / sk::TILE);
    const int ntiles = nb * (nb + 1) / 2;
    int rc;
    if ((rc = sk::grow(h, &h->scratch_e, &h->cap_e, (int64_t)ntiles + 11 * (int64_t)nb + 12))) return rc;
    double *tile_u = h->scratch_e, *blk = tile_u + ntiles, *dout = blk + 11 * (size_t)nb;
    k_energy_pairs<<<ntiles, sk::TILE, 0, st>>>((int)n, nb, m, r, tile_u);
    k_energy_bodies<<<nb, sk::TILE, 0, st>>>((int)n, m, r, v, blk);
    k_energy_final<<<1, 256, 0, st>>>(ntiles, nb, G, tile_u, blk, dout);
    SAKURA_HIP(h, hipGetLastError());
    SAKURA_HIP(h, hipMemcpyAsync(h->host_out, dout, 12 * sizeof(double), hipMemcpyDeviceToHost, st));
    SAKURA_HIP(h, hipStreamSynchronize(st));
    std::memcpy(out, h->host_out, 12 * sizeof(double));
    return SAKURA_OK;
}

} // extern "C"
