// Batched ensembles: many independent small systems (n <= 64 each) advanced
// for all steps inside one persistent kernel.
//
// Each system is handled by a group of L lanes (L >= n, chosen per system size
// by a policy table that sakura_autotune_batch can tune); a wavefront holds
// groups of any sizes, placed by best fit.  Within a group the pairs follow the
// same diagonal schedule as the tile kernel: in sub-step s lane l meets slot
// (l + s) mod L, s = 1 .. floor((L - 1) / 2) plus, for even L, s = L/2 on the
// lower half of the lanes, which visits each unordered pair once.  The
// particle state stays in registers for all steps; positions, velocities and
// masses of the current step are published to LDS for the partners and the
// j-side sums are accumulated in LDS slots that no two lanes share within a
// sub-step.
//
// Work items (groups of systems) are sorted by cost, largest first, and popped
// from an atomic counter by a persistent grid; every wave exits once the queue
// is empty.
//
// One wavefront takes about 1.2 us per sub-step (the solve's dependency chain
// with no other work to hide it), and a system of n particles needs about n/2
// sequential sub-steps per step, so the largest systems set the length of
// the launch.  Items of larger systems therefore go to workgroups of two or
// four wavefronts that hold the same particles and take every second or
// fourth sub-step, each with its own j-side LDS slots; the partial sums are
// combined in a fixed order once per step, so all the wavefronts of a group
// carry bitwise the same state.  The wavefronts per item follow the system
// size (by default four; per size bucket as tuned or set).  The three launch widths run side by side: as parallel
// branches of the captured graph, or, launched directly, on three streams
// joined by events.
#include "common.hpp"

#include <algorithm>

namespace {
using namespace sk;

struct WorkItem {
    int row;   // the item's row of the lane table
    int count; // systems in this item
    int nsub;  // sub-steps per step: those of its largest group
    int pad;
};
// One row of 64 entries per item: lane -> (system, l | L << 8), system -1 for a
// lane without one.  A system of n particles takes L >= n consecutive lanes
// (its group), l the lane's place in it; groups of different sizes share an item.

// MODE selects the starter as in the tile kernel (0 plain, 1 domain
// statistics, 2 the network's starter, 3 harvest rows); WAVES (1, 2 or 4)
// wavefronts share each item's sub-steps; DEFKP (MODE 0) calls the copy of
// the solve with the default parameters built in that forms the whole pair
// map (kepler_map_halves: the batched step splits its drifts into halves).
template <int MODE, int WAVES, bool DEFKP = false>
__global__ __launch_bounds__(TILE * WAVES) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 4 : 1))) void k_batch(int nitems,
                                                        const WorkItem *__restrict__ items,
                                                const int2 *__restrict__ lanes,
                                                const int64_t *__restrict__ offsets,
                                                const double *__restrict__ m,
                                                const double *__restrict__ r,
                                                const double *__restrict__ v,
                                                const double *__restrict__ dt,
                                                double *__restrict__ staged, int64_t ntot,
                                                long long nsteps,
                                                double G, DevCounters *cnt, SlotStats *slots,
                                                kep::KeplerParams kp, const kep::GuessNet net,
                                                unsigned *queue)
{
    __shared__ double sj[7][TILE];         // x y z vx vy vz G m of every lane this step
    __shared__ double sa[WAVES][6][TILE];  // j-side sums, per wavefront
    __shared__ double sacc[WAVES][6][TILE]; // i-side sums, exchanged (WAVES 2)
    __shared__ int s_item;
    const int lane = WAVES == 1 ? (int)threadIdx.x : (int)threadIdx.x % TILE;
    // (wave-uniform, so that the sub-step index and its tests are scalar)
    const int wv = WAVES == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.x / TILE);
    // Every lane solves a problem in every sub-step (lanes without a pair solve
    // tau = 0: one evaluation, converged, never safeguarded); their outcomes are
    // summed per step and the trivial ones taken off at the end.
    unsigned n_live = 0, it_all = 0, it_max_all = 0, n_fb = 0; // per lane
    unsigned n_sub = 0;                                          // per wave: sub-steps taken
    unsigned dom_n = 0, dom_it = 0, n_learned = 0, n_restart = 0; // per lane

    for (;;) {
        int item = 0;
        if constexpr (WAVES == 1) {
            if (lane == 0) item = (int)atomicAdd(queue, 1u);
            item = __shfl(item, 0, 64);
        } else {
            __syncthreads(); // every wavefront is done with the previous item
            if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
            __syncthreads();
            item = s_item;
        }
        item = __builtin_amdgcn_readfirstlane(item); // the item's fields in scalar registers
        if (item >= nitems) break;
        const WorkItem w = items[item];
        const int2 lt = lanes[(size_t)w.row * TILE + lane];
        const bool in_group = lt.x >= 0;
        // a lane without a system is a group of one (its own slot)
        const int L = in_group ? (lt.y >> 8) : 1;
        const int l = in_group ? (lt.y & 0xff) : 0;
        const int sys = in_group ? lt.x : 0;
        const int64_t off = in_group ? offsets[sys] : 0;
        const int nsys_n = in_group ? (int)(offsets[sys + 1] - off) : 0;
        const bool valid = in_group && l < nsys_n;
        const double tau = in_group ? dt[sys] : 0.0;
        const double h = 0.5 * tau;
        const int64_t p = off + l;
        // Byte offset q8 of the partner's slot, (l + s) mod L within the lane's
        // group, stepped with s.  The partner holds a particle while
        // q8 < valid8.  The lane takes sub-steps s <= last_s: its group's
        // floor((L - 1) / 2), plus for even L the middle one s = L/2 on the lower
        // half of the group (the item runs to its largest group's count).
        const int L8 = 8 * L;
        const int base8 = 8 * (lane - l);
        const int lim8 = base8 + L8;
        const int inc8 = 8 * (WAVES % L);
        const int q8_first = base8 + 8 * ((l + 1 + wv) % L);
        const int valid8 = base8 + 8 * nsys_n;
        const int last_s = in_group ? (L - 1) / 2 + ((L & 1) == 0 && 2 * l < L ? 1 : 0) : 0;
        double mi = 0.0, x[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
        if (valid) {
            mi = m[p];
            for (int c = 0; c < 3; ++c) {
                x[c] = r[3 * p + c];
                u[c] = v[3 * p + c];
            }
            bool fin = isfinite(mi) && isfinite(tau);
            for (int c = 0; c < 3; ++c) fin = fin && isfinite(x[c]) && isfinite(u[c]);
            if (!fin) record_error(cnt, ST_NONFINITE, 0);
            else if (!(mi >= 0.0)) record_error(cnt, ST_INVAL, 0);
        }
        const int nsub = w.nsub;
        // sub-steps this wavefront takes per step: s = 1 + wv, 1 + wv + WAVES, ...
        const unsigned nsub_w = nsub > wv ? (unsigned)((nsub - 1 - wv) / WAVES + 1) : 0u;
        const double gmi = G * mi; // the masses as G m (mi is 0 where !valid)

        for (long long step = 0; step < nsteps; ++step) {
            double xh[3];
            for (int c = 0; c < 3; ++c) xh[c] = x[c] + h * u[c]; // (27a)
            __syncthreads(); // the previous step's readers are done
            if (wv == 0) {
                sj[0][lane] = xh[0];
                sj[1][lane] = xh[1];
                sj[2][lane] = xh[2];
                sj[3][lane] = u[0];
                sj[4][lane] = u[1];
                sj[5][lane] = u[2];
                sj[6][lane] = valid ? gmi : 0.0;
            }
            for (int c = 0; c < 6; ++c) sa[wv][c][lane] = 0.0;
            __syncthreads();

            double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            unsigned info_sum = 0, info_max = 0; // per lane, this step: of kep::pack_info
            bool coll_lane = false;              // per lane, this step: a zero separation met
            int q8 = q8_first;
            for (int s = 1 + wv; s <= nsub; s += WAVES) {
#define SJ(c) (*(const double *)((const char *)sj[c] + q8))
#define SA(c) (*(double *)((char *)sa[wv][c] + q8))
                const double gmj = SJ(6);
                const double mu = gmi + gmj;
                const bool act = valid && q8 < valid8 && mu > 0.0 && s <= last_s;
                const double w0 = u[0] - SJ(3), w1 = u[1] - SJ(4), w2 = u[2] - SJ(5);
                const double x0 = fma(-h, w0, xh[0] - SJ(0));
                const double x1 = fma(-h, w1, xh[1] - SJ(1));
                const double x2 = fma(-h, w2, xh[2] - SJ(2));
                const double r0sq = fma(x0, x0, fma(x1, x1, x2 * x2));
                const bool collide = act && !(r0sq > 0.0);
                const bool live = act && !collide;
                kep::PairFlow f;
                double d[6];
                unsigned info;
                if constexpr (MODE == 0 && DEFKP) {
                    // the whole pair map in the solver's copy (the step's drifts
                    // split into halves, h = tau/2): nothing kept across the call
                    const kep::PairMap pm = kep::kepler_map_halves(
                        live ? tau : 0.0, mu, x0, x1, x2, w0, w1, w2, live ? r0sq : 1.0);
                    d[0] = pm.dx0;
                    d[1] = pm.dx1;
                    d[2] = pm.dx2;
                    d[3] = pm.dv0;
                    d[4] = pm.dv1;
                    d[5] = pm.dv2;
                    info = pm.info;
                } else if constexpr (MODE == 0) {
                    const kep::PairCoef c = kep::kepler_flow(live ? tau : 0.0, mu, x0, x1, x2,
                                                             w0, w1, w2, live ? r0sq : 1.0, kp);
                    f.fm1 = c.fm1;
                    f.gmt = c.gmt;
                    f.fdot = c.fdot;
                    f.gdm1 = c.gdm1;
                    info = ((unsigned)c.iters << 16) | c.status;
                } else {
                    const int ql = (q8 - base8) >> 3;
                    double s_net = __builtin_nan("");
                    if (MODE == 2) {
                        const bool cand = live && kep::pair_may_qualify(net, tau, mu, r0sq);
                        if (__any(cand))
                            s_net = kep::net_starter(net, tau, cand ? mu : 0.0, x0, x1, x2, w0,
                                                     w1, w2, r0sq);
                    }
                    kep::NetGuess<MODE, false> gp(net, (int)p, (int)(off + ql), s_net);
                    f = kep::kepler_flow(live ? tau : 0.0, mu, x0, x1, x2, w0, w1, w2,
                                         live ? r0sq : 1.0, kp, gp);
                    if (live && gp.in_dom) {
                        ++dom_n;
                        dom_it += f.iters;
                    }
                    n_learned += (live && gp.used) ? 1u : 0u;
                    n_restart += (live && f.restarted) ? 1u : 0u;
                    info = kep::pack_info(f.iters, f.converged, f.safeguarded);
                }
                if constexpr (!(MODE == 0 && DEFKP)) {
                    const double a = fma(-h, f.fdot, f.fm1);
                    const double b = fma(-h, f.gdm1, f.gmt);
                    d[0] = fma(a, x0, b * w0);
                    d[1] = fma(a, x1, b * w1);
                    d[2] = fma(a, x2, b * w2);
                    d[3] = fma(f.fdot, x0, f.gdm1 * w0);
                    d[4] = fma(f.fdot, x1, f.gdm1 * w1);
                    d[5] = fma(f.fdot, x2, f.gdm1 * w2);
                }
                // m_j / (m_i + m_j) and m_i / (m_i + m_j) times the flow's 1/mu:
                // G m_j and G m_i; lanes without a pair have zero increments
                // (they solve tau = 0)
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    acc[c] = fma(gmj, d[c], acc[c]);
                    SA(c) = fma(-gmi, d[c], SA(c));
                }
#undef SJ
#undef SA
                n_live += live ? 1u : 0u;
                info_sum += info;
                info_max = max(info_max, info);
                coll_lane = coll_lane | collide;
                q8 += inc8;
                q8 = q8 >= lim8 ? q8 - L8 : q8;
                // j-side sums of this sub-step visible to the next (with two
                // wavefronts taking different numbers of sub-steps there is no
                // workgroup barrier here: the wavefront's LDS operations complete
                // in order, and the compiler may not move them across the fence)
                if constexpr (WAVES == 1) __syncthreads();
                else asm volatile("" ::: "memory");
            }
            // the step's outcomes (at most 32 sub-steps: the fields stay apart)
            n_sub += nsub_w;
            it_all += info_sum >> 16;
            n_fb += (info_sum >> 8) & 0xffu;
            it_max_all = max(it_max_all, info_max >> 16);
            unsigned flags = (info_sum & 0xffu) ? ST_NOCONV : 0u;
            if (coll_lane) flags |= ST_COLLIDE;
            double jside[6];
            if constexpr (WAVES == 1) {
                for (int c = 0; c < 6; ++c) jside[c] = sa[0][c][lane];
            } else {
                // the wavefronts' sums in a fixed order, so that all carry the
                // same state (read only: every wavefront reads these slots)
                for (int c = 0; c < 6; ++c) sacc[wv][c][lane] = acc[c];
                __syncthreads();
                for (int c = 0; c < 6; ++c) {
                    double a = sacc[0][c][lane], j = sa[0][c][lane];
#pragma unroll
                    for (int w = 1; w < WAVES; ++w) {
                        a += sacc[w][c][lane];
                        j += sa[w][c][lane];
                    }
                    acc[c] = a;
                    jside[c] = j;
                }
            }
            bool fin = true;
            for (int c = 0; c < 3; ++c) {
                const double rt = xh[c] + (acc[c] + jside[c]);        // (27b)
                const double v1 = u[c] + (acc[3 + c] + jside[3 + c]); // (27c)
                x[c] = rt + h * v1;                                      // (27d)
                u[c] = v1;
                fin = fin && isfinite(x[c]) && isfinite(v1);
            }
            if (valid && !fin) flags |= ST_NONFINITE;
            if (flags) record_error(cnt, flags, step);
        }
        if (valid && wv == 0) {
            for (int c = 0; c < 3; ++c) {
                staged[3 * p + c] = x[c];
                staged[3 * (ntot + p) + c] = u[c];
            }
        }
    }
    // the trivial solves (one evaluation each) taken off
    const unsigned n_solve = wave_sum(n_live);
    const unsigned it_sum = wave_sum(it_all) - (TILE * n_sub - n_solve);
    n_fb = wave_sum(n_fb);
    const unsigned it_max = n_solve ? wave_max(it_max_all) : 0u;
    GuessCount gc;
    if (MODE != 0) {
        gc.dom = wave_sum(dom_n);
        gc.dom_iters = wave_sum(dom_it);
        gc.learned = wave_sum(n_learned);
        gc.restarts = wave_sum(n_restart);
    }
    if (lane == 0) {
        slot_add(slots, blockIdx.x, n_solve, it_sum, n_fb, it_max);
        if (MODE != 0) slot_add_guess(slots, blockIdx.x, gc);
    }
}

template <int WAVES>
void launch_batch_w(int mode, int grid, hipStream_t st, int nitems, const WorkItem *items,
                    const int2 *lanes, const int64_t *offsets, const double *m, const double *r,
                    const double *v, const double *dt, double *staged, int64_t ntot,
                    long long nsteps, double G, DevCounters *cnt, SlotStats *slots,
                    kep::KeplerParams kp, const kep::GuessNet &net, unsigned *queue)
{
#define SAKURA_BATCH_ARGS nitems, items, lanes, offsets, m, r, v, dt, staged, ntot, nsteps, G, \
                          cnt, slots, kp, net, queue
    const bool defkp = kp.tol == kep::DEFAULT_TOL && kp.max_iter == kep::DEFAULT_MAX_ITER;
    switch (mode) {
    case 1: k_batch<1, WAVES><<<grid, TILE * WAVES, 0, st>>>(SAKURA_BATCH_ARGS); break;
    case 2: k_batch<2, WAVES><<<grid, TILE * WAVES, 0, st>>>(SAKURA_BATCH_ARGS); break;
    case 3: k_batch<3, WAVES><<<grid, TILE * WAVES, 0, st>>>(SAKURA_BATCH_ARGS); break;
    default:
        if (defkp) k_batch<0, WAVES, true><<<grid, TILE * WAVES, 0, st>>>(SAKURA_BATCH_ARGS);
        else k_batch<0, WAVES><<<grid, TILE * WAVES, 0, st>>>(SAKURA_BATCH_ARGS);
    }
#undef SAKURA_BATCH_ARGS
}

// The three launches: the items of four, two and one wavefronts (n[0], n[1],
// n[2] items, in that order in the item list) on st[0], st[1], st[2].
void launch_batch(int mode, const int grid[3], const hipStream_t st[3], const int n[3],
                  const WorkItem *items, const int2 *lanes, const int64_t *offsets,
                  const double *m, const double *r, const double *v, const double *dt,
                  double *staged, int64_t ntot, long long nsteps, double G, DevCounters *cnt,
                  SlotStats *slots, kep::KeplerParams kp, const kep::GuessNet &net)
{
    if (n[0])
        launch_batch_w<4>(mode, grid[0], st[0], n[0], items, lanes, offsets, m, r, v, dt,
                          staged, ntot, nsteps, G, cnt, slots, kp, net, &cnt->work_next4);
    if (n[1])
        launch_batch_w<2>(mode, grid[1], st[1], n[1], items + n[0], lanes, offsets, m, r, v, dt,
                          staged, ntot, nsteps, G, cnt, slots, kp, net, &cnt->work_next2);
    if (n[2])
        launch_batch_w<1>(mode, grid[2], st[2], n[2], items + n[0] + n[1], lanes, offsets, m,
                          r, v, dt, staged, ntot, nsteps, G, cnt, slots, kp, net,
                          &cnt->work_next);
}

// Staged results -> caller arrays, only when every system and step succeeded.
__global__ void k_batch_export(int64_t ntot, const double *__restrict__ staged,
                               double *__restrict__ r, double *__restrict__ v,
                               const DevCounters *cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * ntot || cnt->status) return;
    r[i] = staged[i];
    v[i] = staged[3 * ntot + i];
}

} // namespace

namespace {

// Lanes per system of size n under each packing policy: 0 dense (n lanes),
// 1 even (n rounded up to even), 2 power of two.
// Wavefronts per work item for systems of n particles: the handle's setting,
// else four (on the 4096-system benchmark ensemble four for every size with
// 16 wavefronts per CU measured 79 G pair-solves/s, against 66-70 G for four,
// two and one by size class and 8 or 16 per CU).
int batch_width(const sakura_t *h, int n)
{
    const int w = h->batch_width[n];
    return w ? w : 4;
}

// The streams and events of the side-by-side launches (created once).
int branch_streams(sakura_t *h)
{
    if (!h->capture_stream)
        SAKURA_HIP(h, hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    for (hipStream_t *sp : {&h->capture_stream2, &h->capture_stream3})
        if (!*sp) SAKURA_HIP(h, hipStreamCreateWithFlags(sp, hipStreamNonBlocking));
    for (hipEvent_t *ep : {&h->graph_fork, &h->graph_join, &h->graph_join2})
        if (!*ep) SAKURA_HIP(h, hipEventCreateWithFlags(ep, hipEventDisableTiming));
    return SAKURA_OK;
}

int policy_group(int policy, int n)
{
    switch (policy) {
    case 1: return n + (n & 1);                // even group
    case 2: {                                  // power of two
        int L = 1;
        while (L < n) L <<= 1;
        return L;
    }
    default: return n;                         // dense
    }
}

} // namespace

extern "C" {

int sakura_batch_evolve(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m,
                        double *r, double *v, const double *dt, int64_t nsteps, double G,
                        void *stream, sakura_stats *stats)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->failed_step = -1;
    }
    if (nsys < 1 || !offsets || !m || !r || !v || !dt)
        return fail(h, SAKURA_EINVAL, "nsys < 1 or null pointer");
    if (nsys > (1 << 26)) return fail(h, SAKURA_EINVAL, "too many systems");
    if (!std::isfinite(G) || !(G > 0.0)) return fail(h, SAKURA_EINVAL, "G must be finite and > 0");
    if (nsteps < 0) return fail(h, SAKURA_EINVAL, "nsteps < 0");
    if (offsets[0] != 0) return fail(h, SAKURA_EINVAL, "offsets[0] must be 0");
    for (int64_t s = 0; s < nsys; ++s) {
        const int64_t ns = offsets[s + 1] - offsets[s];
        if (ns < 1 || ns > TILE)
            return fail(h, SAKURA_EINVAL, "system " + std::to_string(s) + " has " +
                                              std::to_string(ns) +
                                              " particles; batched systems hold 1..64");
    }
    if (nsteps == 0) return SAKURA_OK;
    const int64_t ntot = offsets[nsys];

    // Work items: each system takes L >= n consecutive lanes (its group; the
    // handle's lane policy), and the systems, largest group first, are placed
    // by best fit on the lanes still free in the open items, so that groups of
    // different sizes share a wavefront.  An item runs to its largest group's
    // sub-step count and goes to the launch of that group's width (four, two or
    // one wavefronts per item); the items of each launch stay in the order they
    // were opened, largest first.
    const int ov = h->opts.tile_override;
    // A call with the same systems and packing settings as the last one
    // reuses its packing, already on the device (a repeated call, as in a
    // time loop, then costs no host work before its launches).
    const bool same_plan =
        h->plan_dev != nullptr && h->plan_dev == h->batch_work && h->plan_override == ov &&
        (int64_t)h->plan_offsets.size() == nsys + 1 &&
        std::equal(offsets, offsets + nsys + 1, h->plan_offsets.begin()) &&
        std::memcmp(h->plan_group, h->batch_group, sizeof h->plan_group) == 0 &&
        std::memcmp(h->plan_width, h->batch_width, sizeof h->plan_width) == 0;
    int nitems = h->plan_nitems;
    int nw[3] = {h->plan_nw[0], h->plan_nw[1], h->plan_nw[2]};
    if (!same_plan) {
    std::vector<int> Ls((size_t)nsys), order((size_t)nsys);
    for (int64_t s = 0; s < nsys; ++s) {
        const int n = (int)(offsets[s + 1] - offsets[s]);
        Ls[(size_t)s] = ov > 0 ? std::max(n, std::min(TILE, ov))
                               : std::max(n, std::min(TILE, h->batch_group[n]));
        order[(size_t)s] = (int)s;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return Ls[(size_t)a] > Ls[(size_t)b]; });
    std::vector<int> bin_of((size_t)nsys), bin_free, bin_nsub, bin_big;
    std::vector<int> by_free[TILE]; // open items by their free lanes (1 .. 63)
    for (const int sy : order) {
        const int L = Ls[(size_t)sy];
        int bin = -1;
        for (int f = L; f < TILE && bin < 0; ++f)
            if (!by_free[f].empty()) {
                bin = by_free[f].back();
                by_free[f].pop_back();
            }
        if (bin < 0) { // a new item: this group is its largest
            bin = (int)bin_free.size();
            bin_free.push_back(TILE);
            bin_nsub.push_back((L - 1) / 2 + ((L & 1) ? 0 : 1));
            bin_big.push_back((int)(offsets[sy + 1] - offsets[sy]));
        }
        bin_free[(size_t)bin] -= L;
        bin_of[(size_t)sy] = bin;
        if (bin_free[(size_t)bin] > 0) by_free[bin_free[(size_t)bin]].push_back(bin);
    }
    nitems = (int)bin_free.size();
    // the lane table: (system, l | L << 8) per lane, (-1, 0) on free lanes
    std::vector<int> lane_tab((size_t)nitems * TILE * 2);
    for (size_t e = 0; e < lane_tab.size(); e += 2) {
        lane_tab[e] = -1;
        lane_tab[e + 1] = 0;
    }
    std::vector<int> fill((size_t)nitems, 0), count((size_t)nitems, 0);
    for (const int sy : order) {
        const int bin = bin_of[(size_t)sy], L = Ls[(size_t)sy];
        for (int l = 0; l < L; ++l) {
            const size_t e = ((size_t)bin * TILE + (size_t)(fill[(size_t)bin] + l)) * 2;
            lane_tab[e] = sy;
            lane_tab[e + 1] = l | (L << 8);
        }
        fill[(size_t)bin] += L;
        ++count[(size_t)bin];
    }
    // items of 4, 2 and 1 wavefronts, in that order
    nw[0] = nw[1] = nw[2] = 0;
    std::vector<int> items;
    items.reserve(4 * (size_t)nitems);
    for (int cls = 0; cls < 3; ++cls)
        for (int bin = 0; bin < nitems; ++bin) {
            const int w = batch_width(h, bin_big[(size_t)bin]);
            if ((w == 4 ? 0 : (w == 2 ? 1 : 2)) != cls) continue;
            items.push_back(bin);
            items.push_back(count[(size_t)bin]);
            items.push_back(bin_nsub[(size_t)bin]);
            items.push_back(0);
            ++nw[cls];
        }
    h->host_work.assign(items.begin(), items.end());
    h->host_work.insert(h->host_work.end(), lane_tab.begin(), lane_tab.end());
    }

    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = grow(h, &h->batch_state, &h->cap_batch, 6 * ntot))) return rc;
    if (!same_plan) {
        h->plan_dev = nullptr; // until the new packing is on the device
        if ((rc = grow(h, &h->batch_work, &h->cap_work, (int64_t)h->host_work.size())))
            return rc;
        if ((rc = grow(h, &h->batch_offsets, &h->cap_offsets, nsys + 1))) return rc;
        SAKURA_HIP(h, hipMemcpyAsync(h->batch_work, h->host_work.data(),
                                     h->host_work.size() * sizeof(int), hipMemcpyHostToDevice,
                                     st));
        SAKURA_HIP(h, hipMemcpyAsync(h->batch_offsets, offsets,
                                     (size_t)(nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                                     st));
        h->plan_offsets.assign(offsets, offsets + nsys + 1);
        std::memcpy(h->plan_group, h->batch_group, sizeof h->plan_group);
        std::memcpy(h->plan_width, h->batch_width, sizeof h->plan_width);
        h->plan_override = ov;
        h->plan_nitems = nitems;
        for (int k = 0; k < 3; ++k) h->plan_nw[k] = nw[k];
        h->plan_dev = h->batch_work;
    }
    const bool timing = stats != nullptr;
    if (timing) {
        while (h->events.size() < 2) {
            hipEvent_t e;
            SAKURA_HIP(h, hipEventCreate(&e));
            h->events.push_back(e);
        }
    }

    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
    const int wpc = std::max(1, h->batch_waves_per_cu);
    const int wgrid[3] = {std::max(1, std::min(nw[0], cus * wpc / 4)),
                          std::max(1, std::min(nw[1], cus * wpc / 2)),
                          std::max(1, std::min(nw[2], cus * wpc))};
    const int grid = cus * wpc; // for the graph key
    const kep::KeplerParams kp{h->opts.kepler_rtol, h->opts.max_iter};
    kep::GuessNet net{};
    const int mode = guess_mode(h, &net);
    if (mode < 0) return fail(h, SAKURA_ENOMODEL, "learned starter requested but no model is loaded");
    const WorkItem *witems = reinterpret_cast<const WorkItem *>(h->batch_work);
    const int2 *wlanes = reinterpret_cast<const int2 *>(h->batch_work + 4 * nitems);
    const unsigned eblocks = (unsigned)((3 * ntot + 255) / 256);

    // The launch sequence is captured once into a graph (on a private stream)
    // and replayed while every argument baked into it stays the same: the
    // pointers, the particle count (state layout, export size) and the item
    // split over the three launch widths (their grids and item ranges).
    char keybuf[640];
    std::snprintf(keybuf, sizeof(keybuf),
                  "%p %p %p %p %p %p %p %lld %lld %lld %a %d %d %d %d %d %a %d %d %u %p %lld %a %a %a %a",
                  (const void *)m, (void *)r, (void *)v, (const void *)dt,
                  (void *)h->batch_state, (void *)h->batch_work, (void *)h->batch_offsets,
                  (long long)nsys, (long long)ntot, (long long)nsteps, G, nitems, nw[0], nw[1],
                  nw[2], grid, kp.tol, kp.max_iter, mode, h->model_gen, (void *)net.rows,
                  net.row_cap, net.tau2_lo, net.tau2_hi, net.b_lo, net.e2_hi);
    const bool use_graph = !h->batch_no_graph;
    if (use_graph && (h->graph_exec == nullptr || h->graph_key != keybuf)) {
        if (h->graph_exec) {
            (void)hipGraphExecDestroy(h->graph_exec);
            h->graph_exec = nullptr;
        }
        if (h->graph) {
            (void)hipGraphDestroy(h->graph);
            h->graph = nullptr;
        }
        if ((rc = branch_streams(h))) return rc;
        // recorded by a function so that a failed record still ends the
        // capture (the stream would otherwise stay in capture mode)
        auto record = [&]() -> int {
            k_clear<<<1, NSLOT, 0, h->capture_stream>>>(h->cnt, h->slots);
            // the three launches as parallel branches of the graph
            SAKURA_HIP(h, hipEventRecord(h->graph_fork, h->capture_stream));
            SAKURA_HIP(h, hipStreamWaitEvent(h->capture_stream2, h->graph_fork, 0));
            SAKURA_HIP(h, hipStreamWaitEvent(h->capture_stream3, h->graph_fork, 0));
            const hipStream_t bst[3] = {h->capture_stream, h->capture_stream2, h->capture_stream3};
            launch_batch(mode, wgrid, bst, nw, witems, wlanes, h->batch_offsets, m, r, v, dt,
                         h->batch_state, ntot, (long long)nsteps, G, h->cnt, h->slots, kp, net);
            SAKURA_HIP(h, hipEventRecord(h->graph_join, h->capture_stream2));
            SAKURA_HIP(h, hipEventRecord(h->graph_join2, h->capture_stream3));
            SAKURA_HIP(h, hipStreamWaitEvent(h->capture_stream, h->graph_join, 0));
            SAKURA_HIP(h, hipStreamWaitEvent(h->capture_stream, h->graph_join2, 0));
            k_batch_export<<<eblocks, 256, 0, h->capture_stream>>>(ntot, h->batch_state, r,
                                                                   v, h->cnt);
            k_fold_stats<<<1, NSLOT, 0, h->capture_stream>>>(h->slots, h->cnt);
            SAKURA_HIP(h, hipGetLastError());
            return SAKURA_OK;
        };
        SAKURA_HIP(h, hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
        const int crc = record();
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(h->capture_stream, &g);
        if (crc || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            h->graph_key.clear();
            return crc ? crc : fail(h, SAKURA_EHIP, std::string("hipStreamEndCapture: ") +
                                                        hipGetErrorString(ee));
        }
        h->graph = g;
        SAKURA_HIP(h, hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
        h->graph_key = keybuf;
    }
    if (timing) SAKURA_HIP(h, hipEventRecord(h->events[0], st));
    if (use_graph) {
        SAKURA_HIP(h, hipGraphLaunch(h->graph_exec, st));
    } else {
        // the three widths side by side on st and two private streams, as in
        // the graph: forked from st after the counters are cleared, joined
        // back before the export
        if ((rc = branch_streams(h))) return rc;
        k_clear<<<1, NSLOT, 0, st>>>(h->cnt, h->slots);
        SAKURA_HIP(h, hipEventRecord(h->graph_fork, st));
        SAKURA_HIP(h, hipStreamWaitEvent(h->capture_stream2, h->graph_fork, 0));
        SAKURA_HIP(h, hipStreamWaitEvent(h->capture_stream3, h->graph_fork, 0));
        const hipStream_t bst[3] = {st, h->capture_stream2, h->capture_stream3};
        launch_batch(mode, wgrid, bst, nw, witems, wlanes, h->batch_offsets, m, r, v, dt,
                     h->batch_state, ntot, (long long)nsteps, G, h->cnt, h->slots, kp, net);
        SAKURA_HIP(h, hipEventRecord(h->graph_join, h->capture_stream2));
        SAKURA_HIP(h, hipEventRecord(h->graph_join2, h->capture_stream3));
        SAKURA_HIP(h, hipStreamWaitEvent(st, h->graph_join, 0));
        SAKURA_HIP(h, hipStreamWaitEvent(st, h->graph_join2, 0));
        k_batch_export<<<eblocks, 256, 0, st>>>(ntot, h->batch_state, r, v, h->cnt);
        k_fold_stats<<<1, NSLOT, 0, st>>>(h->slots, h->cnt);
        SAKURA_HIP(h, hipGetLastError());
    }
    if (timing) SAKURA_HIP(h, hipEventRecord(h->events[1], st));
    SAKURA_HIP(h, hipMemcpyAsync(h->host_cnt, h->cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, st));
    SAKURA_HIP(h, hipStreamSynchronize(st));

    const DevCounters &c = *h->host_cnt;
    if (stats) {
        stats->pair_solves = c.pair_solves;
        stats->iters_total = c.iters_total;
        stats->fallbacks = c.fallbacks;
        stats->iters_max = c.iters_max;
        guess_stats(c, stats);
        stats->pair_launches = 1;
        stats->failed_step = c.status ? c.failed_step : -1;
        float ms = 0.0f;
        SAKURA_HIP(h, hipEventElapsedTime(&ms, h->events[0], h->events[1]));
        stats->call_ms = ms;
        stats->pair_kernel_ms = ms;
    }
    const int code = status_code(c.status);
    if (code) return fail(h, code, std::string(status_text(code)) + " at step " +
                                       std::to_string(c.failed_step));
    return SAKURA_OK;
}

int sakura_batch_set_policy(sakura_t *h, int policy, int waves_per_cu, int use_graph)
{
    if (!h || policy < 0 || policy > 2 || waves_per_cu < 1 || waves_per_cu > 32)
        return SAKURA_EINVAL;
    for (int n = 1; n <= sk::TILE; ++n) {
        h->batch_group[n] = policy_group(policy, n);
        h->batch_width[n] = 0;
    }
    h->batch_waves_per_cu = waves_per_cu;
    h->batch_no_graph = !use_graph;
    return SAKURA_OK;
}

} // extern "C"

namespace {

// System-size buckets of the packing table: 1..8, 9..16, 17..32, 33..64
// particles (items of one wavefront with several systems, of one wavefront, of
// two and of four wavefronts).
constexpr int NBUCKET = 4;
constexpr int BUCKET_LO[NBUCKET] = {1, 9, 17, 33};
constexpr int BUCKET_HI[NBUCKET] = {8, 16, 32, 64};

void set_bucket_policy(sakura_t *h, int b, int policy)
{
    for (int n = BUCKET_LO[b]; n <= BUCKET_HI[b]; ++n) h->batch_group[n] = policy_group(policy, n);
}
void set_bucket_width(sakura_t *h, int b, int width)
{
    for (int n = BUCKET_LO[b]; n <= BUCKET_HI[b]; ++n) h->batch_width[n] = width;
}

// The device's identity in the table: its gfx architecture and compute units.
void device_identity(int device, std::string &arch, int &cus)
{
    hipDeviceProp_t prop;
    arch = "unknown";
    cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':'); // feature suffixes do not matter here
        if (colon != std::string::npos) arch.resize(colon);
        cus = prop.multiProcessorCount;
    }
}

// Apply the handle's table entries for this device: per-bucket policy and
// wavefronts per item, and the grid size (the grid of the last entry that
// names one).
void apply_table(sakura_t *h)
{
    std::string arch;
    int cus;
    device_identity(h->device, arch, cus);
    for (const auto &e : h->batch_table)
        if (e.arch == arch && e.cus == cus && e.bucket >= 0 && e.bucket < NBUCKET) {
            set_bucket_policy(h, e.bucket, e.policy);
            set_bucket_width(h, e.bucket, e.width);
            h->batch_waves_per_cu = e.waves_per_cu;
        }
}

// One probe: the ensemble on scratch copies of r and v, probe_steps steps,
// with the handle's current packing, its launches made directly (no graph
// capture per probe).  The first call warms up; the time is the least of the
// next `reps` calls.
int probe(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m, const double *r,
          const double *v, const double *dt, int64_t probe_steps, double G, void *stream,
          int reps, double *ms)
{
    using namespace sk;
    const int64_t ntot = offsets[nsys];
    hipStream_t st = (hipStream_t)stream;
    double best = 1e300;
    const int keep_no_graph = h->batch_no_graph;
    h->batch_no_graph = 1;
    struct Restore {
        sakura_t *h;
        int v;
        ~Restore() { h->batch_no_graph = v; }
    } restore_graph{h, keep_no_graph};
    for (int rep = 0; rep <= reps; ++rep) {
        hipError_t e = hipMemcpyAsync(h->tune_rv, r, 3 * ntot * sizeof(double),
                                      hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->tune_rv + 3 * ntot, v, 3 * ntot * sizeof(double),
                               hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess)
            return fail(h, SAKURA_EHIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        sakura_stats s;
        const int rc = sakura_batch_evolve(h, nsys, offsets, m, h->tune_rv,
                                           h->tune_rv + 3 * ntot, dt, probe_steps, G, stream,
                                           &s);
        if (rc) return rc;
        if (rep > 0) best = std::min(best, s.call_ms);
    }
    *ms = best;
    return SAKURA_OK;
}

} // namespace

extern "C" {

int sakura_autotune_batch(sakura_t *h, int64_t nsys, const int64_t *offsets, const double *m,
                          const double *r, const double *v, const double *dt,
                          int64_t probe_steps, double G, void *stream, double *best_ms)
{
    using namespace sk;
    if (!h || nsys < 1 || !offsets || probe_steps < 1) return SAKURA_EINVAL;
    const int64_t ntot = offsets[nsys];
    int rc;
    if ((rc = grow(h, &h->tune_rv, &h->cap_tune, 6 * ntot))) return rc;
    // a failed probe leaves the handle's batch settings as they were
    int saved_group[TILE + 1], saved_width[TILE + 1];
    std::memcpy(saved_group, h->batch_group, sizeof(saved_group));
    std::memcpy(saved_width, h->batch_width, sizeof(saved_width));
    const int saved_waves = h->batch_waves_per_cu;
    auto restore = [&](int code) {
        std::memcpy(h->batch_group, saved_group, sizeof(saved_group));
        std::memcpy(h->batch_width, saved_width, sizeof(saved_width));
        h->batch_waves_per_cu = saved_waves;
        return code;
    };
    // the buckets this ensemble has systems in
    bool present[NBUCKET] = {false, false, false, false};
    for (int64_t k = 0; k < nsys; ++k) {
        const int64_t n = offsets[k + 1] - offsets[k];
        for (int b = 0; b < NBUCKET; ++b)
            if (n >= BUCKET_LO[b] && n <= BUCKET_HI[b]) present[b] = true;
    }
    // Probes launch directly (a graph captured anew for every probe setting
    // was tried and its test crashed the host process once, cause not found),
    // coordinate by coordinate: the grid size with the
    // current packing, then each present bucket's packing policy with the
    // others kept.
    const int reps = 2;
    double best = 1e300;
    if ((rc = probe(h, nsys, offsets, m, r, v, dt, probe_steps, G, stream, reps, &best)))
        return restore(rc);
    for (const int wpc : {4, 8, 16}) {
        if (wpc == h->batch_waves_per_cu) continue;
        const int keep = h->batch_waves_per_cu;
        h->batch_waves_per_cu = wpc;
        double t;
        if ((rc = probe(h, nsys, offsets, m, r, v, dt, probe_steps, G, stream, reps, &t)))
            return restore(rc);
        if (t < best) best = t;
        else h->batch_waves_per_cu = keep;
    }
    int chosen[NBUCKET] = {-1, -1, -1, -1}, chosen_w[NBUCKET] = {0, 0, 0, 0};
    for (int b = 0; b < NBUCKET; ++b) {
        if (!present[b]) continue;
        int keep_group[TILE + 1];
        std::memcpy(keep_group, h->batch_group, sizeof(keep_group));
        int best_p = -1;
        for (int p = 0; p < 3; ++p) {
            set_bucket_policy(h, b, p);
            double t;
            if ((rc = probe(h, nsys, offsets, m, r, v, dt, probe_steps, G, stream, reps, &t)))
                return restore(rc);
            if (t < best) {
                best = t;
                best_p = p;
                std::memcpy(keep_group, h->batch_group, sizeof(keep_group));
            }
        }
        std::memcpy(h->batch_group, keep_group, sizeof(keep_group));
        // then the wavefronts per item, with the chosen lanes
        const int keep_w = batch_width(h, BUCKET_LO[b]);
        int best_w = keep_w;
        for (const int w : {1, 2, 4}) {
            if (w == keep_w) continue;
            set_bucket_width(h, b, w);
            double t;
            if ((rc = probe(h, nsys, offsets, m, r, v, dt, probe_steps, G, stream, reps, &t)))
                return restore(rc);
            if (t < best) {
                best = t;
                best_w = w;
            }
        }
        set_bucket_width(h, b, best_w);
        chosen_w[b] = best_w;
        // the policy the bucket holds now (probed or kept)
        chosen[b] = best_p;
        if (best_p < 0) {
            for (int p = 0; p < 3; ++p) {
                bool same = true;
                for (int n = BUCKET_LO[b]; n <= BUCKET_HI[b]; ++n) {
                    const int lanes = h->batch_group[n] ? h->batch_group[n] : n; // 0: dense
                    same = same && lanes == policy_group(p, n);
                }
                if (same) {
                    chosen[b] = p;
                    break;
                }
            }
        }
    }
    // record the choice in the handle's table for this device
    std::string arch;
    int cus;
    device_identity(h->device, arch, cus);
    for (int b = 0; b < NBUCKET; ++b) {
        if (chosen[b] < 0) continue;
        bool found = false;
        for (auto &e : h->batch_table)
            if (e.arch == arch && e.cus == cus && e.bucket == b) {
                e.policy = chosen[b];
                e.waves_per_cu = h->batch_waves_per_cu;
                e.width = chosen_w[b];
                found = true;
            }
        if (!found)
            h->batch_table.push_back(
                {arch, cus, b, chosen[b], h->batch_waves_per_cu, chosen_w[b]});
    }
    if (best_ms) *best_ms = best;
    return SAKURA_OK;
}

int sakura_batch_table_save(const sakura_t *h, const char *path)
{
    if (!h || !path) return SAKURA_EINVAL;
    FILE *f = std::fopen(path, "w");
    if (!f) return SAKURA_EINVAL;
    std::fprintf(f, "# sakura batched packing table: arch cus bucket(1-8,9-16,17-32,33-64) "
                    "policy(0 dense,1 even,2 pow2) waves_per_cu wavefronts_per_item(1,2,4)\n");
    for (const auto &e : h->batch_table)
        std::fprintf(f, "%s %d %d %d %d %d\n", e.arch.c_str(), e.cus, e.bucket, e.policy,
                     e.waves_per_cu, e.width);
    return std::fclose(f) == 0 ? SAKURA_OK : SAKURA_EINVAL;
}

int sakura_batch_table_load(sakura_t *h, const char *path)
{
    if (!h || !path) return SAKURA_EINVAL;
    h->err.clear();
    FILE *f = std::fopen(path, "r");
    if (!f) return sk::fail(h, SAKURA_EINVAL, std::string("cannot open ") + path);
    std::vector<sakura::BatchTuneEntry> rows;
    char line[512];
    int bad = 0;
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[128];
        int cus, b, p, w, iw;
        if (std::sscanf(line, "%127s %d %d %d %d %d", arch, &cus, &b, &p, &w, &iw) != 6 ||
            b < 0 || b >= NBUCKET || p < 0 || p > 2 || w < 1 || w > 32 ||
            (iw != 1 && iw != 2 && iw != 4)) {
            bad = 1;
            break;
        }
        rows.push_back({arch, cus, b, p, w, iw});
    }
    std::fclose(f);
    if (bad) return sk::fail(h, SAKURA_EINVAL, std::string("malformed table line in ") + path);
    for (const auto &r : rows) {
        bool found = false;
        for (auto &e : h->batch_table)
            if (e.arch == r.arch && e.cus == r.cus && e.bucket == r.bucket) {
                e = r;
                found = true;
            }
        if (!found) h->batch_table.push_back(r);
    }
    apply_table(h);
    return SAKURA_OK;
}

int sakura_batch_set_group(sakura_t *h, int n, int lanes)
{
    if (!h || n < 1 || n > sk::TILE || lanes < n || lanes > sk::TILE) return SAKURA_EINVAL;
    h->batch_group[n] = lanes;
    return SAKURA_OK;
}

int sakura_batch_set_width(sakura_t *h, int n, int waves)
{
    if (!h || n < 1 || n > sk::TILE || (waves != 1 && waves != 2 && waves != 4))
        return SAKURA_EINVAL;
    h->batch_width[n] = waves;
    return SAKURA_OK;
}

} // extern "C"
