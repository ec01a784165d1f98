// Shared declarations of the Sakura HIP library: status bits and device
// counters, wavefront helpers, the handle and host-side helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sakura.h"
#include "kepler_device.hpp"
#include "guess_device.hpp"

namespace sk {

constexpr int TILE = 64; // particles per block = lanes per wavefront

enum : unsigned { ST_NONFINITE = 1u, ST_COLLIDE = 2u, ST_NOCONV = 4u, ST_INVAL = 8u };

struct DevCounters {
    unsigned status; // ST_* bits
    unsigned iters_max;
    unsigned long long pair_solves;
    unsigned long long iters_total;
    unsigned long long fallbacks;
    long long failed_step;
    unsigned hist[32];
    unsigned work_next;  // work-queue head of the batched kernel (one-wavefront items)
    unsigned work_next2; // the same for the two-wavefront items
    unsigned work_next4; // and for the four-wavefront items
    unsigned long long dom_pairs, dom_iters; // solves in the starter network's domain
    unsigned long long learned, restarts;    // network starters used; restarts from the plain one
    unsigned defer_ntiles, defer_next;       // deferred-pair list of the current step
    unsigned long long kicks;                // close-pair hybrid: pairs given the eq. (28) kick
    unsigned resid_bits;                     // largest relative Kepler residual (float bits)
};

// Iteration statistics are added into NSLOT counter slots of one cache line
// each (slot = workgroup index mod NSLOT), so that tens of thousands of
// wavefronts never serialise on one address; k_fold_stats sums the slots.
constexpr int NSLOT = 1024;
struct SlotStats {
    unsigned long long pair_solves, iters_total, fallbacks;
    unsigned iters_max;
    unsigned learned, restarts;
    unsigned resid_bits; // largest relative Kepler residual, as the bits of a float >= 0
    unsigned long long dom_pairs, dom_iters;
    unsigned long long kicks;
};
static_assert(sizeof(SlotStats) == 64, "one cache line per slot");

__device__ inline void slot_add(SlotStats *slots, unsigned block, unsigned long long solves,
                                unsigned long long iters, unsigned long long fb, unsigned imax)
{
    SlotStats *sl = slots + (block & (NSLOT - 1));
    atomicAdd(&sl->pair_solves, solves);
    atomicAdd(&sl->iters_total, iters);
    atomicAdd(&sl->fallbacks, fb);
    atomicMax(&sl->iters_max, imax);
}

// Starter statistics: solves in the network's domain and their evaluations,
// network starters used, restarts from the plain starter.
struct GuessCount {
    unsigned long long dom = 0, dom_iters = 0;
    unsigned learned = 0, restarts = 0;
};

__device__ inline void slot_add_guess(SlotStats *slots, unsigned block, const GuessCount &g)
{
    SlotStats *sl = slots + (block & (NSLOT - 1));
    if (g.dom) {
        atomicAdd(&sl->dom_pairs, g.dom);
        atomicAdd(&sl->dom_iters, g.dom_iters);
    }
    if (g.learned) atomicAdd(&sl->learned, g.learned);
    if (g.restarts) atomicAdd(&sl->restarts, g.restarts);
}

__device__ inline void slot_add_kicks(SlotStats *slots, unsigned block, unsigned long long k)
{
    if (k) atomicAdd(&slots[block & (NSLOT - 1)].kicks, k);
}

// Non-negative floats order as their bit patterns do, so the largest residual
// is an unsigned maximum.
__device__ inline void slot_max_resid(SlotStats *slots, unsigned block, unsigned bits)
{
    if (bits) atomicMax(&slots[block & (NSLOT - 1)].resid_bits, bits);
}

__device__ inline unsigned wave_sum(unsigned x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ inline unsigned wave_max(unsigned x)
{
    for (int o = 32; o > 0; o >>= 1) x = max(x, (unsigned)__shfl_xor(x, o, 64));
    return x;
}
__device__ inline unsigned wave_or(unsigned x)
{
    for (int o = 32; o > 0; o >>= 1) x |= (unsigned)__shfl_xor(x, o, 64);
    return x;
}
__device__ inline double wave_sum_d(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ inline void record_error(DevCounters *c, unsigned bits, long long step)
{
    atomicOr(&c->status, bits);
    atomicMin(&c->failed_step, step);
}

__global__ void k_clear(DevCounters *c, SlotStats *slots);
__global__ void k_fold_stats(const SlotStats *slots, DevCounters *c);

} // namespace sk

struct sakura {
    int device = 0;
    int cus = 256; // compute units of the device
    sakura_opts opts{};
    std::string err;
    double *state = nullptr; // [10][np]
    int64_t cap_np = 0;
    double *part = nullptr; // [nb][nb][6][64]
    int64_t cap_part = 0;
    double *scratch_e = nullptr; // energy partials
    int64_t cap_e = 0;
    sk::DevCounters *cnt = nullptr;
    sk::SlotStats *slots = nullptr;
    sk::DevCounters *host_cnt = nullptr; // pinned
    double *host_out = nullptr;          // pinned, 12 doubles
    std::vector<hipEvent_t> events;
    // batched ensembles
    double *batch_state = nullptr; // staged r, v of all systems
    int64_t cap_batch = 0;
    int *batch_work = nullptr; // work items and the sorted system order
    int64_t cap_work = 0;
    int64_t *batch_offsets = nullptr;
    int64_t cap_offsets = 0;
    std::vector<int> host_work;
    // the packing last uploaded to batch_work and batch_offsets, and what it
    // was made from: the systems' offsets, the lanes and widths per system
    // size, the override, the device buffer it went to
    std::vector<int64_t> plan_offsets;
    int plan_group[65] = {0}, plan_width[65] = {0};
    int plan_override = -1, plan_nitems = 0, plan_nw[3] = {0, 0, 0};
    const int *plan_dev = nullptr;
    hipStream_t capture_stream = nullptr;
    hipStream_t capture_stream2 = nullptr; // further branches of the captured batch graph
    hipStream_t capture_stream3 = nullptr;
    hipEvent_t graph_fork = nullptr, graph_join = nullptr, graph_join2 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::string graph_key;
    int batch_group[65] = {0}; // lanes per system of each size (0: the size itself)
    int batch_width[65] = {0}; // wavefronts per work item by system size (0: the default)
    double *tune_rv = nullptr; // autotuner scratch copies of r, v
    int64_t cap_tune = 0;
    int batch_waves_per_cu = 16;
    int batch_no_graph = 0;
    // packing table: per (gfx arch, compute units, system-size bucket) the
    // lane policy and grid size that sakura_autotune_batch chose or a table
    // file supplied
    struct BatchTuneEntry {
        std::string arch;
        int cus, bucket, policy, waves_per_cu, width;
    };
    std::vector<BatchTuneEntry> batch_table;
    // learned starter
    void *net_buf = nullptr;      // packed bf16 fragments and fp32 vectors of the network
    int2 *defer_pairs = nullptr;  // deferred-pair lists of the tile kernel
    int64_t cap_defer = 0;
    int *defer_idx = nullptr;     // per-tile counts, then the compact tile list
    int64_t cap_defer_idx = 0;
    bool has_model = false;
    double hybrid_eta = 0.0;      // close-pair hybrid threshold (0: every pair by Kepler)
    unsigned model_gen = 0;       // bumped by every model load (graph keys)
    kep::GuessNet net{};          // the loaded network (domain of the model)
    // harvest
    bool harvesting = false;
    kep::GuessNet harvest{};      // domain and row buffer of the harvest
    unsigned long long *row_count = nullptr;
    // device address of the allocation-free entry point's static scratch on
    // this handle's device (null, with the reason, if it could not be resolved)
    void *noalloc_scratch = nullptr;
    std::string noalloc_err;
    // network training scratch
    float *mlp_buf = nullptr;
    int64_t cap_mlp = 0;
    double *mlp_part = nullptr;
    int64_t cap_mlp_part = 0;
};

namespace sk {

inline int fail(sakura_t *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    return code;
}

#define SAKURA_HIP(h, call)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return sk::fail((h), SAKURA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
int grow(sakura_t *h, T **buf, int64_t *cap, int64_t need)
{
    if (*cap >= need) return SAKURA_OK;
    if (*buf) {
        SAKURA_HIP(h, hipFree(*buf));
        *buf = nullptr;
        *cap = 0;
    }
    if (hipMalloc((void **)buf, (size_t)need * sizeof(T)) != hipSuccess) {
        *buf = nullptr;
        return fail(h, SAKURA_ENOMEM, "device allocation of " +
                                          std::to_string((size_t)need * sizeof(T)) +
                                          " bytes failed");
    }
    *cap = need;
    return SAKURA_OK;
}

// The single-system path keeps 10 np doubles of state and nb^2 blocks of
// 6 x 64 doubles of partial sums (np = 64 nb >= n); n whose buffers exceed the
// device's memory (or the 2^21 of the tile grid's int indexing) is EINVAL.
inline int check_size(sakura_t *h, int64_t n)
{
    if (n > ((int64_t)1 << 21))
        return fail(h, SAKURA_EINVAL, "n = " + std::to_string(n) + " exceeds 2^21");
    return SAKURA_OK;
}

// The partial sums (part_doubles) and the state of n particles must fit the
// device's memory.
inline int check_capacity(sakura_t *h, int64_t n, int64_t part_doubles)
{
    const int64_t nb = (n + TILE - 1) / TILE;
    const double need = (double)part_doubles * 8.0 + 10.0 * nb * TILE * 8.0;
    size_t total = 0;
    if (hipDeviceTotalMem(&total, h->device) != hipSuccess) total = 0;
    if (total && need > (double)total)
        return fail(h, SAKURA_EINVAL,
                    "n = " + std::to_string(n) + " needs " + std::to_string(need / 1e9) +
                        " GB of partial sums and state; the device holds " +
                        std::to_string((double)total / 1e9) + " GB");
    return SAKURA_OK;
}

// Starter mode of the next launch: -1 learned requested without a model,
// 0 plain, 1 plain with domain statistics (a model is loaded), 2 the
// network's starter, 3 harvest.  *net receives the kernel argument.
inline int guess_mode(const sakura_t *h, kep::GuessNet *net)
{
    if (h->harvesting) {
        *net = h->harvest;
        return 3;
    }
    if (h->opts.guess == SAKURA_GUESS_LEARNED) {
        if (!h->has_model) return -1;
        *net = h->net;
        return 2;
    }
    if (h->has_model) {
        *net = h->net;
        return 1;
    }
    *net = kep::GuessNet{};
    return 0;
}

inline void guess_stats(const DevCounters &c, sakura_stats *st)
{
    st->guess_domain_pairs = c.dom_pairs;
    st->guess_domain_iters = c.dom_iters;
    st->guess_learned = c.learned;
    st->guess_restarts = c.restarts;
    st->pair_kicks = c.kicks;
    float r;
    std::memcpy(&r, &c.resid_bits, sizeof(r));
    st->max_rel_residual = r;
}

inline int status_code(unsigned st)
{
    if (st & ST_INVAL) return SAKURA_EINVAL;
    if (st & ST_NONFINITE) return SAKURA_ENONFINITE;
    if (st & ST_COLLIDE) return SAKURA_ECOLLIDE;
    if (st & ST_NOCONV) return SAKURA_ENOCONV;
    return SAKURA_OK;
}

inline const char *status_text(int code)
{
    switch (code) {
    case SAKURA_EINVAL: return "negative mass";
    case SAKURA_ENONFINITE: return "non-finite position, velocity or mass";
    case SAKURA_ECOLLIDE: return "two particles at zero separation (no softening)";
    case SAKURA_ENOCONV: return "a Kepler solve did not converge";
    default: return "";
    }
}

} // namespace sk
