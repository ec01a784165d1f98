// Learned Kepler starter: model upload (bf16 MFMA fragments), harvest control,
// the evaluation entry point, and the network's training kernels with Adam.
//
// Training runs in fp32 on the vector ALUs, in three kernels per minibatch:
//   k_mlp_sample  one thread per sample: forward pass, loss, backward pass to
//                 the per-sample factors of every weight gradient (A1, A2, D2,
//                 D1, x, dL/do), written to scratch;
//   k_mlp_wgrad   one workgroup per 256 samples: the sums over samples of the
//                 outer products (dW2 = D2^T A1, dW1 = D1^T x, ...), staged
//                 through LDS 32 samples at a time, one partial per workgroup;
//   k_mlp_finish  one thread per parameter: the partials summed in a fixed
//                 order (deterministic), then the Adam update.
// Parameter packing: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
#include "common.hpp"

namespace {
using namespace sk;

constexpr int NIN = 8, NH = 64;
constexpr int P_W1 = 0, P_B1 = 512, P_W2 = 576, P_B2 = 4672, P_W3 = 4736, P_B3 = 4800;
constexpr int NPAR = SAKURA_MLP_PARAMS;
static_assert(P_B3 + 1 == NPAR, "parameter packing");

// Device layout of a loaded network (bytes).
constexpr size_t OFF_W1F = 0, OFF_W2F = 1024, OFF_B1 = 9216, OFF_B2 = 9472, OFF_W3 = 9728,
                 NET_BYTES = 9984;

// float -> bf16, round to nearest even (finite inputs).
uint16_t bf16_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Hidden unit fed by slot j of lane half hh in K-chunk ch of layer 2: the row
// of the layer-1 accumulator register that becomes that slot.
int w2_row(int ch, int hh, int j) { return 32 * (ch >> 1) + 8 * (2 * (ch & 1) + (j >> 2)) + 4 * hh + (j & 3); }

__device__ inline uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// ---------------------------------------------------------------------------
// Evaluation of the pair kernels' root search on independent problems.
template <int MODE>
__global__ __launch_bounds__(TILE) void k_guess_eval(int64_t n, const double *__restrict__ tau,
                                                     const double *__restrict__ mu,
                                                     const double *__restrict__ x0,
                                                     const double *__restrict__ w0,
                                                     double *__restrict__ s_start,
                                                     double *__restrict__ s_root,
                                                     int32_t *__restrict__ info,
                                                     kep::KeplerParams kp, const kep::GuessNet net)
{
    const int64_t k = (int64_t)blockIdx.x * TILE + threadIdx.x;
    const bool valid = k < n;
    double t = 0.0, m = 0.0, x[3] = {1.0, 0.0, 0.0}, w[3] = {0.0, 0.0, 0.0};
    if (valid) {
        t = tau[k];
        m = mu[k];
        for (int c = 0; c < 3; ++c) {
            x[c] = x0[3 * k + c];
            w[c] = w0[3 * k + c];
        }
    }
    const double r0sq = fma(x[0], x[0], fma(x[1], x[1], x[2] * x[2]));
    const bool ok = valid && r0sq > 0.0;
    double s_net = __builtin_nan("");
    if (MODE == 2) {
        const bool cand = ok && kep::pair_may_qualify(net, t, m, r0sq);
        if (__any(cand))
            s_net = kep::net_starter(net, t, cand ? m : 0.0, x[0], x[1], x[2], w[0], w[1], w[2],
                                     r0sq);
    }
    kep::NetGuess<MODE> gp(net, (int)k, 0, s_net);
    const kep::PairFlow f = kep::kepler_flow(ok ? t : 0.0, ok ? m : 0.0, x[0], x[1], x[2], w[0],
                                             w[1], w[2], ok ? r0sq : 1.0, kp, gp);
    if (!valid) return;
    s_start[k] = gp.s_start;
    s_root[k] = gp.s_root;
    info[k] = (gp.in_dom ? 1 : 0) | (gp.used ? 2 : 0) | (f.restarted ? 4 : 0) |
              (f.converged ? 8 : 0) | (min(f.iters, 255) << 8);
}

// ---------------------------------------------------------------------------
// Training kernels.

// One thread per sample b of the minibatch.  The sample is row
// splitmix64(seed, step, b) mod pool of (X, Y) when pool > 0, else row b.
// inv_batch = 1 / B scales dL/do = 2 (o - y) / B.  out (may be null) gets o.
template <bool GRAD>
__global__ __launch_bounds__(256) void k_mlp_sample(int64_t B, const float *__restrict__ params,
                                                    const float *__restrict__ X,
                                                    const float *__restrict__ Y, int64_t pool,
                                                    uint64_t seed, int64_t step, float inv_batch,
                                                    float *__restrict__ out,
                                                    float *__restrict__ A1, float *__restrict__ A2,
                                                    float *__restrict__ D2, float *__restrict__ D1,
                                                    float *__restrict__ XS, float *__restrict__ GS,
                                                    double *__restrict__ loss_part)
{
    __shared__ float w[NPAR];
    __shared__ double red[256];
    for (int p = threadIdx.x; p < NPAR; p += 256) w[p] = params[p];
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0;
    if (b < B) {
        int64_t row = b;
        if (pool > 0)
            row = (int64_t)(splitmix64(seed ^ splitmix64((uint64_t)step * 0x100000001b3ull + (uint64_t)b)) %
                            (uint64_t)pool);
        float x[NIN];
        for (int k = 0; k < NIN; ++k) x[k] = X[row * NIN + k];
        const float y = Y ? Y[row] : 0.0f;
        float a1[NH];
        for (int i = 0; i < NH; ++i) {
            float z = w[P_B1 + i];
            for (int k = 0; k < NIN; ++k) z = fmaf(w[P_W1 + i * NIN + k], x[k], z);
            a1[i] = fmaxf(z, 0.0f);
        }
        float o = w[P_B3];
        unsigned long long mask2 = 0;
        for (int i = 0; i < NH; ++i) {
            float z = w[P_B2 + i];
            for (int j = 0; j < NH; ++j) z = fmaf(w[P_W2 + i * NH + j], a1[j], z);
            const float a2 = fmaxf(z, 0.0f);
            if (z > 0.0f) mask2 |= 1ull << i;
            o = fmaf(w[P_W3 + i], a2, o);
            if (GRAD) A2[b * NH + i] = a2;
        }
        if (out) out[b] = o;
        const float e = o - y;
        e2 = (double)e * (double)e;
        if (GRAD) {
            const float g = 2.0f * e * inv_batch; // dL/do
            GS[b] = g;
            for (int k = 0; k < NIN; ++k) XS[b * NIN + k] = x[k];
            float d1[NH];
            for (int j = 0; j < NH; ++j) d1[j] = 0.0f;
            for (int i = 0; i < NH; ++i) {
                const float d2 = ((mask2 >> i) & 1ull) ? g * w[P_W3 + i] : 0.0f;
                D2[b * NH + i] = d2;
                for (int j = 0; j < NH; ++j) d1[j] = fmaf(w[P_W2 + i * NH + j], d2, d1[j]);
            }
            for (int j = 0; j < NH; ++j) {
                A1[b * NH + j] = a1[j];
                D1[b * NH + j] = a1[j] > 0.0f ? d1[j] : 0.0f;
            }
        }
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_part) loss_part[blockIdx.x] = red[0];
}

// Sums over the 256 samples of one workgroup of the gradient factors; one
// partial gradient per workgroup.
__global__ __launch_bounds__(256) void k_mlp_wgrad(int64_t B, const float *__restrict__ A1,
                                                   const float *__restrict__ A2,
                                                   const float *__restrict__ D2,
                                                   const float *__restrict__ D1,
                                                   const float *__restrict__ XS,
                                                   const float *__restrict__ GS,
                                                   float *__restrict__ part)
{
    constexpr int TS = 32;
    __shared__ float sA1[TS][NH], sA2[TS][NH], sD2[TS][NH], sD1[TS][NH], sX[TS][NIN], sG[TS];
    const int t = threadIdx.x;
    const int i = t >> 2;             // output unit of W2 / W1
    const int jb = (t & 3) * 16;      // 16 inputs of W2
    const int kb = (t & 3) * 2;       // 2 inputs of W1
    float g2[16], g1[2] = {0.0f, 0.0f}, gv = 0.0f;
    for (int k = 0; k < 16; ++k) g2[k] = 0.0f;
    const int64_t s0 = (int64_t)blockIdx.x * 256;
    for (int tile = 0; tile < 256 / TS; ++tile) {
        const int64_t base = s0 + tile * TS;
        __syncthreads();
        for (int e = t; e < TS * NH; e += 256) {
            const int s = e / NH, c = e % NH;
            const bool in = base + s < B;
            const int64_t q = (base + s) * NH + c;
            sA1[s][c] = in ? A1[q] : 0.0f;
            sA2[s][c] = in ? A2[q] : 0.0f;
            sD2[s][c] = in ? D2[q] : 0.0f;
            sD1[s][c] = in ? D1[q] : 0.0f;
        }
        {
            const int s = t / NIN, c = t % NIN; // 256 = TS * NIN
            sX[s][c] = base + s < B ? XS[(base + s) * NIN + c] : 0.0f;
        }
        if (t < TS) sG[t] = base + t < B ? GS[base + t] : 0.0f;
        __syncthreads();
        for (int s = 0; s < TS; ++s) {
            const float d2 = sD2[s][i], d1 = sD1[s][i];
#pragma unroll
            for (int k = 0; k < 16; ++k) g2[k] = fmaf(d2, sA1[s][jb + k], g2[k]);
            g1[0] = fmaf(d1, sX[s][kb], g1[0]);
            g1[1] = fmaf(d1, sX[s][kb + 1], g1[1]);
            if (t < 64) gv += sD1[s][t];
            else if (t < 128) gv += sD2[s][t - 64];
            else if (t < 192) gv = fmaf(sG[s], sA2[s][t - 128], gv);
            else if (t == 192) gv += sG[s];
        }
    }
    float *pp = part + (size_t)blockIdx.x * NPAR;
    for (int k = 0; k < 16; ++k) pp[P_W2 + i * NH + jb + k] = g2[k];
    pp[P_W1 + i * NIN + kb] = g1[0];
    pp[P_W1 + i * NIN + kb + 1] = g1[1];
    if (t < 64) pp[P_B1 + t] = gv;
    else if (t < 128) pp[P_B2 + t - 64] = gv;
    else if (t < 192) pp[P_W3 + t - 128] = gv;
    else if (t == 192) pp[P_B3] = gv;
}

struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2; // c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
};

// Partial gradients summed in chunk order; optionally one Adam step.  Thread 0
// of workgroup 0 also sums the loss partials.
template <bool ADAM>
__global__ __launch_bounds__(256) void k_mlp_finish(int nchunk, const float *__restrict__ part,
                                                    float *__restrict__ grad,
                                                    float *__restrict__ params,
                                                    float *__restrict__ m1, float *__restrict__ m2,
                                                    AdamArgs a, int nloss,
                                                    const double *__restrict__ loss_part,
                                                    double *__restrict__ loss_sum)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss_sum) {
        double s = 0.0;
        for (int k = 0; k < nloss; ++k) s += loss_part[k];
        *loss_sum = s;
    }
    if (p >= NPAR) return;
    double g = 0.0;
    for (int c = 0; c < nchunk; ++c) g += part[(size_t)c * NPAR + p];
    const float gf = (float)g;
    if (grad) grad[p] = gf;
    if (ADAM) {
        const float mm = a.beta1 * m1[p] + (1.0f - a.beta1) * gf;
        const float vv = a.beta2 * m2[p] + (1.0f - a.beta2) * gf * gf;
        m1[p] = mm;
        m2[p] = vv;
        params[p] -= a.lr * (mm * a.c1) / (sqrtf(vv * a.c2) + a.eps);
    }
}

// Per-workgroup sums of the eight inputs, the target and their squares.
__global__ __launch_bounds__(256) void k_row_moments(int64_t n, const float *__restrict__ rows,
                                                     double *__restrict__ part)
{
    __shared__ double red[256];
    double acc[18];
    for (int k = 0; k < 18; ++k) acc[k] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
        for (int k = 0; k < 9; ++k) {
            const double v = rows[r * SAKURA_HARVEST_ROW + k];
            acc[k] += v;
            acc[9 + k] += v * v;
        }
    }
    for (int k = 0; k < 18; ++k) {
        __syncthreads();
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * 18 + k] = red[0];
    }
}

struct Scaling {
    float shift[9], scale[9];
};

// Harvest rows -> scaled network inputs X[n][8] and targets Y[n].
__global__ void k_standardize(int64_t n, const float *__restrict__ rows, Scaling sc,
                              float *__restrict__ X, float *__restrict__ Y)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int k = 0; k < NIN; ++k)
        X[r * NIN + k] = (rows[r * SAKURA_HARVEST_ROW + k] - sc.shift[k]) * sc.scale[k];
    Y[r] = (rows[r * SAKURA_HARVEST_ROW + 8] - sc.shift[8]) * sc.scale[8];
}

// Scratch of a minibatch of B samples inside h->mlp_buf.
struct BatchScratch {
    float *A1, *A2, *D2, *D1, *XS, *GS, *part;
    int nblk, nchunk;
};

size_t batch_floats(int64_t B)
{
    const int64_t nchunk = (B + 255) / 256;
    return (size_t)B * (4 * NH + NIN + 1) + (size_t)nchunk * NPAR;
}

BatchScratch carve(float *p, int64_t B)
{
    BatchScratch s;
    s.nblk = (int)((B + 255) / 256);
    s.nchunk = s.nblk;
    s.A1 = p;
    s.A2 = s.A1 + B * NH;
    s.D2 = s.A2 + B * NH;
    s.D1 = s.D2 + B * NH;
    s.XS = s.D1 + B * NH;
    s.GS = s.XS + B * NIN;
    s.part = s.GS + B;
    return s;
}

bool finite_all(const float *p, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(p[k])) return false;
    return true;
}

bool domain_ok(const double d[4])
{
    for (int k = 0; k < 4; ++k)
        if (std::isnan(d[k])) return false;
    return d[0] >= 0.0 && d[1] >= d[0] && d[3] >= 0.0;
}

void set_domain(kep::GuessNet &g, const double d[4])
{
    g.tau2_lo = d[0] * d[0];
    g.tau4_lo = g.tau2_lo * g.tau2_lo;
    g.tau2_hi = std::isinf(d[1]) ? HUGE_VAL : d[1] * d[1];
    g.b_lo = d[2];
    g.e2_hi = std::isinf(d[3]) ? HUGE_VAL : d[3] * d[3];
}

} // namespace

extern "C" {

int sakura_set_guess_model(sakura_t *h, const void *blob, size_t bytes)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (!blob) {
        h->has_model = false;
        h->net = kep::GuessNet{};
        ++h->model_gen;
        return SAKURA_OK;
    }
    if (bytes != sizeof(sakura_guess_model))
        return fail(h, SAKURA_EINVAL, "model blob of " + std::to_string(bytes) +
                                          " bytes; a sakura_guess_model has " +
                                          std::to_string(sizeof(sakura_guess_model)));
    sakura_guess_model copy;
    std::memcpy(&copy, blob, sizeof(copy));
    const sakura_guess_model *model = &copy;
    if (!finite_all(model->params, NPAR) || !finite_all(model->in_shift, 8) ||
        !finite_all(model->in_scale, 8) || !std::isfinite(model->out_shift) ||
        !std::isfinite(model->out_scale))
        return fail(h, SAKURA_EINVAL, "model holds non-finite values");
    if (!domain_ok(model->domain)) return fail(h, SAKURA_EINVAL, "empty or invalid model domain");
    // bf16 A fragments of layers 1 and 2 in the order the fused evaluation reads
    std::vector<uint8_t> buf(NET_BYTES, 0);
    uint16_t *w1f = reinterpret_cast<uint16_t *>(buf.data() + OFF_W1F);
    for (int mb = 0; mb < 2; ++mb)
        for (int lane = 0; lane < 64; ++lane)
            for (int k = 0; k < 4; ++k) {
                const int row = 32 * mb + (lane & 31), col = 4 * (lane >> 5) + k;
                w1f[(mb * 64 + lane) * 4 + k] = bf16_rne(model->params[P_W1 + row * NIN + col]);
            }
    uint16_t *w2f = reinterpret_cast<uint16_t *>(buf.data() + OFF_W2F);
    for (int mo = 0; mo < 2; ++mo)
        for (int ch = 0; ch < 4; ++ch)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int row = 32 * mo + (lane & 31), col = w2_row(ch, lane >> 5, j);
                    w2f[((mo * 4 + ch) * 64 + lane) * 8 + j] =
                        bf16_rne(model->params[P_W2 + row * NH + col]);
                }
    std::memcpy(buf.data() + OFF_B1, model->params + P_B1, NH * sizeof(float));
    std::memcpy(buf.data() + OFF_B2, model->params + P_B2, NH * sizeof(float));
    std::memcpy(buf.data() + OFF_W3, model->params + P_W3, NH * sizeof(float));
    SAKURA_HIP(h, hipSetDevice(h->device));
    if (!h->net_buf) SAKURA_HIP(h, hipMalloc(&h->net_buf, NET_BYTES));
    SAKURA_HIP(h, hipMemcpy(h->net_buf, buf.data(), NET_BYTES, hipMemcpyHostToDevice));
    kep::GuessNet g{};
    uint8_t *base = static_cast<uint8_t *>(h->net_buf);
    g.w1f = reinterpret_cast<const kep::v4s_t *>(base + OFF_W1F);
    g.w2f = reinterpret_cast<const kep::v8bf_t *>(base + OFF_W2F);
    g.b1 = reinterpret_cast<const float *>(base + OFF_B1);
    g.b2 = reinterpret_cast<const float *>(base + OFF_B2);
    g.w3 = reinterpret_cast<const float *>(base + OFF_W3);
    g.b3 = model->params[P_B3];
    for (int k = 0; k < 8; ++k) {
        g.in_shift[k] = model->in_shift[k];
        g.in_scale[k] = model->in_scale[k];
    }
    g.out_shift = model->out_shift;
    g.out_scale = model->out_scale;
    set_domain(g, model->domain);
    h->net = g;
    h->has_model = true;
    ++h->model_gen;
    return SAKURA_OK;
}

int sakura_set_guess(sakura_t *h, int guess)
{
    if (!h) return SAKURA_EINVAL;
    if (guess != SAKURA_GUESS_ANALYTIC && guess != SAKURA_GUESS_LEARNED)
        return sk::fail(h, SAKURA_EINVAL, "unknown starter");
    h->opts.guess = guess;
    return SAKURA_OK;
}

int sakura_harvest_begin(sakura_t *h, float *rows, int64_t cap, const double domain[4])
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (!rows || cap < 1 || !domain) return fail(h, SAKURA_EINVAL, "null rows/domain or cap < 1");
    if (!domain_ok(domain)) return fail(h, SAKURA_EINVAL, "empty or invalid harvest domain");
    SAKURA_HIP(h, hipSetDevice(h->device));
    if (!h->row_count) SAKURA_HIP(h, hipMalloc((void **)&h->row_count, sizeof(unsigned long long)));
    const unsigned long long zero = 0;
    SAKURA_HIP(h, hipMemcpy(h->row_count, &zero, sizeof(zero), hipMemcpyHostToDevice));
    kep::GuessNet g{};
    set_domain(g, domain);
    g.rows = rows;
    g.row_count = h->row_count;
    g.row_cap = cap;
    h->harvest = g;
    h->harvesting = true;
    return SAKURA_OK;
}

int sakura_harvest_end(sakura_t *h, int64_t *offered)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (!h->harvesting) return fail(h, SAKURA_EINVAL, "no harvest running");
    h->harvesting = false;
    unsigned long long c = 0;
    SAKURA_HIP(h, hipSetDevice(h->device));
    SAKURA_HIP(h, hipDeviceSynchronize());
    SAKURA_HIP(h, hipMemcpy(&c, h->row_count, sizeof(c), hipMemcpyDeviceToHost));
    if (offered) *offered = (int64_t)c;
    return SAKURA_OK;
}

int sakura_guess_eval(sakura_t *h, int64_t n, const double *tau, const double *mu,
                      const double *x0, const double *w0, double *s_start, double *s_root,
                      int32_t *info, void *stream)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (n < 1 || !tau || !mu || !x0 || !w0 || !s_start || !s_root || !info)
        return fail(h, SAKURA_EINVAL, "n < 1 or null pointer");
    if (h->harvesting) return fail(h, SAKURA_EINVAL, "a harvest is running");
    kep::GuessNet net{};
    const int mode = guess_mode(h, &net);
    if (mode < 0) return fail(h, SAKURA_ENOMODEL, "learned starter requested but no model is loaded");
    if (mode == 0) { // no model: nothing is in the domain
        net.tau2_lo = HUGE_VAL;
        net.tau4_lo = HUGE_VAL;
        net.tau2_hi = -1.0;
    }
    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const kep::KeplerParams kp{h->opts.kepler_rtol, h->opts.max_iter};
    const unsigned blocks = (unsigned)((n + TILE - 1) / TILE);
    if (mode == 2)
        k_guess_eval<2><<<blocks, TILE, 0, st>>>(n, tau, mu, x0, w0, s_start, s_root, info, kp, net);
    else
        k_guess_eval<1><<<blocks, TILE, 0, st>>>(n, tau, mu, x0, w0, s_start, s_root, info, kp, net);
    SAKURA_HIP(h, hipGetLastError());
    SAKURA_HIP(h, hipStreamSynchronize(st));
    return SAKURA_OK;
}

int sakura_mlp_forward(sakura_t *h, const float *params, int64_t batch, const float *x,
                       float *out, void *stream)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (batch < 1 || !params || !x || !out) return fail(h, SAKURA_EINVAL, "batch < 1 or null pointer");
    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const unsigned nblk = (unsigned)((batch + 255) / 256);
    k_mlp_sample<false><<<nblk, 256, 0, st>>>(batch, params, x, nullptr, 0, 0, 0, 0.0f, out,
                                              nullptr, nullptr, nullptr, nullptr, nullptr,
                                              nullptr, nullptr);
    SAKURA_HIP(h, hipGetLastError());
    SAKURA_HIP(h, hipStreamSynchronize(st));
    return SAKURA_OK;
}

int sakura_mlp_loss_grad(sakura_t *h, const float *params, int64_t batch, const float *x,
                         const float *y, float *grad, double *loss, void *stream)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (batch < 1 || !params || !x || !y || !grad || !loss)
        return fail(h, SAKURA_EINVAL, "batch < 1 or null pointer");
    if (batch > ((int64_t)1 << 24)) return fail(h, SAKURA_EINVAL, "batch > 2^24");
    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = grow(h, &h->mlp_buf, &h->cap_mlp, (int64_t)batch_floats(batch)))) return rc;
    BatchScratch s = carve(h->mlp_buf, batch);
    if ((rc = grow(h, &h->mlp_part, &h->cap_mlp_part, (int64_t)s.nblk + 1))) return rc;
    double *loss_dev = h->mlp_part + s.nblk;
    k_mlp_sample<true><<<s.nblk, 256, 0, st>>>(batch, params, x, y, 0, 0, 0, 1.0f / (float)batch,
                                               nullptr, s.A1, s.A2, s.D2, s.D1, s.XS, s.GS,
                                               h->mlp_part);
    k_mlp_wgrad<<<s.nchunk, 256, 0, st>>>(batch, s.A1, s.A2, s.D2, s.D1, s.XS, s.GS, s.part);
    k_mlp_finish<false><<<(NPAR + 255) / 256, 256, 0, st>>>(s.nchunk, s.part, grad, nullptr,
                                                            nullptr, nullptr, AdamArgs{}, s.nblk,
                                                            h->mlp_part, loss_dev);
    SAKURA_HIP(h, hipGetLastError());
    double ls = 0.0;
    SAKURA_HIP(h, hipMemcpyAsync(&ls, loss_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    SAKURA_HIP(h, hipStreamSynchronize(st));
    *loss = ls / (double)batch;
    return SAKURA_OK;
}

int sakura_mlp_fit(sakura_t *h, const float *rows, int64_t n, const double domain[4],
                   const sakura_fit_opts *opts, sakura_guess_model *model, float *val_loss,
                   void *stream)
{
    using namespace sk;
    if (!h) return SAKURA_EINVAL;
    h->err.clear();
    if (!rows || !domain || !model || n < 64) return fail(h, SAKURA_EINVAL, "null pointer or n < 64");
    if (!domain_ok(domain)) return fail(h, SAKURA_EINVAL, "empty or invalid domain");
    sakura_fit_opts o{};
    if (opts) o = *opts;
    if (o.epochs <= 0) o.epochs = 20;
    if (o.batch <= 0) o.batch = 4096;
    if (!(o.lr > 0.0f)) o.lr = 3e-3f;
    if (!(o.lr_final > 0.0f)) o.lr_final = 3e-5f;
    if (!(o.val_fraction > 0.0 && o.val_fraction < 0.5)) o.val_fraction = 0.05;
    if (o.batch > (1 << 20)) return fail(h, SAKURA_EINVAL, "batch > 2^20");
    const int64_t n_val = std::max<int64_t>(1, (int64_t)((double)n * o.val_fraction));
    const int64_t n_tr = n - n_val;
    const int64_t B = o.batch;
    SAKURA_HIP(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;

    // scratch: X[n][8], Y[n], params, Adam moments, grad, minibatch factors
    const size_t f_data = (size_t)n * (NIN + 1);
    const size_t f_total = f_data + 4 * (size_t)NPAR + batch_floats(B);
    int rc;
    if ((rc = grow(h, &h->mlp_buf, &h->cap_mlp, (int64_t)f_total))) return rc;
    float *X = h->mlp_buf, *Y = X + (size_t)n * NIN;
    float *P = Y + n, *M1 = P + NPAR, *M2 = M1 + NPAR, *GR = M2 + NPAR;
    BatchScratch s = carve(GR + NPAR, B);
    const int mblk = (int)std::min<int64_t>(1024, (n + 255) / 256);
    if ((rc = grow(h, &h->mlp_part, &h->cap_mlp_part, std::max<int64_t>(18 * mblk, s.nblk + 1))))
        return rc;

    // input and target scaling from the training rows
    k_row_moments<<<mblk, 256, 0, st>>>(n_tr, rows, h->mlp_part);
    SAKURA_HIP(h, hipGetLastError());
    std::vector<double> mom((size_t)18 * mblk);
    SAKURA_HIP(h, hipMemcpyAsync(mom.data(), h->mlp_part, mom.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
    SAKURA_HIP(h, hipStreamSynchronize(st));
    Scaling sc{};
    for (int k = 0; k < 9; ++k) {
        double s1 = 0.0, s2 = 0.0;
        for (int b = 0; b < mblk; ++b) {
            s1 += mom[(size_t)b * 18 + k];
            s2 += mom[(size_t)b * 18 + 9 + k];
        }
        const double mean = s1 / (double)n_tr;
        const double var = std::max(s2 / (double)n_tr - mean * mean, 0.0);
        const double sd = std::sqrt(var);
        if (!std::isfinite(mean) || !std::isfinite(sd))
            return fail(h, SAKURA_EINVAL, "harvest rows hold non-finite values");
        sc.shift[k] = (float)mean;
        sc.scale[k] = (float)(1.0 / std::max(sd, 1e-6 * (1.0 + std::fabs(mean))));
    }
    k_standardize<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, rows, sc, X, Y);

    // initial weights: uniform, He bounds for the ReLU layers (splitmix64 stream)
    std::vector<float> p0(NPAR, 0.0f);
    uint64_t state = o.seed ^ 0x5a4b3c2d1e0f9876ull;
    auto uni = [&state]() {
        uint64_t x = (state += 0x9e3779b97f4a7c15ull);
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        x ^= x >> 31;
        return (double)(x >> 11) * 0x1p-53 * 2.0 - 1.0;
    };
    for (int k = 0; k < NH * NIN; ++k) p0[P_W1 + k] = (float)(uni() * std::sqrt(6.0 / NIN));
    for (int k = 0; k < NH * NH; ++k) p0[P_W2 + k] = (float)(uni() * std::sqrt(6.0 / NH));
    for (int k = 0; k < NH; ++k) p0[P_W3 + k] = (float)(uni() * std::sqrt(3.0 / NH));
    SAKURA_HIP(h, hipMemcpyAsync(P, p0.data(), NPAR * sizeof(float), hipMemcpyHostToDevice, st));
    std::vector<float> zeros(2 * NPAR, 0.0f);
    SAKURA_HIP(h, hipMemcpyAsync(M1, zeros.data(), 2 * NPAR * sizeof(float), hipMemcpyHostToDevice, st));

    const int64_t steps_per_epoch = std::max<int64_t>(1, n_tr / B);
    const int64_t total = steps_per_epoch * o.epochs;
    const float b1 = 0.9f, b2 = 0.999f;
    double b1t = 1.0, b2t = 1.0;
    int64_t step = 0;
    double *loss_dev = h->mlp_part + s.nblk;
    for (int ep = 0; ep < o.epochs; ++ep) {
        for (int64_t k = 0; k < steps_per_epoch; ++k, ++step) {
            b1t *= b1;
            b2t *= b2;
            const double frac = (double)step / (double)std::max<int64_t>(1, total - 1);
            AdamArgs a;
            a.lr = (float)(o.lr_final + 0.5 * (o.lr - o.lr_final) * (1.0 + std::cos(M_PI * frac)));
            a.beta1 = b1;
            a.beta2 = b2;
            a.eps = 1e-8f;
            a.c1 = (float)(1.0 / (1.0 - b1t));
            a.c2 = (float)(1.0 / (1.0 - b2t));
            k_mlp_sample<true><<<s.nblk, 256, 0, st>>>(B, P, X, Y, n_tr, o.seed, step,
                                                       1.0f / (float)B, nullptr, s.A1, s.A2,
                                                       s.D2, s.D1, s.XS, s.GS, nullptr);
            k_mlp_wgrad<<<s.nchunk, 256, 0, st>>>(B, s.A1, s.A2, s.D2, s.D1, s.XS, s.GS, s.part);
            k_mlp_finish<true><<<(NPAR + 255) / 256, 256, 0, st>>>(s.nchunk, s.part, GR, P, M1,
                                                                   M2, a, 0, nullptr, nullptr);
        }
        SAKURA_HIP(h, hipGetLastError());
        // held-out loss, B rows at a time
        double tot = 0.0;
        for (int64_t v0 = 0; v0 < n_val; v0 += B) {
            const int64_t nb = std::min<int64_t>(B, n_val - v0);
            const int blk = (int)((nb + 255) / 256);
            k_mlp_sample<false><<<blk, 256, 0, st>>>(nb, P, X + (size_t)(n_tr + v0) * NIN,
                                                     Y + n_tr + v0, 0, 0, 0, 0.0f, nullptr,
                                                     nullptr, nullptr, nullptr, nullptr, nullptr,
                                                     nullptr, h->mlp_part);
            k_mlp_finish<false><<<1, 256, 0, st>>>(0, s.part, nullptr, nullptr, nullptr, nullptr,
                                                   AdamArgs{}, blk, h->mlp_part, loss_dev);
            double ls = 0.0;
            SAKURA_HIP(h, hipMemcpyAsync(&ls, loss_dev, sizeof(double), hipMemcpyDeviceToHost, st));
            SAKURA_HIP(h, hipStreamSynchronize(st));
            tot += ls;
        }
        if (val_loss) val_loss[ep] = (float)(tot / (double)n_val);
    }
    SAKURA_HIP(h, hipMemcpyAsync(model->params, P, NPAR * sizeof(float), hipMemcpyDeviceToHost, st));
    SAKURA_HIP(h, hipStreamSynchronize(st));
    for (int k = 0; k < 8; ++k) {
        model->in_shift[k] = sc.shift[k];
        model->in_scale[k] = sc.scale[k];
    }
    model->out_shift = sc.shift[8];
    model->out_scale = 1.0f / sc.scale[8];
    for (int k = 0; k < 4; ++k) model->domain[k] = domain[k];
    return SAKURA_OK;
}

} // extern "C"
