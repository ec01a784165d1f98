// Learned Kepler starter: domain test, inputs and the fused network evaluation
// on MFMA (an extension of the method; the paper's solver needs only some
// starting value of the universal variable).
//
// A Kepler problem over time t is fixed, up to scale, by three numbers:
//   tau' = |t| sqrt(mu / r0^3),  e' = sgn(t) (x0.w0) / sqrt(mu r0),
//   b'   = beta r0 / mu = 2 - r0 |w0|^2 / mu,
// (t after the bound-orbit period reduction).  The network maps eight inputs
// built from them,
//   {log2 tau', e', b', tau', e' tau', tau'^2 (3 e'^2 - 1 + b') / 6,
//    tau' max(b',0)^(3/2), e' max(b',0)^(1/2)},
// each shifted and scaled, through 8 -> 64 -> 64 -> 1 (ReLU) to
// y = log(s r0 / t), the log of the root over its free-drift value; the
// starter is then s = (t / r0) exp(y).  y is even under time reversal, which
// is why e' carries the sign of t.
//
// Fused evaluation, one wavefront = 64 pairs.  Layer 1 is H1^T = W1 X^T on
// v_mfma_f32_32x32x8_bf16 (hidden units as rows, pairs as columns, 2 x 2
// blocks of 32 x 32), layer 2 is H2^T = W2 H1^T on v_mfma_f32_32x32x16_bf16
// (K = 64 in four chunks of 16).  The 32 x 32 accumulator layout -- lane l holds
// column l mod 32 and, in register i, row 8 (i / 4) + 4 (l / 32) + i mod 4 --
// gives every lane 16 hidden values of one pair, which after bias, ReLU and
// conversion to bf16 are exactly the lane's B operand of layer 2 once the
// K index is permuted the same way in the A operand (W2, prepacked on the host
// in that order).  Layer 3 is a 64-term dot product on the VALU plus one
// cross-half lane exchange.  Weights are read from global memory (L1/L2
// resident, 10 KB); the whole evaluation runs only for wavefronts that hold a
// pair in the domain.
#pragma once

#include "kepler_device.hpp"

namespace kep {

typedef short v4s_t __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));
typedef float v16f_t __attribute__((ext_vector_type(16)));

constexpr int NET_IN = 8, NET_H = 64;

// Kernel argument: the loaded network, its scaling, the domain, and the
// harvest buffer (rows of HARVEST_ROW floats).
constexpr int HARVEST_ROW = 12;
struct GuessNet {
    const v4s_t *w1f;  // [2][64] layer-1 A fragments (4 bf16 each)
    const v8bf_t *w2f; // [2][4][64] layer-2 A fragments (8 bf16 each)
    const float *b1, *b2, *w3; // [64] each, fp32
    float b3;
    float in_shift[NET_IN], in_scale[NET_IN];
    float out_shift, out_scale;
    double tau2_lo, tau2_hi, b_lo, e2_hi; // domain: tau'^2 range, b' >= b_lo, e'^2 <= e2_hi
    double tau4_lo;                       // tau_lo^4, for the pre-test of pair_may_qualify
    float *rows;                          // harvest rows (device)
    unsigned long long *row_count;        // rows offered so far (device)
    long long row_cap;
    int2 *defer_pairs; // [tiles][DEFER_CAP] pairs (i, j) listed by the tile kernel
    int *defer_count;  // [tiles] entries of each listed tile
    int *defer_tiles;  // compact list of the tiles with entries
};
constexpr int DEFER_CAP = 16; // listed pairs per 64 x 64 tile and step

// Domain test without divisions or square roots: tau'^2 = u^2 mu / r0,
// b' >= b_lo  <=>  beta r0 >= b_lo mu,  e'^2 <= e_hi^2  <=>  eta^2 <= e_hi^2 mu r0.
SAKURA_HD inline bool in_domain(double tau2_lo, double tau2_hi, double b_lo, double e2_hi,
                                double mu, double r0, double r0inv, double eta, double beta,
                                double u)
{
    const double mr = mu * r0inv;
    const double tau2 = u * u * mr;
    return mu > 0.0 && u != 0.0 && tau2 >= tau2_lo && tau2 <= tau2_hi &&
           beta * r0 >= b_lo * mu && eta * eta <= e2_hi * mu * r0;
}
SAKURA_HD inline bool guess_domain(const GuessNet &g, double mu, double r0, double r0inv,
                                   double eta, double beta, double u)
{
    return in_domain(g.tau2_lo, g.tau2_hi, g.b_lo, g.e2_hi, mu, r0, r0inv, eta, beta, u);
}

#ifndef SAKURA_HOST_ONLY
// Plain starter with domain membership (statistics of the pairs a network
// would start), used out of line by kepler_flow_domain.
template <bool RESID = false>
struct DomainOnly {
    static constexpr bool active = true;
    static constexpr bool resid = RESID;
    double tau2_lo, tau2_hi, b_lo, e2_hi;
    bool in_dom = false;

    __device__ int start(double, double mu, double r0, double r0inv, double eta, double beta,
                         double u, double, double, double &)
    {
        in_dom = in_domain(tau2_lo, tau2_hi, b_lo, e2_hi, mu, r0, r0inv, eta, beta, u);
        return START_PLAIN;
    }
    __device__ void done(double, double, double, double, double, double, double, int) {}
};

// The plain flow with domain membership in the result (PairFlow::in_dom),
// kept out of line like the plain kepler_flow; all arguments are values, so
// the policy stays in registers.  RESID: also the residual at the root.
template <bool RESID = false>
__device__ __attribute__((noinline)) PairFlow
kepler_flow_domain(double tau, double mu, double x0, double x1, double x2, double w0, double w1,
                   double w2, double r0sq, const KeplerParams &kp, double tau2_lo,
                   double tau2_hi, double b_lo, double e2_hi)
{
    DomainOnly<RESID> pol{tau2_lo, tau2_hi, b_lo, e2_hi};
    PairFlow f = kepler_flow(tau, mu, x0, x1, x2, w0, w1, w2, r0sq, kp, pol);
    f.in_dom = pol.in_dom;
    return f;
}
#endif

// The eight raw inputs (before shift and scale).
SAKURA_HD inline void guess_inputs(double mu, double r0, double r0inv, double eta, double beta,
                                   double t, double u, float f[NET_IN])
{
    const double mr = mu * r0inv;
    const double taup = fabs(u) * sqrt_step(mr);         // |t| sqrt(mu / r0^3)
    const double rs = rsqrt_refined(mu * r0);             // 1 / sqrt(mu r0)
    const double ep = (t > 0.0 ? eta : -eta) * rs;
    const double bp = beta * r0 * rcp_step(mu);
    const float tf = (float)taup, ef = (float)ep, bf = (float)bp;
    const float bpos = fmaxf(bf, 0.0f), sb = sqrtf(bpos);
    f[0] = log2f(tf);
    f[1] = ef;
    f[2] = bf;
    f[3] = tf;
    f[4] = ef * tf;
    f[5] = tf * tf * (3.0f * ef * ef - 1.0f + bf) * (1.0f / 6.0f);
    f[6] = tf * bpos * sb;
    f[7] = ef * sb;
}

#ifndef SAKURA_HOST_ONLY
// Network output for this lane's pair.  Every lane of the wavefront must call
// it together (MFMA operands come from all 64 lanes); f need only be finite.
__device__ inline float guess_net_eval(const GuessNet &g, const float f[NET_IN])
{
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5; // half of the wavefront

    // Inputs 4h..4h+3 of the own pair, and the other half of the inputs, which
    // the partner lane (lane ^ 32) needs: lane l supplies, for pair block nb,
    // inputs 4h..4h+3 of pair 32 nb + (l mod 32) -- its own pair when nb = h,
    // the partner's pair otherwise.
    float xs[NET_IN];
#pragma unroll
    for (int k = 0; k < NET_IN; ++k) xs[k] = (f[k] - g.in_shift[k]) * g.in_scale[k];
    v4s_t own, send;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float a = h ? xs[4 + k] : xs[k];
        const float b = h ? xs[k] : xs[4 + k];
        own[k] = __builtin_bit_cast(short, (__bf16)a);
        send[k] = __builtin_bit_cast(short, (__bf16)b);
    }
    const int s01 = (int)((unsigned short)send[0] | ((unsigned)(unsigned short)send[1] << 16));
    const int s23 = (int)((unsigned short)send[2] | ((unsigned)(unsigned short)send[3] << 16));
    const int r01 = __shfl_xor(s01, 32, 64);
    const int r23 = __shfl_xor(s23, 32, 64);
    v4s_t oth;
    oth[0] = (short)(r01 & 0xffff);
    oth[1] = (short)((unsigned)r01 >> 16);
    oth[2] = (short)(r23 & 0xffff);
    oth[3] = (short)((unsigned)r23 >> 16);

    // rows of the accumulator registers of this lane within a 32-row block
    // (register i -> row 8 (i / 4) + 4 h + i mod 4): base pointers offset by 4h
    const float *b1h = g.b1 + 4 * h, *b2h = g.b2 + 4 * h, *w3h = g.w3 + 4 * h;
    const v4s_t w1a = g.w1f[lane], w1b = g.w1f[64 + lane];

    float result = 0.0f;
    // one pair block at a time, and weight loads kept next to their use
    // (compiler-only fences), to bound the registers the evaluation needs
#pragma unroll 1
    for (int nb = 0; nb < 2; ++nb) {
        asm volatile("" ::: "memory");
        const v4s_t xb = (nb == h) ? own : oth;
        // layer 1, then bias, ReLU and bf16: the B operands of layer 2
        // (chunk c = hidden rows 16c..16c+15)
        const v16f_t zero = {};
        v8bf_t bfrag[4];
        {
            const v16f_t a0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(w1a, xb, zero, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int r0 = 8 * (j >> 2) + (j & 3), r1 = 16 + r0;
                bfrag[0][j] = (__bf16)fmaxf(a0[j] + b1h[r0], 0.0f);
                bfrag[1][j] = (__bf16)fmaxf(a0[8 + j] + b1h[r1], 0.0f);
            }
        }
        asm volatile("" ::: "memory");
        {
            const v16f_t a1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(w1b, xb, zero, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int r0 = 32 + 8 * (j >> 2) + (j & 3), r1 = 16 + r0;
                bfrag[2][j] = (__bf16)fmaxf(a1[j] + b1h[r0], 0.0f);
                bfrag[3][j] = (__bf16)fmaxf(a1[8 + j] + b1h[r1], 0.0f);
            }
        }
        float part = 0.0f;
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) {
            asm volatile("" ::: "memory");
            v16f_t c = zero;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g.w2f[(mo * 4 + ch) * 64 + lane],
                                                            bfrag[ch], c, 0, 0, 0);
            asm volatile("" ::: "memory");
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int row = 32 * mo + 8 * (i >> 2) + (i & 3);
                part = fmaf(w3h[row], fmaxf(c[i] + b2h[row], 0.0f), part);
            }
        }
        part += __shfl_xor(part, 32, 64);
        if (nb == h) result = part + g.b3;
    }
    return result;
}

// Necessary condition for the domain, from the unreduced tau and |x0|^2 only:
// tau'^2 >= tau_lo^2 with |t| <= |tau| reads tau^4 mu^2 >= tau_lo^4 r0^6.
SAKURA_HD inline bool pair_may_qualify(const GuessNet &g, double tau, double mu, double r0sq)
{
    const double t2 = tau * tau;
    return mu > 0.0 && t2 * t2 * (mu * mu) >= g.tau4_lo * (r0sq * r0sq * r0sq);
}
// The same test with tau^4 / tau_lo^4 formed once per launch (q4 from
// may_qualify_scale; zero without a model) and widened by 2^-40 so that its
// rounding never drops a pair the test above keeps: mu^2 q4 >= r0^6, with no
// branch (mu = 0 or q4 = 0 fails it for every r0 > 0).
SAKURA_HD inline double may_qualify_scale(const GuessNet &g, double tau)
{
    const double t2 = tau * tau;
    return t2 * t2 / g.tau4_lo * (1.0 + 0x1p-40);
}
SAKURA_HD inline bool pair_may_qualify_q(double q4, double mu, double r0sq)
{
    return mu * mu * q4 >= r0sq * r0sq * r0sq;
}

#ifndef SAKURA_HOST_ONLY
// The network's starter for a pair, or NaN outside the domain: the setup of
// the root search (period reduction, tau', e', b'), the inputs and the fused
// evaluation.  Every lane of the wavefront must call it together; a lane
// without a pair passes mu = 0.  Called ahead of the root search, where little
// else is live, so the evaluation does not raise the search's register use.
__device__ inline double net_starter(const GuessNet &g, double tau, double mu, double x0,
                                     double x1, double x2, double w0, double w1, double w2,
                                     double r0sq)
{
    const bool ok = mu > 0.0 && r0sq > 0.0;
    const double rs = ok ? r0sq : 1.0;
    const double r0inv = rsqrt_refined(rs);
    const double r0 = rs * r0inv;
    const double eta = fma(x0, w0, fma(x1, w1, x2 * w2));
    const double vsq = fma(w0, w0, fma(w1, w1, w2 * w2));
    const double beta = fma(2.0 * mu, r0inv, -vsq);
    double s_half, tshift_mu;
    const double t = reduce_time(tau, mu, beta, s_half, tshift_mu); // as kepler_flow does
    const double u = t * r0inv;
    const bool dom = ok && guess_domain(g, mu, r0, r0inv, eta, beta, u);
    float f[NET_IN];
    guess_inputs(dom ? mu : 1.0, dom ? r0 : 1.0, dom ? r0inv : 1.0, dom ? eta : 0.0,
                 dom ? beta : 1.0, dom ? t : 1.0, dom ? u : 1.0, f);
    const float o = guess_net_eval(g, f);
    return dom ? u * (double)__expf(fmaf(g.out_scale, o, g.out_shift)) : __builtin_nan("");
}
#endif

// Starter policies with a loaded network.  MODE 1: plain starter, domain
// membership recorded; MODE 2: the network's starter (s_net, computed ahead
// by net_starter) for pairs in the domain; MODE 3: plain starter, and every
// pair in the domain appends a harvest row {8 raw inputs, y = log(s r0 / t) at
// the converged root, i, j, evaluations} (the last three as int32 bits).
// RESID: the flow also reports the relative residual at the root (one more
// evaluation; the deferred pairs of the tile kernel and the evaluation kernel).
template <int MODE, bool RESID = (MODE == 2)>
struct NetGuess {
    static constexpr bool active = true;
    static constexpr bool resid = RESID;
    const GuessNet &g;
    int pi, pj;          // particle indices (harvest rows)
    bool in_dom = false; // the pair lies in the network's domain
    bool used = false;   // the network's starter replaced the plain one
    double s_start = 0.0, s_root = 0.0;
    double s_net;        // MODE 2: the network's starter from net_starter (NaN: none)

    __device__ NetGuess(const GuessNet &net, int i, int j, double snet = __builtin_nan(""))
        : g(net), pi(i), pj(j), s_net(snet) {}

    __device__ int start(double t, double mu, double r0, double r0inv, double eta,
                         double beta, double u, double lo, double hi, double &s)
    {
        in_dom = guess_domain(g, mu, r0, r0inv, eta, beta, u);
        s_start = s;
        if (MODE != 2 || !in_dom || !(s_net > lo && s_net < hi)) return START_PLAIN; // also NaN
        s = s_net;
        s_start = s_net;
        used = true;
        return START_REPLACED;
    }

    __device__ void done(double s, double t, double mu, double r0, double r0inv, double eta,
                         double beta, int iters)
    {
        s_root = s;
        if (MODE != 3) return;
        const unsigned long long mask = __ballot(in_dom);
        if (!mask) return;
        const int lane = threadIdx.x & 63;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(g.row_count, (unsigned long long)__popcll(mask));
        base = __shfl(base, 0, 64);
        const unsigned long long below = lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
        const unsigned long long row = base + (unsigned long long)__popcll(below);
        if (!in_dom || row >= (unsigned long long)g.row_cap) return;
        float f[NET_IN];
        const double u = t * r0inv;
        guess_inputs(mu, r0, r0inv, eta, beta, t, u, f);
        float *out = g.rows + row * HARVEST_ROW;
#pragma unroll
        for (int k = 0; k < NET_IN; ++k) out[k] = f[k];
        out[8] = logf((float)(s * rcp_refined(u)));
        out[9] = __int_as_float(pi);
        out[10] = __int_as_float(pj);
        out[11] = __int_as_float(iters);
    }
};
#endif

} // namespace kep
