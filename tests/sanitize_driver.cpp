// CPU driver for the sanitizer build (tests/test_sanitize.py): runs the
// oracle's entry points and the host build of the device pair solver on small
// seeded inputs, ragged and edge-case sizes included, so that AddressSanitizer
// and UndefinedBehaviorSanitizer see every loop and branch they take.  Input
// generation only (a splitmix64 stream); it computes nothing of the method.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../oracle/sakura_oracle.h"

extern "C" void host_pair_flow(int64_t n, const double *tau, const double *mu, const double *x,
                               const double *w, int general, double *coef, int *iters,
                               unsigned *status);

namespace {
uint64_t g_state = 0x5aced1a7ull;
double uniform() // splitmix64 -> [0, 1)
{
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-53;
}
double sym() { return 2.0 * uniform() - 1.0; }

struct System {
    std::vector<double> m, r, v;
};
System cloud(int n, double massless_fraction)
{
    System s;
    s.m.resize(n);
    s.r.resize(3 * (size_t)n);
    s.v.resize(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        s.m[i] = uniform() < massless_fraction ? 0.0 : (0.5 + uniform()) / n;
        for (int c = 0; c < 3; ++c) {
            s.r[3 * i + c] = sym();
            s.v[3 * i + c] = 0.3 * sym();
        }
    }
    return s;
}

int fails = 0;
void check(int rc, int want, const char *what)
{
    if (rc != want) {
        std::fprintf(stderr, "%s returned %d, expected %d\n", what, rc, want);
        ++fails;
    }
}
} // namespace

int main()
{
    double sum = 0.0;
    for (int n : {2, 3, 17, 65}) {
        for (double mf : {0.0, 0.3}) {
            System s = cloud(n, mf);
            const double tau = 1e-2;
            check(sref_step(n, s.m.data(), s.r.data(), s.v.data(), tau, 1.0, SREF_SOLVER_KEPLER),
                  0, "sref_step");
            check(sref_step(n, s.m.data(), s.r.data(), s.v.data(), -tau, 1.0,
                            SREF_SOLVER_KEPLER_LITERAL), 0, "sref_step literal");
            check(sref_step(n, s.m.data(), s.r.data(), s.v.data(), tau, 1.0, SREF_SOLVER_DKD), 0,
                  "sref_step dkd");
            for (int scheme = 0; scheme < 3; ++scheme)
                check(sref_evolve_scheme(n, s.m.data(), s.r.data(), s.v.data(), tau, 2, 1.0,
                                         scheme), 0, "sref_evolve_scheme");
            int64_t nk = 0;
            check(sref_step_hybrid(n, s.m.data(), s.r.data(), s.v.data(), tau, 1.0, 0.05, &nk), 0,
                  "sref_step_hybrid");
            std::vector<int64_t> rows = {0, n - 1};
            std::vector<double> ro(6), vo(6);
            check(sref_step_rows(n, s.m.data(), s.r.data(), s.v.data(), tau, 1.0, 2, rows.data(),
                                 ro.data(), vo.data()), 0, "sref_step_rows");
            check(sref_step_rows_hybrid(n, s.m.data(), s.r.data(), s.v.data(), tau, 1.0, 0.05, 2,
                                        rows.data(), ro.data(), vo.data()), 0,
                  "sref_step_rows_hybrid");
            double e[12];
            check(sref_energy(n, s.m.data(), s.r.data(), s.v.data(), 1.0, e), 0, "sref_energy");
            for (double x : s.r) sum += x;
            sum += e[0] + (double)nk;
        }
    }
    // error paths: bad arguments and coincident particles
    {
        System s = cloud(4, 0.0);
        check(sref_step(0, s.m.data(), s.r.data(), s.v.data(), 1e-2, 1.0, 0), SREF_EINVAL,
              "sref_step n=0");
        check(sref_step(4, s.m.data(), s.r.data(), s.v.data(), NAN, 1.0, 0), SREF_EINVAL,
              "sref_step dt=nan");
        for (int c = 0; c < 3; ++c) {
            s.r[3 + c] = s.r[c];
            s.v[3 + c] = s.v[c];
        }
        check(sref_step(4, s.m.data(), s.r.data(), s.v.data(), 1e-2, 1.0, 0), SREF_ECOLLIDE,
              "sref_step collision");
    }
    // Kepler flows of every kind: oracle and the host-built device solver
    const int nk = 4000;
    std::vector<double> tau(nk), mu(nk), x(3 * nk), w(3 * nk), coef(4 * nk);
    std::vector<int> it(nk);
    std::vector<unsigned> st(nk);
    for (int k = 0; k < nk; ++k) {
        mu[k] = std::pow(10.0, -6.0 + 6.0 * uniform());
        const double r0 = std::pow(10.0, -3.0 + 3.0 * uniform());
        const double vesc = std::sqrt(2.0 * mu[k] / r0);
        const double vv = vesc * (0.05 + 2.0 * uniform());
        for (int c = 0; c < 3; ++c) {
            x[3 * k + c] = r0 * sym();
            w[3 * k + c] = vv * sym();
        }
        tau[k] = (k % 7 == 0 ? 0.0 : sym()) * std::pow(10.0, -4.0 + 4.0 * uniform());
        double x1[3], w1[3], cf[4];
        int iters = 0;
        const int rc = sref_kepler(tau[k], mu[k], &x[3 * k], &w[3 * k], x1, w1, cf, &iters);
        if (rc == 0) sum += cf[0] + cf[2];
        double feat[8], y = 0.0;
        int dom = 0;
        const double domain[4] = {0.25, 64.0, -1.0, 3.0};
        sref_guess_sample(tau[k], mu[k], &x[3 * k], &w[3 * k], domain, feat, &y, &dom);
        sum += dom ? y : 0.0;
    }
    host_pair_flow(nk, tau.data(), mu.data(), x.data(), w.data(), 0, coef.data(), it.data(),
                   st.data());
    host_pair_flow(nk, tau.data(), mu.data(), x.data(), w.data(), 1, coef.data(), it.data(),
                   st.data());
    for (int k = 0; k < nk; ++k) sum += coef[4 * k + 2] + it[k];
    // the reference network
    std::vector<double> p(SREF_MLP_PARAMS), xb(8 * 33), yb(33), out(33), grad(SREF_MLP_PARAMS);
    for (double &q : p) q = 0.2 * sym();
    for (double &q : xb) q = sym();
    for (double &q : yb) q = sym();
    double loss = 0.0;
    check(sref_mlp_forward(p.data(), 33, xb.data(), out.data()), 0, "sref_mlp_forward");
    check(sref_mlp_loss_grad(p.data(), 33, xb.data(), yb.data(), &loss, grad.data()), 0,
          "sref_mlp_loss_grad");
    sum += loss + out[0] + sref_stumpff_c2(-3.0) + sref_stumpff_c3(50.0);
    std::printf("checksum %.17g\n", sum);
    if (fails) return 1;
    std::printf("SANITIZED_RUN_OK\n");
    return 0;
}
