// Host build of the device pair solver, for the CPU test of its logic
// (tests/test_solver_host.py).  The hardware reciprocal and reciprocal-square-
// root estimates are modelled by the exact values perturbed by 6e-8 relative
// (beyond the 2^-24.2 measured on gfx950), and a "wavefront" is one lane, so
// every wave-uniform choice of the solver is taken per problem.
#include <cmath>
#include <cstdint>
using std::copysign;
using std::fabs;
using std::fma;
using std::fmax;
using std::fmin;
using std::log1p;
using std::rint;
using std::sqrt;
#define SAKURA_HD
#define SAKURA_WAVE_ALL(p) (p)
#define SAKURA_NO_SCALAR_ASM
#define __builtin_amdgcn_rcp(x) ((1.0 / (x)) * (1.0 + 6e-8))
#define __builtin_amdgcn_rsq(x) ((1.0 / std::sqrt(x)) * (1.0 - 6e-8))
#include "../paper_1402_3325_amd/csrc/kepler_device.hpp"

// coef[4 i ..] = (f - 1, g - tau, fdot, gdot - 1) of problem i (mu already
// multiplied back in), iters[i], status[i] (bit 0: not converged, bit 8:
// safeguarded).  general != 0 takes the solve with run-time parameters.
extern "C" void host_pair_flow(int64_t n, const double *tau, const double *mu, const double *x,
                               const double *w, int general, double *coef, int *iters,
                               unsigned *status)
{
    const kep::KeplerParams kp{kep::DEFAULT_TOL, kep::DEFAULT_MAX_ITER};
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + 3 * i, *wi = w + 3 * i;
        const double r0sq = fma(xi[0], xi[0], fma(xi[1], xi[1], xi[2] * xi[2]));
        const kep::PairCoef o =
            general ? kep::kepler_flow(tau[i], mu[i], xi[0], xi[1], xi[2], wi[0], wi[1], wi[2],
                                       r0sq, kp)
                    : kep::kepler_flow_default(tau[i], mu[i], xi[0], xi[1], xi[2], wi[0], wi[1],
                                               wi[2], r0sq);
        coef[4 * i] = mu[i] * o.fm1;
        coef[4 * i + 1] = mu[i] * o.gmt;
        coef[4 * i + 2] = mu[i] * o.fdot;
        coef[4 * i + 3] = mu[i] * o.gdm1;
        iters[i] = o.iters;
        status[i] = o.status;
    }
}
