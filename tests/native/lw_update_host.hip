// Host-side check of the blocked logarithmic weight update used by the
// load-balanced phase kernels (lw_block_update): for sequences of factors
// bbar / (W - E_0) that carry the running product far outside the range of a
// double, the blocked form must give the per-step sum of logarithms.
// Built with hipcc and run on the CPU by tests/test_host_native.py.
#include <cmath>
#include <cstdio>

#include "lrdmc_devfn.hpp"

int main()
{
    // (bbar, den) pairs: ordinary factors, factors far above and below one,
    // a subnormal denominator (bbar / den overflows to inf), a subnormal
    // numerator (bbar / den underflows)
    const double cases[][2] = {
        {1.3, 1.1}, {0.7, 1.2}, {1e300, 1e-5}, {1e300, 1e-5}, {1e-300, 1e5}, {1e-300, 1e5},
        {1.0, 4.9e-324}, {2.0, 1.0}, {4.9e-324, 1.0}, {3.0, 7.0}, {1e200, 1e-200}, {0.5, 2.0}};
    const int nc = (int)(sizeof(cases) / sizeof(cases[0]));
    double worst = 0.0;
    int bad = 0;
    for (int start = 0; start < nc; ++start) {
        for (int nsteps : {1, 5, 31, 32, 33, 64, 100}) {
            double lw = 0.0, wprod = 1.0, ref = 0.0;
            for (int k = 0; k < nsteps; ++k) {
                const double* c = cases[(start + k) % nc];
                lrdmc::lw_block_update(lw, wprod, c[0], c[1], k + 1);
                ref += std::log(c[0]) - std::log(c[1]);
                if (!(wprod >= 0x1p-600 && wprod <= 0x1p600)) ++bad;   // product stays in range
            }
            lw += std::log(wprod);
            const double err = std::fabs(lw - ref) / std::fmax(1.0, std::fabs(ref));
            if (!std::isfinite(lw)) ++bad;
            if (err > worst) worst = err;
        }
    }
    std::printf("worst_rel_err %.3e bad %d\n", worst, bad);
    return (bad == 0 && worst < 1e-13) ? 0 : 1;
}
