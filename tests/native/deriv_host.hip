// Host-side check of the derivative formulas of the adjoint pass
// (lrdmc_deriv.hpp) against fourth-order central differences: basis-function
// gradients against the basis values (written out here), Hessians against
// differences of the gradients, Laplacian gradients against differences of
// the Hessian trace, and the Pade pair function's r-derivatives up to third
// order and its parameter derivatives against differences in r and in
// (A, B, b). Built with hipcc and run on the CPU by tests/test_host_native.py.
#include <cmath>
#include <cstdio>

#include "lrdmc_deriv.hpp"

// basis value of type t (0 s Gaussian, 1..3 p Gaussian along x, y, z,
// 4 Slater 1s) at displacement d, written from its definition
static double value(int t, double al, const double* d)
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (t == 4) return std::exp(-al * std::sqrt(r2));
    const double e = std::exp(-al * r2);
    return t == 0 ? e : d[t - 1] * e;
}

// fourth-order central difference of f along a scalar parameter
template <class F>
static double diff4(F f, double h)
{
    return (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12.0 * h);
}

static double worst = 0.0;
static void check(double got, double want, double scale)
{
    const double e = std::fabs(got - want) / std::fmax(scale, 1e-300);
    if (!(e <= worst)) worst = std::isnan(e) ? INFINITY : e;
}

int main()
{
    const double h = 1e-3;
    const int hj[6] = {0, 0, 0, 1, 1, 2}, hk[6] = {0, 1, 2, 1, 2, 2};
    const double pts[][3] = {{0.3, -0.4, 0.5}, {1.1, 0.2, -0.7}, {-0.05, 0.8, 0.15}, {0.6, 0.6, -0.6}};
    const double als[] = {0.4, 1.3, 2.7};
    for (int t = 0; t < 5; ++t)
        for (double al : als)
            for (const auto& p : pts) {
                double g[3], H[6], gl[3], g1[3];
                lrdmc::basis_d3(t, al, p, g, H, gl);
                lrdmc::basis_grad(t, al, p, g1);
                double sc = 0.0;
                for (int j = 0; j < 3; ++j) sc = std::fmax(sc, std::fabs(g[j]));
                for (int j = 0; j < 3; ++j) {
                    auto vf = [&](double s) { double q[3] = {p[0], p[1], p[2]}; q[j] += s; return value(t, al, q); };
                    check(g[j], diff4(vf, h), sc);
                    check(g1[j], g[j], sc);
                }
                double hs = 0.0;
                for (int m = 0; m < 6; ++m) hs = std::fmax(hs, std::fabs(H[m]));
                for (int m = 0; m < 6; ++m) {
                    const int j = hj[m], k = hk[m];
                    auto gf = [&](double s) {
                        double q[3] = {p[0], p[1], p[2]}, gg[3];
                        q[k] += s;
                        lrdmc::basis_grad(t, al, q, gg);
                        return gg[j];
                    };
                    check(H[m], diff4(gf, h), hs);
                }
                double ls = 0.0;
                for (int j = 0; j < 3; ++j) ls = std::fmax(ls, std::fabs(gl[j]));
                for (int j = 0; j < 3; ++j) {
                    auto lf = [&](double s) {
                        double q[3] = {p[0], p[1], p[2]}, gg[3], HH[6], ll[3];
                        q[j] += s;
                        lrdmc::basis_d3(t, al, q, gg, HH, ll);
                        return HH[0] + HH[3] + HH[5];
                    };
                    check(gl[j], diff4(lf, h), ls);
                }
            }
    const double pars[][3] = {{0.25, 0.0, 1.0}, {0.5, 0.1, 0.8}, {-0.25, 0.3, 1.7}};
    const double rs[] = {0.2, 0.9, 2.5, 6.0};
    for (const auto& pp : pars)
        for (double r : rs) {
            lrdmc::PadeD f;
            lrdmc::pade_full(pp, r, f);
            auto at = [&](double dr, int ip, double dp) {
                double q[3] = {pp[0], pp[1], pp[2]};
                if (ip >= 0) q[ip] += dp;
                lrdmc::PadeD o;
                lrdmc::pade_full(q, r + dr, o);
                return o;
            };
            const double s = 1.0 + std::fabs(f.u) + std::fabs(f.du);
            check(f.du, diff4([&](double x) { return at(x, -1, 0).u; }, h), s);
            check(f.d2u, diff4([&](double x) { return at(x, -1, 0).du; }, h), s);
            check(f.d3u, diff4([&](double x) { return at(x, -1, 0).d2u; }, h), s);
            // the value itself against its definition
            check(f.u, (pp[0] * r + pp[1] * r * r) / (1.0 + pp[2] * r), s);
            for (int ip = 0; ip < 3; ++ip) {
                check(f.u_p[ip], diff4([&](double x) { return at(0, ip, x).u; }, h), s);
                check(f.du_p[ip], diff4([&](double x) { return at(0, ip, x).du; }, h), s);
                check(f.d2u_p[ip], diff4([&](double x) { return at(0, ip, x).d2u; }, h), s);
            }
        }
    std::printf("worst_rel_err %.3e\n", worst);
    return worst < 1e-8 ? 0 : 1;
}
