// Higher derivatives used by the adjoint pass: basis-function gradients,
// Hessians and Laplacian gradients, and the Pade pair function with its
// r-derivatives up to third order and their parameter derivatives.
// Host-and-device so that the formulas can be checked on the CPU.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace lrdmc {

// gradient of basis function type t (0 s Gaussian, 1..3 p Gaussian along
// x, y, z, 4 Slater 1s) with exponent al at displacement d = r - R
__host__ __device__ inline void basis_grad(int t, double al, const double* d, double* g)
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (t == 4) {
        const double r = sqrt(r2), e = exp(-al * r);
        for (int j = 0; j < 3; ++j) g[j] = -al * d[j] / r * e;
    } else {
        const double e = exp(-al * r2);
        if (t == 0) {
            for (int j = 0; j < 3; ++j) g[j] = -2.0 * al * d[j] * e;
        } else {
            const int q = t - 1;
            for (int j = 0; j < 3; ++j) g[j] = ((j == q) ? e : 0.0) - 2.0 * al * d[q] * d[j] * e;
        }
    }
}

// gradient g[3], Hessian H[6] (xx, xy, xz, yy, yz, zz) and gradient of the
// Laplacian gl[3]
__host__ __device__ inline void basis_d3(int t, double al, const double* d, double* g, double* H,
                                         double* gl)
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const int hj[6] = {0, 0, 0, 1, 1, 2}, hk[6] = {0, 1, 2, 1, 2, 2};
    if (t == 4) {
        const double r = sqrt(r2), ir = 1.0 / r, e = exp(-al * r);
        for (int j = 0; j < 3; ++j) g[j] = -al * d[j] * ir * e;
        for (int m = 0; m < 6; ++m) {
            const int j = hj[m], k = hk[m];
            const double dd = d[j] * d[k];
            H[m] = e * (al * al * dd * ir * ir - al * ((j == k ? ir : 0.0) - dd * ir * ir * ir));
        }
        const double c = 2.0 * al * ir * ir * ir - al * al * al * ir + 2.0 * al * al * ir * ir;
        for (int j = 0; j < 3; ++j) gl[j] = e * c * d[j];
    } else if (t == 0) {
        const double e = exp(-al * r2);
        for (int j = 0; j < 3; ++j) g[j] = -2.0 * al * d[j] * e;
        for (int m = 0; m < 6; ++m) {
            const int j = hj[m], k = hk[m];
            H[m] = (4.0 * al * al * d[j] * d[k] - (j == k ? 2.0 * al : 0.0)) * e;
        }
        const double c = 20.0 * al * al - 8.0 * al * al * al * r2;
        for (int j = 0; j < 3; ++j) gl[j] = c * d[j] * e;
    } else {
        const int q = t - 1;
        const double e = exp(-al * r2), dq = d[q];
        for (int j = 0; j < 3; ++j) g[j] = ((j == q) ? e : 0.0) - 2.0 * al * dq * d[j] * e;
        for (int m = 0; m < 6; ++m) {
            const int j = hj[m], k = hk[m];
            H[m] = (-2.0 * al * ((q == j ? d[k] : 0.0) + (q == k ? d[j] : 0.0)) +
                    dq * (4.0 * al * al * d[j] * d[k] - (j == k ? 2.0 * al : 0.0))) * e;
        }
        const double l0 = 4.0 * al * al * r2 - 10.0 * al;
        const double c = 28.0 * al * al - 8.0 * al * al * al * r2;
        for (int j = 0; j < 3; ++j) gl[j] = ((j == q) ? l0 : 0.0) * e + dq * d[j] * c * e;
    }
}

// u(r) = (A r + B r^2)/(1 + b r): value, r-derivatives, and d/d(A, B, b) of
// u, u' and u''
struct PadeD {
    double u, du, d2u, d3u;
    double u_p[3], du_p[3], d2u_p[3];
};

__host__ __device__ inline void pade_full(const double* p, double r, PadeD& f)
{
    const double A = p[0], B = p[1], b = p[2];
    const double D = 1.0 + b * r, iD = 1.0 / D, iD2 = iD * iD, iD3 = iD2 * iD, iD4 = iD3 * iD;
    f.u = (A * r + B * r * r) * iD;
    f.du = (A + 2.0 * B * r + B * b * r * r) * iD2;
    f.d2u = 2.0 * (B - A * b) * iD3;
    f.d3u = -6.0 * b * (B - A * b) * iD4;
    f.u_p[0] = r * iD;
    f.u_p[1] = r * r * iD;
    f.u_p[2] = -r * f.u * iD;
    f.du_p[0] = iD2;
    f.du_p[1] = (2.0 * r + b * r * r) * iD2;
    f.du_p[2] = -r * (2.0 * A + 3.0 * B * r + B * b * r * r) * iD3;
    f.d2u_p[0] = -2.0 * b * iD3;
    f.d2u_p[1] = 2.0 * iD3;
    f.d2u_p[2] = -2.0 * A * iD3 - 6.0 * r * (B - A * b) * iD4;
}

}  // namespace lrdmc
