// Device helpers shared by the projection-phase kernels: Philox4x64-10,
// DPP wavefront collectives, the Pade pair function and the Gaussian / Slater
// basis functions.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "lrdmc_dev.hpp"

namespace lrdmc {

// Loads and stores through pointers known to address global memory (the
// descriptor's pointers are otherwise generic, and generic accesses also wait
// on the LDS counter).
template <class T>
__device__ __forceinline__ T gld(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// 1/x to about one ulp: hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// 1/sqrt(x) to about one ulp: hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Load-balanced weight update (Sec. II.C: w <- w bbar / (W - E_0)) in blocked
// logarithmic form.  The factors are multiplied into wprod, which stays in
// [2^-600, 2^600]; its logarithm is added to lw every 32 steps (step_no counts
// from 1).  A factor that would carry the product out of that range (or that
// is itself not a finite positive number, as bbar / den can be for a
// subnormal den) is added to lw as log(bbar) - log(den) together with the
// product so far, so lw stays what the per-step sum of logarithms gives.
__host__ __device__ __forceinline__ void lw_block_update(double& lw, double& wprod, double bbar,
                                                         double den, int step_no)
{
    const double np = wprod * (bbar / den);
    if (np > 0x1p-600 && np < 0x1p600) {
        wprod = np;
    } else {
        lw += log(wprod) + (log(bbar) - log(den));
        wprod = 1.0;
    }
    if ((step_no & 31) == 0) {
        lw += log(wprod);
        wprod = 1.0;
    }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0..c3), key
// (k0, k1); uniform = top 53 bits of the first output word times 2^-53.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double philox_uniform(uint64_t k0, uint64_t k1, uint64_t c0,
                                                 uint64_t c1, uint64_t c2, uint64_t c3)
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += w0; k1 += w1; }
        const uint64_t h0 = __umul64hi(m0, c0), l0 = m0 * c0;
        const uint64_t h1 = __umul64hi(m1, c2), l1 = m1 * c2;
        const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
    }
    return (double)(c0 >> 11) * 0x1.0p-53;
}

// All four output words of one Philox4x64-10 evaluation.
__device__ __forceinline__ void philox4(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1,
                                        uint64_t c2, uint64_t c3, uint64_t out[4])
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += w0; k1 += w1; }
        const uint64_t h0 = __umul64hi(m0, c0), l0 = m0 * c0;
        const uint64_t h1 = __umul64hi(m1, c2), l1 = m1 * c2;
        const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Random lattice orientation of one walker for one projection phase (App. D:
// the versors of the discretized Laplacian rotate with random angles).  A
// uniformly random rotation is that of a uniformly random unit quaternion; a
// point uniform in the unit 4-ball has a uniform direction, so q = 2U - 1 per
// component (the four words of Philox counter (slot, j, attempt, 4)) is
// accepted once 1e-3 <= |q|^2 <= 1, for attempts 0..63 (identity if all fail).
// Lattice step vectors st[3 d + x] = a R[x][d], R the quaternion rotation
// matrix divided by |q|^2.  Every operation is rounded on its own in the order
// written (no contraction into fused multiply-adds), so the steps, and the
// positions they move, are reproducible bit for bit by any implementation that
// evaluates the same expressions in the same order.
__device__ __forceinline__ void lattice_steps(uint64_t seed, uint64_t sysid, uint64_t slot, uint64_t j,
                                           double a, double* st, double* uv = nullptr)
{
#pragma clang fp contract(off)
    double R[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    for (uint64_t k = 0; k < 64; ++k) {
        uint64_t o[4];
        philox4(seed, sysid, slot, j, k, 4, o);
        const double w = 2.0 * ((double)(o[0] >> 11) * 0x1.0p-53) - 1.0;
        const double x = 2.0 * ((double)(o[1] >> 11) * 0x1.0p-53) - 1.0;
        const double y = 2.0 * ((double)(o[2] >> 11) * 0x1.0p-53) - 1.0;
        const double z = 2.0 * ((double)(o[3] >> 11) * 0x1.0p-53) - 1.0;
        const double ww = w * w, xx = x * x, yy = y * y, zz = z * z;
        const double n = ((ww + xx) + yy) + zz;
        if (!(n <= 1.0 && n >= 1e-3)) continue;
        const double xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
        R[0] = (((ww + xx) - yy) - zz) / n;
        R[1] = (2.0 * (xy - wz)) / n;
        R[2] = (2.0 * (xz + wy)) / n;
        R[3] = (2.0 * (xy + wz)) / n;
        R[4] = (((ww - xx) + yy) - zz) / n;
        R[5] = (2.0 * (yz - wx)) / n;
        R[6] = (2.0 * (xz - wy)) / n;
        R[7] = (2.0 * (yz + wx)) / n;
        R[8] = (((ww - xx) - yy) + zz) / n;
        break;
    }
    for (int d = 0; d < 3; ++d)
        for (int x = 0; x < 3; ++x) st[3 * d + x] = a * R[3 * x + d];
    // the versors themselves, uv[3 d + x] = R[x][d]
    if (uv)
        for (int d = 0; d < 3; ++d)
            for (int x = 0; x < 3; ++x) uv[3 * d + x] = R[3 * x + d];
}

// Fixed lattice axes: st = a on the diagonal (versors uv: the identity).
__device__ __forceinline__ void lattice_steps_fixed(double a, double* st, double* uv = nullptr)
{
    for (int q = 0; q < 9; ++q) st[q] = (q % 4 == 0) ? a : 0.0;
    if (uv)
        for (int q = 0; q < 9; ++q) uv[q] = (q % 4 == 0) ? 1.0 : 0.0;
}

// Quadrature point q (0..5 = +u0, -u0, +u1, -u1, +u2, -u2) of the sphere of
// radius r around the atom at c, along the versors uv[3 d + x]: c +- r u_d,
// each product and sum rounded on its own, so that a non-local move lands on
// the same point as in any implementation evaluating the same expressions.
__device__ __forceinline__ void nl_point(const double* c, double r, const double* uv, int q, double* o)
{
#pragma clang fp contract(off)
    const int d = q >> 1;
    const bool neg = (q & 1) != 0;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        const double t = r * uv[3 * d + x];
        o[x] = c[x] + (neg ? -t : t);
    }
}

// |r - c| with the products and sums rounded in the written order and a
// correctly rounded square root.
__device__ __forceinline__ double exact_distance(const double* r, const double* c)
{
#pragma clang fp contract(off)
    const double dx = r[0] - c[0], dy = r[1] - c[1], dz = r[2] - c[2];
    return __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
}

// Point q of electron position r: r itself (q = 0) or its lattice neighbour
// q = 1..6 in move order (+d0, -d0, +d1, -d1, +d2, -d2) with the step vectors
// st[3 d + x]: every coordinate moved by one addition of the signed step
// (the same additions as the move itself; with fixed axes two of them add 0).
__device__ __forceinline__ void point_qv(const double* r, int q, const double* st, double* o)
{
    if (q == 0) { o[0] = r[0]; o[1] = r[1]; o[2] = r[2]; return; }
    const int d = (q - 1) >> 1;
    const bool neg = ((q - 1) & 1) != 0;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        const double v = st[3 * d + x];
        o[x] = r[x] + (neg ? -v : v);
    }
}

// ---------------------------------------------------------------------------
// wavefront collectives on DPP (data-parallel primitives: lane shuffles that
// run in the VALU, no LDS round trip).  A double moves as two 32-bit halves.
// Every lane receives the same (lane 63) result so that control flow stays
// uniform; the reduction order is fixed, so results are bit-reproducible.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane63(double v)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_mov<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x114, 0xf>(v);   // row_shr:4
    v += dpp_mov<0x118, 0xf>(v);   // row_shr:8
    v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_mov<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return lane63(v);
}

// maximum over the 64 lanes (every lane receives it); lanes without a DPP
// source contribute 0, so it serves non-negative data
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_mov<0xb1, 0xf>(v));
    v = fmax(v, dpp_mov<0x4e, 0xf>(v));
    v = fmax(v, dpp_mov<0x114, 0xf>(v));
    v = fmax(v, dpp_mov<0x118, 0xf>(v));
    v = fmax(v, dpp_mov<0x142, 0xa>(v));
    v = fmax(v, dpp_mov<0x143, 0xc>(v));
    return lane63(v);
}

// sums over each row of 16 lanes (result in the row's last lane), and over
// pairs of rows (result in lanes 31 and 63)
__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_mov<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x114, 0xf>(v);   // row_shr:4
    v += dpp_mov<0x118, 0xf>(v);   // row_shr:8
    return v;
}

__device__ __forceinline__ double row32_sum(double v)
{
    v = row16_sum(v);
    v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    return v;
}

__device__ __forceinline__ double lane_value(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// inclusive prefix sum over the 64 lanes (Hillis-Steele inside 16-lane rows,
// then row broadcasts)
__device__ __forceinline__ double wave_incl_scan(double v, int)
{
    v += dpp_mov<0x111, 0xf>(v);   // row_shr:1
    v += dpp_mov<0x112, 0xf>(v);   // row_shr:2
    v += dpp_mov<0x114, 0xf>(v);   // row_shr:4
    v += dpp_mov<0x118, 0xf>(v);   // row_shr:8
    v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_mov<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// Pade pair function u(r) = (A r + B r^2)/(1 + b r) with u' and u''.
__device__ __forceinline__ double pade_u(const double* p, double r)
{
    return (p[0] * r + p[1] * r * r) / (1.0 + p[2] * r);
}
// u, u'/r and u'' + 2u'/r (the pieces of the gradient and Laplacian), with
// one division for 1/(1 + b r) and one for 1/r
__device__ __forceinline__ void pade_derivs(const double* p, double r, double& u, double& du_r,
                                            double& lap)
{
    const double A = p[0], B = p[1], b = p[2];
    const double iden = 1.0 / (1.0 + b * r), ir = 1.0 / r;
    const double i2 = iden * iden;
    u = (A * r + B * r * r) * iden;
    const double du = (A + 2.0 * B * r + B * b * r * r) * i2;
    du_r = du * ir;
    lap = 2.0 * (B - A * b) * i2 * iden + 2.0 * du_r;
}

__device__ __forceinline__ double norm3(double x, double y, double z)
{
    return sqrt(x * x + y * y + z * z);
}

// Point q of electron position r: r itself (q = 0) or its lattice neighbour
// q = 1..6 in move order (+a x, -a x, +a y, -a y, +a z, -a z); the displaced
// coordinate is formed by the same single addition as the move itself.
__device__ __forceinline__ void point_q(const double* r, int q, double a, double* o)
{
    o[0] = r[0]; o[1] = r[1]; o[2] = r[2];
    if (q == 1) o[0] = r[0] + a;
    if (q == 2) o[0] = r[0] + (-a);
    if (q == 3) o[1] = r[1] + a;
    if (q == 4) o[1] = r[1] + (-a);
    if (q == 5) o[2] = r[2] + a;
    if (q == 6) o[2] = r[2] + (-a);
}

// Value of basis function mu at point r.
__device__ __forceinline__ double basis_value(const DevSys& s, int mu, const double* r)
{
    const double* Ra = s.btab + 4 * mu;
    const double dx = r[0] - Ra[0], dy = r[1] - Ra[1], dz = r[2] - Ra[2];
    const double d2 = dx * dx + dy * dy + dz * dz, al = Ra[3];
    const int t = s.btype[mu];
    if (t == 4) return exp(-al * sqrt(d2));
    const double g = exp(-al * d2);
    if (t == 0) return g;
    return (t == 1 ? dx : (t == 2 ? dy : dz)) * g;
}

// Value, gradient and Laplacian of basis function mu at r.
__device__ __forceinline__ void basis_vgl(const DevSys& s, int mu, const double* r, double& v,
                                          double* g, double& l)
{
    const double* Ra = s.btab + 4 * mu;
    const double d[3] = {r[0] - Ra[0], r[1] - Ra[1], r[2] - Ra[2]};
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], al = Ra[3];
    const int t = s.btype[mu];
    if (t == 4) {
        const double dd = sqrt(d2), e = exp(-al * dd);
        v = e;
        for (int c = 0; c < 3; ++c) g[c] = -al * d[c] / dd * e;
        l = (al * al - 2.0 * al / dd) * e;
    } else if (t == 0) {
        const double e = exp(-al * d2);
        v = e;
        for (int c = 0; c < 3; ++c) g[c] = -2.0 * al * d[c] * e;
        l = (4.0 * al * al * d2 - 6.0 * al) * e;
    } else {
        const int q = t - 1;
        const double e = exp(-al * d2);
        v = d[q] * e;
        for (int c = 0; c < 3; ++c) g[c] = ((c == q) ? e : 0.0) - 2.0 * al * d[q] * d[c] * e;
        l = d[q] * e * (4.0 * al * al * d2 - 10.0 * al);
    }
}

// The same two functions from the displacement d = r - R, d2 = |d|^2.
__device__ __forceinline__ double basis_value_d(int t, double al, double dx, double dy, double dz,
                                                double d2)
{
    if (t == 4) return exp(-al * sqrt(d2));
    const double g = exp(-al * d2);
    if (t == 0) return g;
    return (t == 1 ? dx : (t == 2 ? dy : dz)) * g;
}

__device__ __forceinline__ void basis_vgl_d(int t, double al, double dx, double dy, double dz,
                                            double d2, double& v, double* g, double& l)
{
    const double d[3] = {dx, dy, dz};
    if (t == 4) {
        const double dd = sqrt(d2), e = exp(-al * dd), id = 1.0 / dd;
        v = e;
        for (int c = 0; c < 3; ++c) g[c] = -al * d[c] * id * e;
        l = (al * al - 2.0 * al * id) * e;
        return;
    }
    // s and p Gaussians share one exponential
    const double e = exp(-al * d2);
    if (t == 0) {
        v = e;
        for (int c = 0; c < 3; ++c) g[c] = -2.0 * al * d[c] * e;
        l = (4.0 * al * al * d2 - 6.0 * al) * e;
    } else {
        const int q = t - 1;
        const double dq = d[q];
        v = dq * e;
        for (int c = 0; c < 3; ++c) g[c] = ((c == q) ? e : 0.0) - 2.0 * al * dq * d[c] * e;
        l = dq * e * (4.0 * al * al * d2 - 10.0 * al);
    }
}

// ---------------------------------------------------------------------------
// per-walker state views
// ---------------------------------------------------------------------------
}  // namespace lrdmc
