// Mixed-precision projection phase for large systems (up to 128 electrons,
// 64 orbitals per spin, hundreds of basis functions): one 256-thread
// workgroup per walker.
//
// The same method steps as the FP64 phase kernel (ratios of all 6N lattice
// moves, App. D lattice diagonal and local energy, Algorithm 1 / Algorithm 2
// weight update, heat-bath move, Sherman-Morrison update), with the data
// placement of a system whose walker state does not fit on chip:
//   HBM (FP32, per walker): orbital values at the 6N moves and orbital
//     derivatives at the current positions, both k-major per spin so that the
//     determinant-ratio and gradient dot products read them coalesced; Slater
//     rows; transposed inverses.
//   LDS: positions and potentials (FP64), ratios, Jastrow caches, cached
//     determinant gradients/Laplacians (FP32), the moved electron's basis
//     rows, block-reduction scratch.
// Precision: basis functions, Jastrow sums and ratios in FP32; the orbital
// GEMM on MFMA in FP32 or BF16 with FP32 accumulation; positions, potentials,
// weights, all sums that form W, bbar and e_L, and the periodic refresh of
// the inverses (Newton-Schulz correction or Gauss-Jordan) in FP64.  The local
// energy is formed as the continuum local energy plus
// sum_i (nu_opt,i - nu_zv,i) (App. D identity), which avoids the
// cancellation in W - bbar when bbar is known only to FP32 accuracy.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lrdmc_dev.hpp"
#include "lrdmc_devfn.hpp"

namespace lrdmc {

extern __shared__ double lds[];

#define LDSD(off) (reinterpret_cast<double*>(reinterpret_cast<char*>(lds) + (off)))
#define LDSF(off) (reinterpret_cast<float*>(reinterpret_cast<char*>(lds) + (off)))

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_m __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// block collectives (1, 2 or 4 wavefronts); red is an LDS scratch of 4
// doubles (8 for block_sum2, 20 for the scan with a flag)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int tid = threadIdx.x, nwv = blockDim.x >> 6;
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = red[0];
    for (int q = 1; q < nwv; ++q) t += red[q];
    return t;
}

// two block sums with one pair of barriers (red holds [waves][2])
__device__ __forceinline__ void block_sum2(double& v0, double& v1, double* red)
{
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    const int tid = threadIdx.x, nwv = blockDim.x >> 6;
    __syncthreads();
    if ((tid & 63) == 0) { red[2 * (tid >> 6)] = v0; red[2 * (tid >> 6) + 1] = v1; }
    __syncthreads();
    double t0 = red[0], t1 = red[1];
    for (int q = 1; q < nwv; ++q) { t0 += red[2 * q]; t1 += red[2 * q + 1]; }
    v0 = t0; v1 = t1;
}

// Global-memory data written by some waves of the workgroup and read by others
// after the barrier.  The workgroup-scope fence orders the accesses in the
// compiler but is lowered without a wait for outstanding vector-memory stores
// (it relies on the vector L1 serving the waves of a CU in order); the explicit
// wait makes every store of this wave complete before the barrier, so the
// hand-off does not depend on that ordering.
__device__ __forceinline__ void global_handoff()
{
    __threadfence_block();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

__device__ __forceinline__ double block_max(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int tid = threadIdx.x, nwv = blockDim.x >> 6;
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = red[0];
    for (int q = 1; q < nwv; ++q) t = fmax(t, red[q]);
    return t;
}

// exclusive prefix of v over the block (thread order) and the block total
// exclusive block scan of v with the block total; when any is given, also the
// block OR of flag (wave flags in red[16 + wave])
__device__ __forceinline__ double block_excl_scan(double v, double* red, double& total,
                                                  int flag = 0, bool* any = nullptr)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
    const double inc = wave_incl_scan(v, lane);
    double prev = __shfl_up(inc, 1);
    if (lane == 0) prev = 0.0;
    const bool wflag = any && __ballot(flag) != 0;
    __syncthreads();
    if (lane == 63) red[wv] = inc;
    if (any && lane == 0) red[16 + wv] = wflag ? 1.0 : 0.0;
    __syncthreads();
    double off = 0.0;
    for (int q = 0; q < wv; ++q) off += red[q];
    total = red[0];
    for (int q = 1; q < nwv; ++q) total += red[q];
    if (any) {
        double f = 0.0;
        for (int q = 0; q < nwv; ++q) f += red[16 + q];
        *any = f > 0.0;
    }
    return off + prev;
}

// FP32 Pade parameter row and the pair terms from the squared distance
// (hardware reciprocal square root and reciprocal, about 1 ulp in FP32)
struct PadeF { float A, B, b; };
__device__ __forceinline__ PadeF pade_row(const DevMix& s, int jr)
{
    const double* p = s.jas + 3 * jr;
    return PadeF{(float)gld(p), (float)gld(p + 1), (float)gld(p + 2)};
}
__device__ __forceinline__ float pade_u2f(const PadeF& p, float r2)
{
    const float r = r2 * __builtin_amdgcn_rsqf(r2);
    return r * (p.A + p.B * r) * __builtin_amdgcn_rcpf(1.0f + p.b * r);
}
// u, u'/r, u'' + 2u'/r from r and 1/r
__device__ __forceinline__ void pade_derivs_rf(const PadeF& p, float r, float ir, float& u,
                                               float& du_r, float& lap)
{
    const float iden = __builtin_amdgcn_rcpf(1.0f + p.b * r), i2 = iden * iden;
    u = (p.A * r + p.B * r * r) * iden;
    const float du = (p.A + 2.0f * p.B * r + p.B * p.b * r * r) * i2;
    du_r = du * ir;
    lap = 2.0f * (p.B - p.A * p.b) * i2 * iden + 2.0f * du_r;
}

__device__ __forceinline__ int mspin(const DevMix& s, int i) { return i >= s.Nup; }
__device__ __forceinline__ int mcol(const DevMix& s, int i) { return i >= s.Nup ? i - s.Nup : i; }
__device__ __forceinline__ int mnspin(const DevMix& s, int sp) { return sp ? s.Ndn : s.Nup; }
__device__ __forceinline__ int mee_row(const DevMix& s, int i, int k)
{
    return ((i >= s.Nup) == (k >= s.Nup)) ? 0 : 1;
}

// partner k of electron i: position (FP64) and Pade parameter row
__device__ __forceinline__ void mpartner(const DevMix& s, const double* pos, int i, int k,
                                         double* pk, int& jr)
{
    if (k < s.N) {
        pk[0] = pos[3 * k]; pk[1] = pos[3 * k + 1]; pk[2] = pos[3 * k + 2];
        jr = mee_row(s, i, k);
    } else {
        const int I = k - s.N;
        pk[0] = gld(s.R + 3 * I); pk[1] = gld(s.R + 3 * I + 1); pk[2] = gld(s.R + 3 * I + 2);
        jr = 2 + gld(s.spec + I);
    }
}

// nuclear potential of nucleus I from the squared distance r2 and ir = 1/r
// (FP64): nu and its lattice bound nu^a
__device__ __forceinline__ void nuc_pot(const DevMix& s, int I, double r2, double ir, double ia,
                                        double& nu, double& nua)
{
    const double Z = gld(s.Z + I);
    if (gld(s.core + I) == 0) {
        nu = -Z * ir;
        nua = -Z * (ir < ia ? ir : ia);
    } else {
        const double rc = gld(s.rc + I);
        nu = nua = -Z * rsqrt_nr(r2 + rc * rc);
    }
}

// ---------------------------------------------------------------------------
// orbital rows of electron j at r: 11 rows (value, 6 neighbours, gradient,
// Laplacian) x n_j columns into LDS rows[11][ns]
// ---------------------------------------------------------------------------
__device__ __noinline__ void mixed_rows(const DevMix* __restrict__ dm, int j, const double* r, double a)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int Nb = s.Nb;
    const bool bf = s.gemm == kGemmBF16;
    float* B = LDSF(s.l_U);                      // [11][nb32 + 4] basis rows (zero padded; the
    const int ldb = s.nb32 + 4;                  // extra 4 floats spread the rows over the banks)
    float* rows = LDSF(s.l_rows);
    const int n = mnspin(s, mspin(s, j));
    const int tiles = (n + 15) / 16;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int nkb = s.nb32 / 32;
    const long plane = (long)((s.ns + 15) / 16) * nkb * 64;
    // the padding columns [Nb, ldb) of the 11 rows are read by the BF16 GEMM
    for (int z = tid; z < 11 * (ldb - Nb); z += (int)blockDim.x) {
        const int row = z / (ldb - Nb);
        B[row * ldb + Nb + (z - row * (ldb - Nb))] = 0.0f;
    }
    auto put = [&](int row, int mu, float v) { B[row * ldb + mu] = v; };
    // one thread per basis function: a Gaussian factorizes along the lattice
    // versors, so its values at the six neighbours r + s a e_c follow from
    // exp(-alpha d^2), exp(-alpha a^2) and exp(-+2 alpha a d.e_c) (d = r - centre);
    // Slater functions, and exponents beyond the FP32 range, take the seven
    // points directly
    const float af = (float)a;
    const double* st64 = LDSD(s.l_ev);          // step vectors a e_c, [3 c + x]
    const float* st32 = LDSF(s.l_ev + 72);
    for (int mu = tid; mu < Nb; mu += (int)blockDim.x) {
        const double4_t rec = gld((const double4_t*)(s.btab + 4 * mu));
        const int t = gld(s.btype + mu);
        const float d[3] = {(float)(r[0] - rec[0]), (float)(r[1] - rec[1]), (float)(r[2] - rec[2])};
        const float d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], al = (float)rec[3];
        const float m2al = -2.0f * al;
        // a d.e_c along each versor
        float sd[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            sd[cc] = d[0] * st32[3 * cc] + d[1] * st32[3 * cc + 1] + d[2] * st32[3 * cc + 2];
        bool fac = t != 4;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) fac = fac && fabsf(m2al * sd[cc]) < 80.0f;
        float v, g0, g1, g2, l;
        if (fac) {
            // rows 2c+1, 2c+2: the difference D = chi(r + st_c) - chi(r - st_c)
            // and the second difference S = chi(r + st_c) + chi(r - st_c) - 2 chi(r)
            // of the neighbour values, from G+- = e K E^+-1 (E = exp(x), x = -2 alpha a d.e_c)
            // written with m = expm1(x) so that neither cancels:
            //   G+ - G- = e K (E - 1/E),  E - 1/E = m (1 + 1/E),      m = E - 1
            //   G+ + G- - 2e = e (K (E + 1/E - 2) + 2 (K - 1)),  E + 1/E - 2 = m^2 / E
            const float e = expf(-al * d2), km1 = expm1f(-al * af * af), K = 1.0f + km1;
            const int ax = t - 1;
            const float f0 = t == 0 ? 1.0f : (ax == 0 ? d[0] : (ax == 1 ? d[1] : d[2]));
            const float eK = e * K;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                // E^-1 from its own exponential (1 + m rounds to 0 for x below
                // -17 in FP32), m^2 / E as m (m / E), which stays finite for
                // every |x| < 80
                const float x = m2al * sd[cc];
                const float m = expm1f(x), iE = expf(-x);
                const float sh = m * (1.0f + iE), ch = m * (m * iE);
                const float gdif = eK * sh;                    // G+ - G-
                const float gsec = e * (K * ch + 2.0f * km1);  // G+ + G- - 2e
                // the p factor moves by the step's component h along its axis:
                //   f+- = f0 +- h, D = f0 (G+ - G-) + h (G+ + G-), S = f0 (G+ + G- - 2e) + h (G+ - G-)
                const float h = t != 0 ? st32[3 * cc + (ax < 0 ? 0 : ax)] : 0.0f;
                put(2 * cc + 1, mu, f0 * gdif + h * (eK * (2.0f + ch)));
                put(2 * cc + 2, mu, f0 * gsec + h * gdif);
            }
            v = f0 * e;
            if (t == 0) {
                g0 = -2.0f * al * d[0] * e; g1 = -2.0f * al * d[1] * e; g2 = -2.0f * al * d[2] * e;
                l = (4.0f * al * al * d2 - 6.0f * al) * e;
            } else {
                g0 = (ax == 0 ? e : 0.0f) - 2.0f * al * f0 * d[0] * e;
                g1 = (ax == 1 ? e : 0.0f) - 2.0f * al * f0 * d[1] * e;
                g2 = (ax == 2 ? e : 0.0f) - 2.0f * al * f0 * d[2] * e;
                l = f0 * e * (4.0f * al * al * d2 - 10.0f * al);
            }
        } else {
            // the six neighbour values directly, then their difference and
            // second difference along each versor (rows 2c+1, 2c+2)
            float w[6];
            for (int q = 1; q < 7; ++q) {
                double p[3];
                point_qv(r, q, st64, p);
                const float dx = (float)(p[0] - rec[0]), dy = (float)(p[1] - rec[1]),
                            dz = (float)(p[2] - rec[2]);
                const float dq2 = dx * dx + dy * dy + dz * dz;
                if (t == 4) w[q - 1] = expf(-al * sqrtf(dq2));
                else {
                    const float e = expf(-al * dq2);
                    w[q - 1] = (t == 0 ? 1.0f : (t == 1 ? dx : (t == 2 ? dy : dz))) * e;
                }
            }
            const float dx = d[0], dy = d[1], dz = d[2];
            if (t == 4) {
                const float dd = sqrtf(d2), e = expf(-al * dd), id = 1.0f / dd;
                v = e; g0 = -al * dx * id * e; g1 = -al * dy * id * e; g2 = -al * dz * id * e;
                l = (al * al - 2.0f * al * id) * e;
            } else if (t == 0) {
                const float e = expf(-al * d2);
                v = e; g0 = -2.0f * al * dx * e; g1 = -2.0f * al * dy * e; g2 = -2.0f * al * dz * e;
                l = (4.0f * al * al * d2 - 6.0f * al) * e;
            } else {
                const float e = expf(-al * d2);
                const float dq = t == 1 ? dx : (t == 2 ? dy : dz);
                v = dq * e;
                g0 = (t == 1 ? e : 0.0f) - 2.0f * al * dq * dx * e;
                g1 = (t == 2 ? e : 0.0f) - 2.0f * al * dq * dy * e;
                g2 = (t == 3 ? e : 0.0f) - 2.0f * al * dq * dz * e;
                l = dq * e * (4.0f * al * al * d2 - 10.0f * al);
            }
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                put(2 * cc + 1, mu, w[2 * cc] - w[2 * cc + 1]);
                put(2 * cc + 2, mu, (w[2 * cc] - v) + (w[2 * cc + 1] - v));
            }
        }
        put(0, mu, v);
        put(7, mu, g0); put(8, mu, g1); put(9, mu, g2);
        put(10, mu, l);
    }
    __syncthreads();
    for (int t = wv; t < tiles; t += (int)(blockDim.x >> 6)) {
        float4_t acc = {0.f, 0.f, 0.f, 0.f};
        const int col = 16 * t + i16;
        // rows 11..15 of the A tile are never stored: lanes i16 >= 11 read row 0
        const int ar = i16 < 11 ? i16 : 0;
        if (bf) {
            // 16x16x32 BF16 tiles, lane holds 8 consecutive inner indices.
            // Each FP32 operand is split into a BF16 high part and a BF16
            // residual; hi*hi + hi*lo + lo*hi keeps about 16 significant bits.
            // The coefficient operands (shared by all walkers, L2-resident) are
            // double-buffered: k-blocks kb + 2, kb + 3 load into one register
            // pair while kb, kb + 1 are multiplied from the other, with no
            // copies between them (indices clamped, so that every load stays
            // in bounds; the tail blocks are skipped)
            const bf16x8_t* cb = reinterpret_cast<const bf16x8_t*>(s.Cbf) + (long)t * nkb * 64;
            const float* a_row = B + ar * ldb + 8 * k4;
            auto ldc = [&](int kb, bf16x8_t& h, bf16x8_t& l) {
                const long o = (long)min(kb, nkb - 1) * 64 + lane;
                h = gld(cb + o);
                l = gld(cb + plane + o);
            };
            auto mul = [&](int kb, const bf16x8_t& h, const bf16x8_t& l) {
                if (kb >= nkb) return;
                const float4_t* src = reinterpret_cast<const float4_t*>(a_row + 32 * kb);
                const float4_t v0 = src[0], v1 = src[1];
                const float xa[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
                bf16x8_t ah, alo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 hh = (__bf16)xa[e];
                    ah[e] = hh;
                    alo[e] = (__bf16)(xa[e] - (float)hh);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, h, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, l, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, h, acc, 0, 0, 0);
            };
            bf16x8_t h0, l0, h1, l1, h2, l2, h3, l3;
            ldc(0, h0, l0);
            ldc(1, h1, l1);
#pragma unroll 1
            for (int kb = 0; kb < nkb; kb += 4) {
                ldc(kb + 2, h2, l2);
                ldc(kb + 3, h3, l3);
                mul(kb, h0, l0);
                mul(kb + 1, h1, l1);
                ldc(kb + 4, h0, l0);
                ldc(kb + 5, h1, l1);
                mul(kb + 2, h2, l2);
                mul(kb + 3, h3, l3);
            }
        } else {
            // 16x16x4 FP32 tiles; the coefficient column loads are
            // double-buffered in groups of KF k-steps (indices clamped)
            constexpr int KF = 8;
            const int nk = (Nb + 3) / 4;
            const float* cf = s.Cf + min(col, n - 1);
            auto ldf = [&](int s0, float* v) {
#pragma unroll
                for (int u = 0; u < KF; ++u) {
                    const int mu = min(4 * (s0 + u) + k4, Nb - 1);
                    v[u] = gld(cf + (long)mu * s.ns);
                }
            };
            auto mulf = [&](int s0, const float* v) {
#pragma unroll
                for (int u = 0; u < KF; ++u) {
                    // lane (i16, k4) supplies A[i16][mu] and C[mu][col]
                    const int mu = 4 * (s0 + u) + k4;
                    const float av = mu < Nb ? B[ar * ldb + mu] : 0.0f;
                    const float bv = (mu < Nb && col < n) ? v[u] : 0.0f;
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
                }
            };
            float f0[KF], f1[KF];
            ldf(0, f0);
#pragma unroll 1
            for (int s0 = 0; s0 < nk; s0 += 2 * KF) {
                ldf(s0 + KF, f1);
                mulf(s0, f0);
                ldf(s0 + 2 * KF, f0);
                if (s0 + KF < nk) mulf(s0 + KF, f1);
            }
        }
        // D[row][col]: row = 4 (lane >> 4) + v
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * k4 + v;
            if (row < 11 && col < n) rows[row * s.ns + col] = acc[v];
        }
    }
    __syncthreads();
}

// store electron j's rows into the walker block (global, FP32)
__device__ __noinline__ void mixed_store_rows(const DevMix* __restrict__ dm, float* st, int j, bool arow)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x;
    const int sp = mspin(s, j), c = mcol(s, j), n = mnspin(s, sp), ns = s.ns;
    const float* rows = LDSF(s.l_rows);
    float* Phi = st + s.g_Phi + (long)sp * ns * 6 * ns;
    float* dPhi = st + s.g_dPhi + (long)sp * ns * 4 * ns;
    for (int idx = tid; idx < 11 * n; idx += (int)blockDim.x) {
        const int row = idx / n, k = idx - row * n;
        const float v = rows[row * ns + k];
        if (row == 0) { if (arow) st[s.g_Arow + (long)j * ns + k] = v; }
        else if (row <= 6) Phi[(long)k * 6 * ns + 6 * c + row - 1] = v;
        else dPhi[(long)k * 4 * ns + 4 * c + row - 7] = v;
    }
    global_handoff();
}

// FP64 Gauss-Jordan (in place, partial pivoting) of the transposed Slater
// matrix of spin sp read from Arow ([N][ns], FP32 or FP64); writes the
// transposed inverse AiT[c][k] (FP32 or FP64, row stride ns).
//
// Per pivot column k: every wavefront finds the pivot row bi (largest
// |M[r][k]|, r >= k, first among equals: a wavefront maximum, n <= 64); the
// column k, the pivot row and row k are staged in LDS; one barrier; every
// thread updates its elements as if rows k and bi had been interchanged
// first (row k <- pivot row scaled, row bi <- old row k, eliminated); one
// barrier.  The row interchanges are undone at the end as one column
// permutation of the output.
template <class TS, class TD>
__device__ bool gj_inverse(const DevMix& s, const TS* Arow, TD* AiT, int sp)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = mnspin(s, sp);
    if (!n) return true;
    const int off = sp ? s.Nup : 0, ns = s.ns;
    const int ldm = n + 1;                       // odd row stride: columns spread over the banks
    double* M = LDSD(s.l_U);                     // [n][ldm]
    double* colk = M + n * ldm;                  // [n] column k
    double* prow = colk + n;                     // [n] pivot row
    double* qrow = prow + n;                     // [n] row k
    int* piv = reinterpret_cast<int*>(LDSF(s.l_tmp));   // [n] pivot rows
    int* cperm = piv + n;                               // [n] output column permutation
    // fixed column per thread, rows strided: no division in the n^2 loops
    const int rs = nt / n, c0 = tid % n, r0 = tid / n;
    const bool act = tid < rs * n;
    if (act)
        for (int r = r0; r < n; r += rs) M[r * ldm + c0] = (double)Arow[(long)(off + c0) * ns + r];
    __syncthreads();
    bool ok = true;
    const int lane = tid & 63;
    for (int k = 0; k < n; ++k) {
        const double v = (lane >= k && lane < n) ? fabs(M[lane * ldm + k]) : -1.0;
        const double best = wave_max(v);
        if (!(best > 0.0)) { ok = false; break; }
        const int bi = __ffsll((long long)__ballot(v == best)) - 1;
        for (int r = tid; r < n; r += nt) {
            colk[r] = M[r * ldm + k];
            prow[r] = M[bi * ldm + r];
            qrow[r] = M[k * ldm + r];
        }
        if (tid == 0) piv[k] = bi;
        __syncthreads();
        if (act) {
            const double id = 1.0 / prow[k];
            const double mk = (c0 == k ? 1.0 : prow[c0]) * id;
            const double qc = qrow[c0], qk = qrow[k];
            // eight rows per batch: all loads before the stores
            for (int rb = r0; rb < n; rb += 8 * rs) {
                double mv[8], cv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int r = rb + t * rs;
                    mv[t] = r < n ? M[r * ldm + c0] : 0.0;
                    cv[t] = r < n ? colk[r] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int r = rb + t * rs;
                    if (r < n) {
                        const double src = r == bi ? qc : mv[t];
                        const double cr = r == bi ? qk : cv[t];
                        M[r * ldm + c0] = r == k ? mk : (c0 == k ? 0.0 : src) - cr * mk;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (ok) {
        // the interchanges (k, piv[k]) applied to the columns in reverse order
        if (tid == 0) {
            for (int c = 0; c < n; ++c) cperm[c] = c;
            for (int k = n - 1; k >= 0; --k) {
                const int p = piv[k], t = cperm[k];
                cperm[k] = cperm[p];
                cperm[p] = t;
            }
        }
        __syncthreads();
        if (act) {
            const int cs = cperm[c0];
            for (int r = r0; r < n; r += rs) AiT[(long)r * ns + c0] = (TD)M[r * ldm + cs];
        }
    }
    global_handoff();
    return ok;
}

__device__ __noinline__ bool mixed_refresh_inverse(const DevMix* __restrict__ dm, float* st, int sp)
{
    const DevMix& s = *dm;
    return gj_inverse<float, float>(s, st + s.g_Arow, st + s.g_AinvT + (long)sp * s.ns * s.ns, sp);
}

// Determinant gradients / Laplacians gD[j][0..3] = dPhi_j . AinvT[c_j] and
// determinant ratios Rdet_p = Phi_p . AinvT[c] of every move of the electrons
// of spin sp, with the inverse staged in LDS (the basis-row block is free
// here; mixed_rows restores its zero padding).
__device__ __noinline__ void mixed_spin_update(const DevMix* __restrict__ dm, const float* st, int sp,
                                               bool staged)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x, nt = blockDim.x, ns = s.ns, lda = ns + 1;
    const int n = mnspin(s, sp), off = sp ? s.Nup : 0;
    if (!n) return;
    float* AiL = LDSF(s.l_U);                    // [n][ns + 1]
    if (!staged) {
        const float* Ai = st + s.g_AinvT + (long)sp * ns * ns;
        for (int idx = tid; idx < n * ns; idx += nt) {
            const int r = idx / ns;
            AiL[r * lda + idx - r * ns] = Ai[idx];
        }
        __syncthreads();
    }
    float* gD = LDSF(s.l_gD);
    float* Rdet = LDSF(s.l_Rdet);
    // column c of the inverse against electron c's gradient / Laplacian rows
    // (one float4 per orbital k) and its six neighbour rows (three float2):
    // kp adjacent lanes per electron split k (k = part, part + kp, ...), KB = 4
    // orbitals per batch, so that 16 loads (160 bytes) per lane are in flight
    // (the walker blocks live in HBM); the kp partial sums are combined across
    // the lanes
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f4v* dPhi4 = reinterpret_cast<const f4v*>(st + s.g_dPhi + (long)sp * ns * 4 * ns);
    const f2v* Phi2 = reinterpret_cast<const f2v*>(st + s.g_Phi + (long)sp * ns * 6 * ns);
    constexpr int KB = 4;
    int kp = 1;
    while (kp < 16 && 2 * kp * n <= nt) kp *= 2;
    const int per = nt / kp;
    for (int c0 = 0; c0 < n; c0 += per) {
        const int c = c0 + tid / kp, part = tid & (kp - 1);
        float acc[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (c < n) {
            const float* a = AiL + c * lda;
            for (int k0 = part; k0 < n; k0 += KB * kp) {
                f4v G[KB];
                f2v Q[KB][3];
#pragma unroll
                for (int u = 0; u < KB; ++u) {
                    const int k = k0 + u * kp;
                    if (k < n) {
                        G[u] = gld(dPhi4 + (long)k * ns + c);
                        const f2v* q = Phi2 + (long)k * 3 * ns + 3 * c;
                        Q[u][0] = gld(q); Q[u][1] = gld(q + 1); Q[u][2] = gld(q + 2);
                    } else {
                        G[u] = 0.f;
                        Q[u][0] = Q[u][1] = Q[u][2] = 0.f;
                    }
                }
#pragma unroll
                for (int u = 0; u < KB; ++u) {
                    const int k = k0 + u * kp;
                    const float av = k < n ? a[k] : 0.f;
                    acc[0] += G[u].x * av; acc[1] += G[u].y * av;
                    acc[2] += G[u].z * av; acc[3] += G[u].w * av;
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        acc[4 + 2 * m] += Q[u][m].x * av;
                        acc[5 + 2 * m] += Q[u][m].y * av;
                    }
                }
            }
        }
        for (int m = 1; m < kp; m <<= 1)
#pragma unroll
            for (int t = 0; t < 10; ++t) acc[t] += __shfl_xor(acc[t], m);
        if (c < n && part == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) gD[4 * (off + c) + t] = acc[t];
            // determinant ratio minus one of the moves +-e_m: the electron's
            // own Slater row times its inverse column is 1, so
            // R - 1 = (+-D.a + S.a) / 2 with the difference and second
            // difference rows (no cancellation against 1)
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const float dd = acc[4 + 2 * m], ss = acc[5 + 2 * m];
                Rdet[6 * (off + c) + 2 * m] = 0.5f * (ss + dd);
                Rdet[6 * (off + c) + 2 * m + 1] = 0.5f * (ss - dd);
            }
        }
    }
    __syncthreads();
}

// Ratios of every move, kept as R - 1 (both arrays): with R_det - 1 = q and
// the Jastrow exponent change x, R - 1 = q e^x + (e^x - 1)
__device__ __forceinline__ void mixed_full_ratios(const DevMix& s)
{
    float* R = LDSF(s.l_R);
    const float* Rdet = LDSF(s.l_Rdet);
    const float* dJ = LDSF(s.l_dJ);
    for (int p = threadIdx.x; p < s.P; p += (int)blockDim.x) {
        const float em = expm1f(dJ[p]);
        R[p] = Rdet[p] * (1.0f + em) + em;
    }
    __syncthreads();
}

// sum over the lane pair (quad_perm [1,0,3,2])
__device__ __forceinline__ float pair_sum(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, false));
}

// Pade terms of the six lattice neighbours of a point at FP32 difference f
// from a partner (squared distance r2f): squared distances |f|^2 + a^2 +- 2 f.st_c
// (st_c = a e_c, the walker's step vectors), kept positive; q adds
// u(neighbour) - u(point) in move order (+e_0, -e_0, +e_1, ...)
// The change u(r') - u(r) is formed without subtracting two values of u:
// with r'^2 - r^2 = a^2 +- 2 f.st_c (no cancellation) and r' - r = (r'^2 - r^2)/(r' + r),
//   u(r') - u(r) = (r' - r) (A + B (r + r') + b B r r') / ((1 + b r)(1 + b r')).
__device__ __forceinline__ void neighbour_du(const PadeF& p, const float f[3], float r2f, float aa,
                                             const float* st32, float q[6])
{
    const float r20 = fmaxf(r2f, 1e-30f);
    const float r = r20 * __builtin_amdgcn_rsqf(r20);
    const float iden0 = __builtin_amdgcn_rcpf(1.0f + p.b * r);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float t2 = 2.0f * (f[0] * st32[3 * c] + f[1] * st32[3 * c + 1] + f[2] * st32[3 * c + 2]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float dr2 = h ? aa - t2 : aa + t2;
            const float r2n = fmaxf(r20 + dr2, 1e-30f);
            const float rn = r2n * __builtin_amdgcn_rsqf(r2n);
            const float dr = dr2 * __builtin_amdgcn_rcpf(fmaxf(r + rn, 1e-30f));
            const float num = p.A + p.B * (r + rn) + p.b * p.B * r * rn;
            q[2 * c + h] += dr * num * iden0 * __builtin_amdgcn_rcpf(1.0f + p.b * rn);
        }
    }
}

// Jastrow caches and potentials of every electron from scratch; returns V_ee.
// Two threads per electron (adjacent lanes, partners k = h, h + 2, ...),
// combined over the lane pair; every pass keeps both lanes of a pair.  Each
// pair's FP64 difference is formed once and serves the gradient, Laplacian,
// potentials and the exponent changes of the electron's six moves.
__device__ __noinline__ double mixed_jastrow_all(const DevMix* __restrict__ dm, double a)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x;
    const double* pos = LDSD(s.l_pos);
    float* dJ = LDSF(s.l_dJ);
    float* Jg = LDSF(s.l_Jg);
    float* Jl = LDSF(s.l_Jl);
    double* nue = LDSD(s.l_nue);
    double* nua = LDSD(s.l_nua);
    const int K = s.N + s.M;
    const double ia = 1.0 / a;
    const float aa = (float)(a * a);
    const float* st32 = LDSF(s.l_ev + 72);
    double vee = 0.0;
    for (int base = 0; base < 2 * s.N; base += (int)blockDim.x) {
        const int it = base + tid, j = it >> 1, h = it & 1;
        const bool jv = it < 2 * s.N;
        const double* rj = pos + 3 * (jv ? j : 0);
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, l = 0.f;
        float dq[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        double nu = 0.0, nv = 0.0;
        #pragma unroll 1
        for (int k = h; jv && k < K; k += 2) {
            if (k == j) continue;
            const bool isel = k < s.N;
            double pk[3];
            int jr;
            mpartner(s, pos, j, k, pk, jr);
            const double d0 = rj[0] - pk[0], d1 = rj[1] - pk[1], d2 = rj[2] - pk[2];
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2, ir = rsqrt_nr(r2);
            if (isel || s.has_en) {
                const PadeF pr = pade_row(s, jr);
                float u, dur, lp;
                pade_derivs_rf(pr, (float)(r2 * ir), (float)ir, u, dur, lp);
                g0 += dur * (float)d0; g1 += dur * (float)d1; g2 += dur * (float)d2;
                l += lp;
                if (isel && k > j) vee += ir;
                const float f[3] = {(float)d0, (float)d1, (float)d2};
                neighbour_du(pr, f, (float)r2, aa, st32, dq);
            }
            if (!isel) {
                double a1, a2;
                nuc_pot(s, k - s.N, r2, ir, ia, a1, a2);
                nu += a1; nv += a2;
            }
        }
        g0 = pair_sum(g0); g1 = pair_sum(g1); g2 = pair_sum(g2); l = pair_sum(l);
#pragma unroll
        for (int q = 0; q < 6; ++q) dq[q] = pair_sum(dq[q]);
        nu += dpp_mov<0xb1, 0xf>(nu);
        nv += dpp_mov<0xb1, 0xf>(nv);
        if (jv && h == 0) {
            Jg[3 * j] = g0; Jg[3 * j + 1] = g1; Jg[3 * j + 2] = g2; Jl[j] = l;
            nue[j] = nu; nua[j] = nv;
#pragma unroll
            for (int q = 0; q < 6; ++q) dJ[6 * j + q] = dq[q];
        }
    }
    vee = block_sum(vee, LDSD(s.l_red));
    __syncthreads();
    return vee;
}

// Newton-Schulz correction of the FP32 inverse of spin sp that the
// Sherman-Morrison updates have carried since the last rebuild:
// E = I - A X (X = A^-1, X[k][c] = AiT[c][k]), X' = X + X E, both products
// on FP64 MFMA from the FP32 rows and inverse staged in LDS.  X' has error
// O(|E|^2).  Returns 0 when max|E| < kNsTight (corrected, done), 1 when
// max|E| < kNsLoose (corrected; one more step brings it below the tight
// bound), 2 otherwise (not applied: the rows are to be inverted afresh).
constexpr double kNsTight = 3e-4, kNsLoose = 3e-3;
__device__ __noinline__ int mixed_ns_correct(const DevMix* __restrict__ dm, float* st, int sp)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    const int n = mnspin(s, sp), off = sp ? s.Nup : 0, ns = s.ns, ld = n + 1;
    if (!n) return 0;
    float* Rl = LDSF(s.l_U);                     // [n][n + 1] Slater rows, then E
    float* Tl = Rl + n * ld;                     // [n][n + 1] AiT
    const float* Arow = st + s.g_Arow + (long)off * ns;
    float* AiT = st + s.g_AinvT + (long)sp * ns * ns;
    for (int idx = tid; idx < n * n; idx += nt) {
        const int r = idx / n, k = idx - r * n;
        Rl[r * ld + k] = Arow[(long)r * ns + k];
        Tl[r * ld + k] = AiT[(long)r * ns + k];
    }
    __syncthreads();
    const int TR = (n + 15) / 16, i16 = lane & 15, k4 = lane >> 4;   // TR <= 4
    double emax = 0.0;
    // E = I - R T^T: a row tile of R per wavefront; E then replaces those rows
    for (int rt = wv; rt < TR; rt += nwv) {
        double4_m acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = (double4_m){0.0, 0.0, 0.0, 0.0};
        const int j = 16 * rt + i16;
        for (int k0 = 0; k0 < n; k0 += 4) {
            const int k = k0 + k4;
            const double av = (j < n && k < n) ? (double)Rl[j * ld + k] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= TR) continue;
                const int c = 16 * t + i16;
                const double bv = (c < n && k < n) ? (double)Tl[c * ld + k] : 0.0;
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= TR) continue;
            const int c = 16 * t + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int jr = 16 * rt + k4 + 4 * v;
                if (jr < n && c < n) {
                    const double e = (jr == c ? 1.0 : 0.0) - acc[t][v];
                    emax = fmax(emax, fabs(e));
                    Rl[jr * ld + c] = (float)e;
                }
            }
        }
    }
    emax = block_max(emax, LDSD(s.l_red));   // also the barrier before E is read
    if (!(emax < kNsLoose)) return 2;
    // X' = X + X E, i.e. AiT'[c][k] = AiT[c][k] + sum_j E[j][c] AiT[j][k]
    for (int rt = wv; rt < TR; rt += nwv) {
        double4_m acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = (double4_m){0.0, 0.0, 0.0, 0.0};
        const int c = 16 * rt + i16;
        for (int j0 = 0; j0 < n; j0 += 4) {
            const int j = j0 + k4;
            const double av = (j < n && c < n) ? (double)Rl[j * ld + c] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= TR) continue;
                const int k = 16 * t + i16;
                const double bv = (j < n && k < n) ? (double)Tl[j * ld + k] : 0.0;
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= TR) continue;
            const int k = 16 * t + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int cr = 16 * rt + k4 + 4 * v;
                if (cr < n && k < n) AiT[(long)cr * ns + k] = (float)((double)Tl[cr * ld + k] + acc[t][v]);
            }
        }
    }
    global_handoff();
    return emax < kNsTight ? 0 : 1;
}

// periodic: a refresh of carried inverses (scheduled, or at the start of a
// phase), which first tries one or two Newton-Schulz corrections of each
// inverse; otherwise (rows rebuilt from positions, a tiny determinant ratio)
// the inverses are rebuilt by Gauss-Jordan.  jas: the Jastrow caches and
// potentials are rebuilt from the positions as well (the pair-difference
// updates of one move add a rounding each, far less than the rank-one updates
// of the inverse, so the scheduled refreshes rebuild them only every
// kJastrowEvery-th time)
constexpr int kJastrowEvery = 4;
__device__ __noinline__ bool mixed_refresh(const DevMix* __restrict__ dm, float* st, double a,
                                           bool periodic, bool jas = true)
{
    const DevMix& s = *dm;
    bool ok = true;
    for (int sp = 0; sp < 2; ++sp) {
        int st_ns = 2;
        if (periodic) {
            st_ns = mixed_ns_correct(&s, st, sp);
            if (st_ns == 1) st_ns = mixed_ns_correct(&s, st, sp) == 2 ? 2 : 0;
        }
        if (st_ns != 0) ok = mixed_refresh_inverse(&s, st, sp) && ok;
    }
    if (jas) {
        const double vee = mixed_jastrow_all(&s, a);
        if (threadIdx.x == 0) LDSD(s.l_scal)[kScVee] = vee;
    }
    mixed_spin_update(&s, st, 0, false);
    mixed_spin_update(&s, st, 1, false);
    mixed_full_ratios(s);
    return ok;
}

// pre, tot: the thread's exclusive prefix of the positive-ratio sums of the
// thread chunks (thread t owns moves [t per, (t + 1) per)) and their total,
// reused by the heat bath at the same configuration
struct MLocal { double bbar, W, eL, pre, tot; };

// lattice-regularized diagonal and local energy (App. D), e_L formed as the
// continuum local energy plus sum_i (nu_opt,i - nu_zv,i)
__device__ __noinline__ MLocal mixed_evaluate(const DevMix* __restrict__ dm, double a, int nu_mode)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x;
    const float* R = LDSF(s.l_R);
    const float* gD = LDSF(s.l_gD);
    const float* Jg = LDSF(s.l_Jg);
    const float* Jl = LDSF(s.l_Jl);
    const double* nue = LDSD(s.l_nue);
    const double* nua = LDSD(s.l_nua);
    double* red = LDSD(s.l_red);
    const int per = (s.P + (int)blockDim.x - 1) / (int)blockDim.x;
    const int p0 = tid * per, p1 = min(p0 + per, s.P);
    double loc = 0.0;
    int anyneg = 0;
    for (int p = p0; p < p1; ++p) {
        const double r = 1.0 + (double)R[p];
        if (r > 0) loc += r;
        else if (r < 0) anyneg = 1;
    }
    double bs;
    bool anynode;
    const double pre = block_excl_scan(loc, red, bs, anyneg, &anynode);
    double econt = 0.0, dnu = 0.0;
    const double ia2 = 1.0 / (a * a);
    for (int j = tid; j < s.N; j += (int)blockDim.x) {
        const double j0 = Jg[3 * j], j1 = Jg[3 * j + 1], j2 = Jg[3 * j + 2];
        const double lap = (double)gD[4 * j + 3] +
                           2.0 * ((double)gD[4 * j] * j0 + (double)gD[4 * j + 1] * j1 +
                                  (double)gD[4 * j + 2] * j2) +
                           (double)Jl[j] + j0 * j0 + j1 * j1 + j2 * j2;
        double lapA = 0.0;
        int nd = 0;
        for (int q = 0; q < 6; ++q) {
            const double rm1 = (double)R[6 * j + q];
            lapA += rm1 * ia2;
            if (1.0 + rm1 < 0) nd = 1;
        }
        if (nu_mode == 1) nd = anynode;
        if (nu_mode == 2) nd = 1;
        const double nuzv = nue[j] + 0.5 * (lapA - lap);
        const double numax = nuzv > nua[j] ? nuzv : nua[j];
        const double nuopt = nd ? numax : nuzv;
        econt += -0.5 * lap + nue[j];
        dnu += nuopt - nuzv;
    }
    block_sum2(econt, dnu, red + 8);            // clear of the heat-bath picks at red + 4
    MLocal L;
    L.bbar = bs / (2.0 * a * a);
    L.eL = econt + LDSD(s.l_scal)[kScVee] + s.vii + dnu;
    L.W = L.eL + L.bbar;
    L.pre = pre;
    L.tot = bs;
    return L;
}

// FP64 16x16x4 MFMA tiles of the phase-end evaluation: A operand lane
// (row i16, inner k4), B operand lane (inner k4, column i16), accumulator
// element v of lane (i16, k4) = D[k4 + 4v][i16].

// FP64 Slater rows A64[i][k] = sum_mu chi_mu(r_i) C[mu][k] (k < ns): in rounds
// of one row tile of 16 electrons per wavefront, the basis values of the
// round's electrons in chunks of fkc functions ([16 waves][fkc + 1] in LDS),
// the product on MFMA with every column tile of the row tile.  Where the
// scratch block has room, the chunk's coefficients are staged in LDS beside
// the basis values ([fkc][16 TC + 1]) by coalesced loads of all threads, so
// that the products read both operands from LDS.
__device__ __noinline__ void final_slater_rows(const DevMix& s, const double* pos, double* A64)
{
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    const int N = s.N, Nb = s.Nb, ns = s.ns, kc = max(4, s.fkc), ldc = kc + 1;
    const int TR = (N + 15) / 16, TC = (ns + 15) / 16;   // TC <= 4
    const int i16 = lane & 15, k4 = lane >> 4;
    double* Bc = LDSD(s.l_U);                    // [16 nwv][kc + 1]
    double* Cc = Bc + 16 * nwv * ldc;            // [kc][16 TC + 1]
    const int w16 = 16 * TC, ldcc = w16 + 1, ctot = kc * w16;
    const bool stage = (long)(16 * nwv * ldc + kc * ldcc) * 8 <= (long)(s.l_R - s.l_U);
    for (int r0 = 0; r0 < TR; r0 += nwv) {
        const int rows0 = 16 * r0, nrows = 16 * min(nwv, TR - r0), tr = r0 + wv;
        double4_m acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = (double4_m){0.0, 0.0, 0.0, 0.0};
        for (int m0 = 0; m0 < Nb; m0 += kc) {
            const int cnt = min(kc, Nb - m0);
            for (int it = tid; it < nrows * kc; it += nt) {
                const int el = it / kc, m = it - el * kc, e = rows0 + el;
                double v = 0.0;
                if (e < N && m < cnt) {
                    const double* r = pos + 3 * e;
                    const double4_t rec = gld((const double4_t*)(s.btab + 4 * (m0 + m)));
                    const double dx = r[0] - rec[0], dy = r[1] - rec[1], dz = r[2] - rec[2];
                    v = basis_value_d(gld(s.btype + m0 + m), rec[3], dx, dy, dz,
                                      dx * dx + dy * dy + dz * dz);
                }
                Bc[el * ldc + m] = v;
            }
            if (stage) {
                for (int idx = tid; idx < ctot; idx += nt) {
                    const int m = idx / w16, col = idx - m * w16;
                    Cc[m * ldcc + col] = (m < cnt && col < ns)
                                             ? gld(s.C64 + (long)(m0 + m) * s.Norb + col) : 0.0;
                }
            }
            __syncthreads();
            if (tr < TR) {
                for (int k0 = 0; k0 < cnt; k0 += 4) {
                    const int mu = m0 + k0 + k4;
                    const double av = Bc[(16 * wv + i16) * ldc + k0 + k4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (t >= TC) continue;
                        const int col = 16 * t + i16;
                        const double bv = stage ? Cc[(k0 + k4) * ldcc + col]
                                                : ((col < ns && k0 + k4 < cnt)
                                                       ? gld(s.C64 + (long)mu * s.Norb + col) : 0.0);
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
        if (tr < TR) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= TC) continue;
                const int col = 16 * t + i16;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * tr + k4 + 4 * v;
                    if (row < N && col < ns) A64[(long)row * ns + col] = acc[t][v];
                }
            }
        }
    }
}

// Z[mu][c] = sum_k C[mu][k] Ainv[k][c] of spin sp (Ai64 holds AiT[c][k]) on
// MFMA: each wavefront takes row tiles of 16 basis functions with every
// column tile.  The inverse is staged in LDS once (row stride n + 1), and a
// tile's coefficient operands (at most 16 k-steps, n <= 64) are all fetched
// before its products, so that their latencies overlap.
__device__ __noinline__ void final_z(const DevMix& s, int sp, const double* AiT, double* Z)
{
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    const int n = mnspin(s, sp), Nb = s.Nb, ns = s.ns, ldt = n + 1;
    const int TR = (Nb + 15) / 16, TC = (n + 15) / 16;   // TC <= 4
    const int i16 = lane & 15, k4 = lane >> 4;
    double* T = LDSD(s.l_U);                     // [n][n + 1] AiT of the spin
    for (int idx = tid; idx < n * n; idx += nt) {
        const int c = idx / n, k = idx - c * n;
        T[c * ldt + k] = AiT[(long)c * ns + k];
    }
    __syncthreads();
    for (int tr = wv; tr < TR; tr += nwv) {
        double4_m acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = (double4_m){0.0, 0.0, 0.0, 0.0};
        const int mu_a = 16 * tr + i16;
        double av[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k = 4 * q + k4;
            av[q] = (mu_a < Nb && k < n) ? gld(s.C64 + (long)mu_a * s.Norb + k) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (4 * q >= n) break;
            const int k = 4 * q + k4;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= TC) continue;
                const int c = 16 * t + i16;
                const double bv = (c < n && k < n) ? T[c * ldt + k] : 0.0;
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv, acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= TC) continue;
            const int c = 16 * t + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int mu = 16 * tr + k4 + 4 * v;
                if (mu < Nb && c < n) Z[(long)c * Nb + mu] = acc[t][v];
            }
        }
    }
    __syncthreads();   // T is restaged by the next call
}

// ---------------------------------------------------------------------------
// FP64 estimator evaluation: everything recomputed from the positions in FP64
// (Slater rows, Gauss-Jordan inverses, ratios, Jastrow, local energy), so that
// e_L and W handed to the reconfiguration and the energy estimate carry no
// FP32 error.  The determinant ratios and derivatives are contracted as
// chi(r') . (C Ainv)[:, c]: Z = C Ainv is formed once per spin, after which each
// of the 6 moves, the gradient and the Laplacian of an electron is one dot
// product over the basis instead of an orbital row times a column.
// ---------------------------------------------------------------------------
__device__ __noinline__ MLocal mixed_final_fp64(const DevMix* __restrict__ dm, int wid, double a,
                                                int nu_mode, bool& ok)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x, nt = blockDim.x, ns = s.ns, N = s.N, P = s.P, Nb = s.Nb;
    const int lane = tid & 63;
    double* g64 = s.s64 + (long)wid * s.stride64;
    double* A64 = g64;                           // [N][ns]       Slater rows
    double* Ai64 = g64 + (long)N * ns;           // [2][ns][ns]   transposed inverses AiT[c][k]
    double* Z64 = Ai64 + 2L * ns * ns;           // [2][ns][Nb]   Z[c][mu] = sum_k C[mu][k] Ainv[k][c]
    const double* pos = LDSD(s.l_pos);
    const double* st64 = LDSD(s.l_ev);           // the walker's lattice step vectors
    double* F = LDSD(s.l_F);
    double* R64 = F;                             // [P]
    double* gD64 = F + P;                        // [N][4]
    double* dJ64 = gD64 + 4 * N;                 // [P]
    double* Jg64 = dJ64 + P;                     // [N][3]
    double* Jl64 = Jg64 + 3 * N;                 // [N]
    double* nue = LDSD(s.l_nue);
    double* nua = LDSD(s.l_nua);
    double* red = LDSD(s.l_red);
    // Slater rows on MFMA
    final_slater_rows(s, pos, A64);
    global_handoff();
    ok = gj_inverse<double, double>(s, A64, Ai64, 0);
    ok = gj_inverse<double, double>(s, A64, Ai64 + (long)ns * ns, 1) && ok;
    // Z = C Ainv per spin on MFMA
    for (int sp = 0; sp < 2; ++sp)
        if (mnspin(s, sp)) final_z(s, sp, Ai64 + (long)sp * ns * ns, Z64 + (long)sp * Nb * ns);
    global_handoff();
    // per electron: the 6 neighbour values, gradient and Laplacian of the
    // basis, each contracted with Z[c][:].  A group of 16 adjacent lanes serves
    // one electron (functions mu = g, g + 16, ...: coalesced reads of Z[c]),
    // its partial sums combined over the group by DPP (row mirrors), with no
    // barrier per electron.  A Gaussian's values at the six neighbours follow
    // from exp(-alpha d^2), exp(-alpha a^2) and exp(-+2 alpha a d_c)
    // (d = r - centre; exponent clamped to +-700, where the value at r has
    // underflowed); Slater functions take the seven points directly
    {
        const int g16 = lane & 15, ngrp = nt >> 4;
        for (int i0 = 0; i0 < N; i0 += ngrp) {
            const int i = i0 + (tid >> 4);
            double t[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            if (i < N) {
                const int sp = mspin(s, i), c = mcol(s, i);
                const double* Zc = Z64 + (long)sp * Nb * ns + (long)c * Nb;
                const double* ri = pos + 3 * i;
                // the next function's Z entry and record are fetched while
                // the current one is evaluated
                double zn = g16 < Nb ? Zc[g16] : 0.0;
                double4_t recn = gld((const double4_t*)(s.btab + 4 * (g16 < Nb ? g16 : 0)));
                int tyn = gld(s.btype + (g16 < Nb ? g16 : 0));
                for (int mu = g16; mu < Nb; mu += 16) {
                    const double z = zn;
                    const double4_t rec = recn;
                    const int ty = tyn;
                    const int mn = mu + 16 < Nb ? mu + 16 : mu;
                    zn = Zc[mn];
                    recn = gld((const double4_t*)(s.btab + 4 * mn));
                    tyn = gld(s.btype + mn);
                    const double al = rec[3];
                    const double d[3] = {ri[0] - rec[0], ri[1] - rec[1], ri[2] - rec[2]};
                    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    double v, gg[3], l;
                    if (ty == 4) {
                        for (int q = 1; q <= 6; ++q) {
                            double pq[3];
                            point_qv(ri, q, st64, pq);
                            const double dx = pq[0] - rec[0], dy = pq[1] - rec[1], dz = pq[2] - rec[2];
                            t[q - 1] += z * basis_value_d(ty, al, dx, dy, dz, dx * dx + dy * dy + dz * dz);
                        }
                        basis_vgl_d(ty, al, d[0], d[1], d[2], d2, v, gg, l);
                    } else {
                        const double e = exp(-al * d2), K = exp(-al * a * a);
                        const int ax = ty - 1;
                        const double f0 = ty == 0 ? 1.0 : d[ax];
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            const double sdc = d[0] * st64[3 * cc] + d[1] * st64[3 * cc + 1] +
                                               d[2] * st64[3 * cc + 2];
                            const double x = fmin(fmax(-2.0 * al * sdc, -700.0), 700.0);
                            const double tc = exp(x);
                            const double sp = ty != 0 ? st64[3 * cc + (ax < 0 ? 0 : ax)] : 0.0;
                            const double fp = f0 + sp;
                            const double fm = f0 - sp;
                            t[2 * cc] += z * (fp * (e * (K * tc)));
                            t[2 * cc + 1] += z * (fm * (e * (K * recip(tc))));
                        }
                        if (ty == 0) {
                            v = e;
#pragma unroll
                            for (int cc = 0; cc < 3; ++cc) gg[cc] = -2.0 * al * d[cc] * e;
                            l = (4.0 * al * al * d2 - 6.0 * al) * e;
                        } else {
                            v = f0 * e;
#pragma unroll
                            for (int cc = 0; cc < 3; ++cc)
                                gg[cc] = ((cc == ax) ? e : 0.0) - 2.0 * al * f0 * d[cc] * e;
                            l = f0 * e * (4.0 * al * al * d2 - 10.0 * al);
                        }
                    }
                    t[6] += z * gg[0]; t[7] += z * gg[1]; t[8] += z * gg[2]; t[9] += z * l;
                }
            }
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                double w = t[q];
                w += dpp_mov<0xb1, 0xf>(w);       // quad_perm [1,0,3,2]
                w += dpp_mov<0x4e, 0xf>(w);       // quad_perm [2,3,0,1]
                w += dpp_mov<0x141, 0xf>(w);      // row_half_mirror
                w += dpp_mov<0x140, 0xf>(w);      // row_mirror
                t[q] = w;
            }
            if (i < N && g16 == 0) {
#pragma unroll
                for (int q = 0; q < 6; ++q) R64[6 * i + q] = t[q];
#pragma unroll
                for (int q = 0; q < 4; ++q) gD64[4 * i + q] = t[6 + q];
            }
        }
        __syncthreads();
    }
    // Jastrow: exponent changes of the 6N moves, gradients and Laplacians;
    // potentials and V_ee.  Two threads per electron (adjacent lanes, partners
    // k = h, h + 2, ...), combined over the lane pair; the six neighbours'
    // squared distances from each pair's difference d as |d|^2 + a^2 +- 2 d.st_c
    const int K = N + s.M;
    const double aa = a * a;
    double vee = 0.0;
    for (int base = 0; base < 2 * N; base += nt) {
        const int it = base + tid, j = it >> 1, h = it & 1;
        const bool jv = it < 2 * N;
        const double* rj = pos + 3 * (jv ? j : 0);
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0, nu = 0.0, nv = 0.0;
        double dq[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        #pragma unroll 1
        for (int k = h; jv && k < K; k += 2) {
            if (k == j) continue;
            const bool isel = k < N;
            double pk[3];
            int jr;
            mpartner(s, pos, j, k, pk, jr);
            const double d[3] = {rj[0] - pk[0], rj[1] - pk[1], rj[2] - pk[2]};
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], ir = rsqrt_nr(r2);
            if (isel || s.has_en) {
                const double* pj = s.jas + 3 * jr;
                double u, dur, lp;
                pade_derivs(pj, r2 * ir, u, dur, lp);
                g0 += dur * d[0]; g1 += dur * d[1]; g2 += dur * d[2];
                l += lp;
                if (isel && k > j) vee += ir;
                const double b2 = r2 + aa;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double t2 = 2.0 * (d[0] * st64[3 * c] + d[1] * st64[3 * c + 1] +
                                             d[2] * st64[3 * c + 2]);
                    dq[2 * c] += pade_u(pj, sqrt(fmax(b2 + t2, 0.0))) - u;
                    dq[2 * c + 1] += pade_u(pj, sqrt(fmax(b2 - t2, 0.0))) - u;
                }
            }
            if (!isel) {
                double a1, a2;
                nuc_pot(s, k - N, r2, ir, 1.0 / a, a1, a2);
                nu += a1; nv += a2;
            }
        }
        g0 += dpp_mov<0xb1, 0xf>(g0); g1 += dpp_mov<0xb1, 0xf>(g1); g2 += dpp_mov<0xb1, 0xf>(g2);
        l += dpp_mov<0xb1, 0xf>(l);
        nu += dpp_mov<0xb1, 0xf>(nu); nv += dpp_mov<0xb1, 0xf>(nv);
#pragma unroll
        for (int q = 0; q < 6; ++q) dq[q] += dpp_mov<0xb1, 0xf>(dq[q]);
        if (jv && h == 0) {
            Jg64[3 * j] = g0; Jg64[3 * j + 1] = g1; Jg64[3 * j + 2] = g2; Jl64[j] = l;
            nue[j] = nu; nua[j] = nv;
#pragma unroll
            for (int q = 0; q < 6; ++q) dJ64[6 * j + q] = dq[q];
        }
    }
    vee = block_sum(vee, red);
    // ratios, lattice diagonal, local energy (App. D), as in the FP64 kernel
    double bs = 0.0;
    int anyneg = 0;
    for (int p = tid; p < P; p += (int)blockDim.x) {
        const double r = R64[p] * exp(dJ64[p]);
        R64[p] = r;
        if (r > 0) bs += r;
        else if (r < 0) anyneg = 1;
    }
    const bool anynode = block_sum(anyneg ? 1.0 : 0.0, red) > 0.0;
    bs = block_sum(bs, red);
    double econt = 0.0, dnu = 0.0;
    const double ia2 = 1.0 / (a * a);
    for (int j = tid; j < N; j += (int)blockDim.x) {
        const double j0 = Jg64[3 * j], j1 = Jg64[3 * j + 1], j2 = Jg64[3 * j + 2];
        const double lap = gD64[4 * j + 3] +
                           2.0 * (gD64[4 * j] * j0 + gD64[4 * j + 1] * j1 + gD64[4 * j + 2] * j2) +
                           Jl64[j] + j0 * j0 + j1 * j1 + j2 * j2;
        double lapA = 0.0;
        int nd = 0;
        for (int q = 0; q < 6; ++q) {
            const double r = R64[6 * j + q];
            lapA += (r - 1.0) * ia2;
            if (r < 0) nd = 1;
        }
        if (nu_mode == 1) nd = anynode;
        if (nu_mode == 2) nd = 1;
        const double nuzv = nue[j] + 0.5 * (lapA - lap);
        const double numax = nuzv > nua[j] ? nuzv : nua[j];
        econt += -0.5 * lap + nue[j];
        dnu += (nd ? numax : nuzv) - nuzv;
    }
    econt = block_sum(econt, red);
    dnu = block_sum(dnu, red);
    if (tid == 0) LDSD(s.l_scal)[kScVee] = vee;
    MLocal L;
    L.bbar = bs / (2.0 * a * a);
    L.eL = econt + vee + s.vii + dnu;
    L.W = L.eL + L.bbar;
    return L;
}

// heat-bath choice over the block: first p with cumulative positive ratio > xi * total
__device__ __noinline__ int mixed_heat_bath(const DevMix* __restrict__ dm, double xi, double pre,
                                            double tot)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x;
    const float* R = LDSF(s.l_R);
    int* pick = reinterpret_cast<int*>(LDSD(s.l_red) + 4);
    const int per = (s.P + (int)blockDim.x - 1) / (int)blockDim.x;
    const int p0 = tid * per, p1 = min(p0 + per, s.P);
    double c = pre;
    if (!(tot > 0)) return -1;
    const double t = xi * tot;
    int found = s.P, lastpos = -1;
    for (int p = p0; p < p1; ++p) {
        const double r = 1.0 + (double)R[p];
        if (r > 0) {
            c += r;
            lastpos = p;
            if (found == s.P && c > t) found = p;
        }
    }
    if (tid == 0) { pick[0] = s.P; pick[1] = -1; }
    __syncthreads();
    if (found < s.P) atomicMin(pick, found);
    if (lastpos >= 0) atomicMax(pick + 1, lastpos);
    __syncthreads();
    const int res = pick[0] < s.P ? pick[0] : pick[1];
    __syncthreads();
    return res;
}

// apply move p: Sherman-Morrison on the moved spin's inverse (HBM), new rows of
// the moved electron, determinant gradients of the moved spin, Jastrow caches,
// ratios of the moved spin
__device__ __noinline__ bool mixed_apply_move(const DevMix* __restrict__ dm, float* st, double a, int p)
{
    const DevMix& s = *dm;
    const int tid = threadIdx.x, ns = s.ns;
    const int i = p / 6, d = (p / 2) % 3, sg = p % 2;
    const int sp = mspin(s, i), c = mcol(s, i), n = mnspin(s, sp);
    const double ia = 1.0 / a;
    double* pos = LDSD(s.l_pos);
    float* Rdet = LDSF(s.l_Rdet);
    const float Rd = 1.0f + Rdet[p];
    const double rold[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    const double* st64 = LDSD(s.l_ev);
    const float* st32 = LDSF(s.l_ev + 72);
    double rnew[3];
    point_qv(rold, 2 * d + sg + 1, st64, rnew);

    // new orbital rows of electron i first: the basis block is then free for
    // the LDS copy of the moved spin's inverse
    mixed_rows(&s, i, rnew, a);

    // Sherman-Morrison on the LDS copy (row stride ns + 1), written back to
    // HBM; the ratio and gradient products below read the same copy
    float* Ai = st + s.g_AinvT + (long)sp * ns * ns;
    const float* Phi = st + s.g_Phi + (long)sp * ns * 6 * ns;
    const int lda = ns + 1, nt = (int)blockDim.x;
    float* AiL = LDSF(s.l_U);
    float* tmp = LDSF(s.l_tmp);
    float* u = tmp;               // [ns] accepted orbital row
    float* rowc = tmp + ns;       // [ns] column c of the inverse
    float* beta = tmp + 2 * ns;   // [ns]
    const int q2 = 6 * c + 2 * d;                 // difference and second-difference rows
    typedef float f4v __attribute__((ext_vector_type(4)));
    // rows of the inverse in float4 pieces when that still gives every lane
    // a piece
    const int q4 = ns >> 2;
    const bool vec4 = (ns & 3) == 0 && n * q4 >= nt;
    if (vec4) {
        const f4v* A4 = reinterpret_cast<const f4v*>(Ai);
        for (int i0 = tid; i0 < n * q4; i0 += 4 * nt) {
            f4v v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (i0 + t * nt < n * q4) v[t] = gld(A4 + i0 + t * nt);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int idx = i0 + t * nt;
                if (idx < n * q4) {
                    const int r = idx / q4, k0 = 4 * (idx - r * q4);
                    float* dst = AiL + r * lda + k0;
                    dst[0] = v[t].x; dst[1] = v[t].y; dst[2] = v[t].z; dst[3] = v[t].w;
                }
            }
        }
    } else {
        for (int idx = tid; idx < n * ns; idx += nt) {
            const int r = idx / ns;
            AiL[r * lda + idx - r * ns] = gld(Ai + idx);
        }
    }
    // the accepted orbital row u = phi(r_i +- st_d) = phi(r_i) + (+-D + S) / 2
    for (int k = tid; k < n; k += nt) {
        const float dd = gld(Phi + (long)k * 6 * ns + q2), ss = gld(Phi + (long)k * 6 * ns + q2 + 1);
        u[k] = gld(st + s.g_Arow + (long)i * ns + k) + 0.5f * (sg ? ss - dd : ss + dd);
        rowc[k] = gld(Ai + (long)c * ns + k);
    }
    __syncthreads();
    {
        // beta[cc] = u . AiL[cc]: kc threads per row (1, 2 or 4), k strided,
        // summed over the kc lanes
        const int kc = nt >= 4 * n ? 4 : (nt >= 2 * n ? 2 : 1);
        const int cc = tid / kc, ch = tid - cc * kc;
        for (int c0 = 0; c0 < n; c0 += nt / kc) {
            const int row = c0 + cc;
            float v = 0.f;
            if (row < n)
                for (int k = ch; k < n; k += kc) v += u[k] * AiL[row * lda + k];
            if (kc >= 2) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, false));
            if (kc == 4) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4e, 0xf, 0xf, false));
            if (row < n && ch == 0) beta[row] = v;
        }
    }
    __syncthreads();
    // the Sherman-Morrison denominator u . Ainv[:, c] as the dot product itself
    // (beta[c]), so that the updated inverse is that of the updated rows to
    // FP32 rounding even where the ratio is small
    const float iR = 1.0f / beta[c];
    if (vec4) {
        // four consecutive k per lane, one float4 store (columns k >= n of a
        // smaller spin block are padding and receive zeros)
        f4v* A4 = reinterpret_cast<f4v*>(Ai);
        for (int idx = tid; idx < n * q4; idx += nt) {
            const int cc = idx / q4, k0 = 4 * (idx - cc * q4);
            const float bc = beta[cc] * iR;
            float o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = k0 + t;
                float v = 0.f;
                if (k < n) {
                    v = cc == c ? rowc[k] * iR : AiL[cc * lda + k] - rowc[k] * bc;
                    AiL[cc * lda + k] = v;
                }
                o[t] = v;
            }
            f4v w;
            w.x = o[0]; w.y = o[1]; w.z = o[2]; w.w = o[3];
            gst(A4 + idx, w);
        }
    } else {
        for (int idx = tid; idx < n * n; idx += nt) {
            const int cc = idx / n, k = idx - cc * n;
            const float v = cc == c ? rowc[k] * iR : AiL[cc * lda + k] - rowc[k] * (beta[cc] * iR);
            AiL[cc * lda + k] = v;
            gst(Ai + (long)cc * ns + k, v);
        }
    }
    for (int k = tid; k < n; k += nt) gst(st + s.g_Arow + (long)i * ns + k, u[k]);
    __syncthreads();
    mixed_store_rows(&s, st, i, false);
    mixed_spin_update(&s, st, sp, true);

    // Jastrow caches of the moved electron (7 points) and of its partners
    const int K = s.N + s.M;
    float* dJ = LDSF(s.l_dJ);
    float* Jg = LDSF(s.l_Jg);
    float* Jl = LDSF(s.l_Jl);
    float* dje = LDSF(s.l_dje);
    double* red = LDSD(s.l_red);
    // every partner of the moved electron once: its gradient, Laplacian and
    // potentials at the new position, the exponent changes of its six next
    // moves (from the same FP64 difference), and the pair-term changes of the
    // partners; one block reduction of the 13 sums
    const float aa = (float)(a * a);
    double g0 = 0, g1 = 0, g2 = 0, l = 0, dvee = 0, nu = 0, nua = 0;
    float dq[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    #pragma unroll 1
    for (int k = tid; k < K; k += (int)blockDim.x) {
        if (k == i) continue;
        const bool isel = k < s.N;
        double pk[3];
        int jr;
        mpartner(s, pos, i, k, pk, jr);
        const PadeF prm = pade_row(s, jr);
        const double n0 = rnew[0] - pk[0], n1 = rnew[1] - pk[1], n2 = rnew[2] - pk[2];
        const double rn2 = n0 * n0 + n1 * n1 + n2 * n2, irn = rsqrt_nr(rn2);
        if (isel || s.has_en) {
            float un, dnr, lpn;
            pade_derivs_rf(prm, (float)(rn2 * irn), (float)irn, un, dnr, lpn);
            g0 += dnr * n0; g1 += dnr * n1; g2 += dnr * n2;
            l += lpn;
            const float f[3] = {(float)n0, (float)n1, (float)n2};
            neighbour_du(prm, f, (float)rn2, aa, st32, dq);
            if (isel) {
                const double o0 = rold[0] - pk[0], o1 = rold[1] - pk[1], o2 = rold[2] - pk[2];
                const double ro2 = o0 * o0 + o1 * o1 + o2 * o2, iro = rsqrt_nr(ro2);
                float uo, dor, lpo;
                pade_derivs_rf(prm, (float)(ro2 * iro), (float)iro, uo, dor, lpo);
                dje[k] = un - uo;
                Jg[3 * k] += (float)(-(dnr * n0) + dor * o0);
                Jg[3 * k + 1] += (float)(-(dnr * n1) + dor * o1);
                Jg[3 * k + 2] += (float)(-(dnr * n2) + dor * o2);
                Jl[k] += lpn - lpo;
                dvee += irn - iro;
            }
        }
        if (!isel) {
            double a1, a2;
            nuc_pot(s, k - s.N, rn2, irn, ia, a1, a2);
            nu += a1; nua += a2;
        }
    }
    float* dJi = tmp + 3 * ns;                   // [6] new exponent changes of electron i
    {
        double* red13 = red + 8;                 // [waves][13]
        const int lane = tid & 63, wv = tid >> 6, nwv = (int)blockDim.x >> 6;
        double sv[13] = {g0, g1, g2, l, dvee, nu, nua, dq[0], dq[1], dq[2], dq[3], dq[4], dq[5]};
#pragma unroll
        for (int t = 0; t < 13; ++t) {
            const double v = wave_sum(sv[t]);
            if (lane == 0) red13[wv * 13 + t] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 13; ++t) {
            double v = red13[t];
            for (int q = 1; q < nwv; ++q) v += red13[q * 13 + t];
            sv[t] = v;
        }
        g0 = sv[0]; g1 = sv[1]; g2 = sv[2]; l = sv[3]; dvee = sv[4]; nu = sv[5]; nua = sv[6];
#pragma unroll
        for (int t = 0; t < 6; ++t)
            if (tid == t) dJi[t] = (float)sv[7 + t];
    }
    // Jastrow exponent changes of the other electrons' moves
    for (int qp = tid; qp < s.P; qp += (int)blockDim.x) {
        const int j = qp / 6;
        if (j == i) continue;
        const PadeF prm = pade_row(s, mee_row(s, i, j));
        double r2[3];
        point_qv(pos + 3 * j, qp - 6 * j + 1, st64, r2);
        const float n0 = (float)(r2[0] - rnew[0]), n1 = (float)(r2[1] - rnew[1]),
                    n2 = (float)(r2[2] - rnew[2]);
        const float o0 = (float)(r2[0] - rold[0]), o1 = (float)(r2[1] - rold[1]),
                    o2 = (float)(r2[2] - rold[2]);
        const float un = pade_u2f(prm, n0 * n0 + n1 * n1 + n2 * n2);
        const float uo = pade_u2f(prm, o0 * o0 + o1 * o1 + o2 * o2);
        dJ[qp] += (un - uo) - dje[j];
    }
    __syncthreads();
    if (tid == 0) {
        for (int qq = 0; qq < 6; ++qq) dJ[6 * i + qq] = dJi[qq];
        Jg[3 * i] = (float)g0; Jg[3 * i + 1] = (float)g1; Jg[3 * i + 2] = (float)g2;
        Jl[i] = (float)l;
        LDSD(s.l_nue)[i] = nu; LDSD(s.l_nua)[i] = nua;
        LDSD(s.l_scal)[kScVee] += dvee;
        pos[3 * i] = rnew[0]; pos[3 * i + 1] = rnew[1]; pos[3 * i + 2] = rnew[2];
    }
    __syncthreads();
    mixed_full_ratios(s);
    return fabsf(Rd) < 1e-6f;
}

// ---------------------------------------------------------------------------
// the phase kernel: one workgroup (128 or 256 threads) per walker, the walkers
// of every system of the batch in one launch (workgroups of system k are
// start[k] .. start[k+1]-1).  build != 0 first evaluates every electron's
// orbital rows from its position.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMixThreads) void phase_mixed(MixBatch b, PhaseArgs pa, int build)
{
    int k = 0;
    while (k + 1 < b.nsys && (int)blockIdx.x >= b.start[k + 1]) ++k;
    const DevMix& s = b.tab[k];
    const int wid = (int)blockIdx.x - b.start[k];
    if (wid >= s.nw) return;
    const int jb = *s.jp;
    const double E0 = *s.e0p;
    const int tid = threadIdx.x;
    float* st = s.state + (long)wid * s.stride;
    double* pos = LDSD(s.l_pos);
    for (int q = tid; q < 3 * s.N; q += (int)blockDim.x) pos[q] = s.pos[(long)wid * 3 * s.N + q];
    // lattice step vectors of this walker for this phase: the coordinate axes,
    // or a random orientation drawn from its own Philox stream
    if (tid == 0) {
        double stp[9];
        if (pa.rotate) lattice_steps(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb, pa.a, stp);
        else lattice_steps_fixed(pa.a, stp);
        for (int q = 0; q < 9; ++q) {
            LDSD(s.l_ev)[q] = stp[q];
            LDSF(s.l_ev + 72)[q] = (float)stp[q];
        }
    }
    __syncthreads();
    const double a = pa.a;
    // every electron's orbital rows from its position: for new walkers, and
    // at every phase of a randomized lattice (the neighbour rows depend on the
    // orientation drawn for the phase)
    if (build || pa.rotate) {
        for (int j = 0; j < s.N; ++j) {
            const double r[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
            mixed_rows(&s, j, r, a);
            mixed_store_rows(&s, st, j, true);
        }
    }
    unsigned long long n_neg = 0, n_nomove = 0, n_refresh = 1, n_small = 0, n_sing = 0,
                       n_capped = 0;
    // rows rebuilt from positions are inverted afresh; otherwise the carried
    // inverse (the walker's own, or its parent's after the reconfiguration)
    // is corrected like a scheduled refresh
    if (!mixed_refresh(&s, st, a, !build)) n_sing++;

    double lw = s.lw[wid];
    // load-balanced weight factors bbar / (W - E_0) multiplied in blocks
    // (lw_block_update): one logarithm per 32 steps instead of one per step
    double wprod = 1.0;
    double tau_left = pa.tau;
    int it = 0, since = 0, n_sched = 0;
    MLocal L;
    int32_t* tr = s.trace ? s.trace + (long)wid * s.trace_cap : nullptr;
    for (;;) {
        if (pa.scheme == 0 && it >= pa.nproj) break;
        L = mixed_evaluate(&s, a, pa.nu_mode);
        int q;
        if (pa.scheme == 0) {
            const double den = L.W - E0;
            if (!(den > 0)) { lw = -INFINITY; n_neg++; }
            else if (!(L.bbar > 0)) { lw = -INFINITY; n_nomove++; }
            else {
                lw_block_update(lw, wprod, L.bbar, den, it + 1);
            }
            const double xi = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb,
                                             (uint64_t)it, kMove);
            q = mixed_heat_bath(&s, xi, L.pre, L.tot);
            if (tr && it < s.trace_cap && tid == 0) tr[it] = q;
            ++it;
        } else {
            const double xt = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb,
                                             (uint64_t)it, kPersist);
            const double t = (L.bbar > 0) ? -log1p(-xt) / L.bbar : INFINITY;
            if (!(L.bbar > 0)) n_nomove++;
            const bool capped = it + 1 >= pa.conv_cap;
            if (capped && t < tau_left) n_capped++;
            const bool stop = !(t < tau_left) || capped;
            const double tx = stop ? tau_left : t;
            lw -= tx * L.eL;
            tau_left = stop ? 0.0 : tau_left - tx;
            ++it;
            if (stop) {
                if (tr && it - 1 < s.trace_cap && tid == 0) tr[it - 1] = -1;
                break;
            }
            const double xi = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb,
                                             (uint64_t)(it - 1), kMove);
            q = mixed_heat_bath(&s, xi, L.pre, L.tot);
            if (tr && it - 1 < s.trace_cap && tid == 0) tr[it - 1] = q;
        }
        if (q >= 0) {
            const bool small = mixed_apply_move(&s, st, a, q);
            ++since;
            if (small) n_small++;
            if (small || since >= pa.refresh_every) {
                const bool jas = small || ++n_sched % kJastrowEvery == 0;
                if (!mixed_refresh(&s, st, a, !small, jas)) n_sing++;
                n_refresh++;
                since = 0;
            }
        }
    }
    lw += log(wprod);
    // estimator values at the final configuration, in FP64; beside them the
    // values the mixed-precision step computed there, and the largest ratio
    // error, for the error report
    {
        if (pa.scheme == 0) L = mixed_evaluate(&s, a, pa.nu_mode);
        const MLocal Lm = L;
        bool ok64 = true;
        L = mixed_final_fp64(&s, wid, a, pa.nu_mode, ok64);
        if (!ok64) n_sing++;
        // the estimator weight w / (W - E_0) at the final configuration needs
        // W - E_0 > 0 as every step's factor does: otherwise the walker dies
        if (pa.scheme == 0 && pa.nproj > 0 && !(L.W - E0 > 0)) { lw = -INFINITY; n_neg++; }
        if (s.diag) {
            const float* R = LDSF(s.l_R);
            const double* R64 = LDSD(s.l_F);
            double e = 0.0;
            for (int p = tid; p < s.P; p += (int)blockDim.x)
                e = fmax(e, fabs((1.0 + (double)R[p]) - R64[p]) / fmax(1.0, fabs(R64[p])));
            e = block_max(e, LDSD(s.l_red));
            if (tid == 0) {
                double* dg = s.diag + (long)wid * 4;
                dg[0] = Lm.eL; dg[1] = Lm.W; dg[2] = Lm.bbar; dg[3] = e;
            }
        }
    }

    const bool nonfinite = !(isfinite(L.eL) && isfinite(L.W)) || isnan(lw) || lw == INFINITY;
    for (int q = tid; q < 3 * s.N; q += (int)blockDim.x) s.pos[(long)wid * 3 * s.N + q] = pos[q];
    if (tid == 0) {
        s.lw[wid] = lw;
        s.eL[wid] = L.eL;
        s.Wd[wid] = L.W;
        s.iters[wid] = it;
        unsigned long long* cn = pa.counters;
        atomicAdd(cn + kCntIters, (unsigned long long)it);
        if (n_neg) atomicAdd(cn + kCntNegW, n_neg);
        if (n_nomove) atomicAdd(cn + kCntNoMove, n_nomove);
        atomicAdd(cn + kCntRefresh, n_refresh);
        if (n_small) atomicAdd(cn + kCntSmallR, n_small);
        if (n_sing) atomicAdd(cn + kCntSingular, n_sing);
        if (n_capped) atomicAdd(cn + kCntCapped, n_capped);
        if (nonfinite) atomicAdd(cn + kCntNonfinite, 1ull);
        atomicMax(cn + kCntMaxIters, (unsigned long long)it);
        atomicMin(cn + kCntMinIters, (unsigned long long)it);
    }
}

// gather of whole mixed walker blocks after the comb (state double-buffered)
__global__ void branch_gather_mixed(const DevMix* __restrict__ sys, const int32_t* sel,
                                    const float* old_state, const double* pos_old,
                                    const double* eL_old, const double* W_old)
{
    const DevMix& s = *sys;
    const int al = blockIdx.x;
    if (al >= s.nw) return;
    const int b = sel[al];
    const float4_t* src = reinterpret_cast<const float4_t*>(old_state + (long)b * s.stride);
    float4_t* dst = reinterpret_cast<float4_t*>(s.state + (long)al * s.stride);
    for (long q = threadIdx.x; q < s.stride / 4; q += blockDim.x) dst[q] = src[q];
    for (int q = threadIdx.x; q < 3 * s.N; q += blockDim.x)
        s.pos[(long)al * 3 * s.N + q] = pos_old[(long)b * 3 * s.N + q];
    if (threadIdx.x == 0) {
        s.lw[al] = 0.0;
        s.eL[al] = eL_old[b];
        s.Wd[al] = W_old[b];
    }
}

}  // namespace lrdmc
