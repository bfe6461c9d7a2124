// Projection phase of lattice-regularized DMC on gfx950: one wavefront per
// walker, the walker's hot state resident in LDS for the whole phase.
//
// One phase = the inner loop of Algorithm 1 (conventional: iterate until the
// walker's remaining time tau_left reaches 0) or Algorithm 2 (load-balanced:
// N_proj steps).  Every iteration evaluates the guiding-function ratios of all
// 6N single-electron lattice moves (App. D discretized Laplacian), the
// fixed-node lattice diagonal W(x) with the spin-flip term and the regularized
// potential nu_opt (App. D), the local energy e_L = W - bbar (Sec. II.C), the
// weight update (Algorithm 1 / Algorithm 2), and a heat-bath choice of the
// move with probability p_{x',x} (Sec. II.C partition of the Green's
// function).
//
// Work per iteration is incremental: only the moved electron's orbital rows
// (its 6 new lattice neighbours, gradient and Laplacian) are evaluated; the
// rows of the other electrons are unchanged by definition.  The inverse
// Slater matrix of the moved spin is updated by Sherman-Morrison, the Jastrow
// caches by pair differences, and everything that accumulates rounding is
// rebuilt in FP64 every `refresh_every` moves (Gauss-Jordan with partial
// pivoting on the exact orbital rows).
#include <hip/hip_runtime.h>
#include <math.h>

#include "lrdmc_dev.hpp"
#include "lrdmc_devfn.hpp"

namespace lrdmc {

// Optional per-section cycle counters (instrumentation builds only): the
// wavefront's s_memtime clock accumulated per section and written out per
// walker.  Compiled away unless LRDMC_SECTION_TIMERS is defined.
#ifdef LRDMC_SECTION_TIMERS
#define LRDMC_T0() unsigned long long t_mark_ = __builtin_amdgcn_s_memtime()
#define LRDMC_T(k)                                                           \
    do {                                                                     \
        const unsigned long long t_now_ = __builtin_amdgcn_s_memtime();      \
        sect[k] += t_now_ - t_mark_;                                         \
        t_mark_ = t_now_;                                                    \
    } while (0)
#else
#define LRDMC_T0() (void)0
#define LRDMC_T(k) (void)0
#endif

// A workgroup is one wavefront: LDS operations of a wavefront complete in
// issue order, so exchanging data between its lanes through LDS needs only a
// compiler-level barrier (no s_barrier and no drain of outstanding memory
// operations).  Global-memory data written by one lane and read by another
// additionally needs block_visible().
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }
__device__ __forceinline__ void block_visible()
{
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

// Per-walker state: offsets (in doubles) of the LDS-resident arrays inside
// the dynamic shared-memory block, and the walker's block of the global
// spill area: the orbital rows at the moves, Phi[p][k] (row p = proposal p,
// row length n_s), and the orbital derivatives, dPhi[4 j + c][k] (c = x, y, z,
// Laplacian), so that the rows of one electron are contiguous and are written
// as whole cache lines when it moves.
extern __shared__ double lds[];

// orbital values per lane fetched ahead of the ratio and derivative updates
constexpr int kPre = 8;

struct Walker {
    int pos, R, Rdet, dJ, Arow, AinvT, Jg, Jl, nue, nua, dje, scal, B, rows, tmp, C, nuc, jas, gd, ev,
        Vnl, nlin;
    double* Phi;
    double* dPhi;
    double* ArowG;          // Slater rows in global memory (large-system kernel)
    double* AinvG;          // both inverses in global memory (one-spin LDS residency)
    double* GJg;            // the refresh's left half in global memory (same)
};

__device__ __forceinline__ Walker walker_view(const DevSys& s)
{
    Walker w;
    w.pos = s.o_pos; w.R = s.o_R; w.Rdet = s.o_Rdet; w.dJ = s.o_dJ; w.Arow = s.o_Arow;
    w.AinvT = s.o_AinvT; w.Jg = s.o_Jg; w.Jl = s.o_Jl; w.nue = s.o_nue; w.nua = s.o_nua;
    w.dje = s.o_dje; w.scal = s.o_scal; w.B = s.o_B; w.rows = s.o_rows; w.tmp = s.o_tmp;
    w.C = s.o_C;
    w.nuc = s.o_nuc;
    w.jas = s.o_jas;
    w.gd = s.o_gd;
    w.ev = s.o_ev;
    w.Vnl = s.o_Vnl;
    w.nlin = s.o_nlin;
    double* base = s.spill + (long)blockIdx.x * s.spill_stride;
    w.Phi = base + s.s_Phi;
    w.dPhi = base + s.s_dPhi;
    w.ArowG = base + s.s_Arow;
    w.AinvG = base + s.s_AinvG;
    w.GJg = base + s.s_GJ;
    return w;
}

__device__ __forceinline__ int spin_of(const DevSys& s, int i) { return i >= s.Nup; }
// proposals per configuration: the 6N lattice moves, and 6N quadrature
// points with a pseudopotential
template <bool kNl>
__device__ __forceinline__ int n_prop(const DevSys& s) { return kNl ? s.PT : s.P; }
__device__ __forceinline__ int col_of(const DevSys& s, int i) { return i >= s.Nup ? i - s.Nup : i; }
__device__ __forceinline__ int nspin(const DevSys& s, int sp) { return sp ? s.Ndn : s.Nup; }
__device__ __forceinline__ int ee_row(const DevSys& s, int i, int k)
{
    return ((i >= s.Nup) == (k >= s.Nup)) ? 0 : 1;
}

// Partner k of an electron: another electron (k < N, position in LDS) or a
// nucleus (k >= N).  Returns its position and the row of its Pade parameters.
__device__ __forceinline__ void partner(const DevSys& s, const Walker& w, int i, int k, double* pk,
                                       int& jrow)
{
    if (k < s.N) {
        pk[0] = lds[w.pos + 3 * k]; pk[1] = lds[w.pos + 3 * k + 1]; pk[2] = lds[w.pos + 3 * k + 2];
        jrow = ee_row(s, i, k);
    } else {
        const double* nr = lds + w.nuc + kNucLen * (k - s.N);
        pk[0] = nr[0]; pk[1] = nr[1]; pk[2] = nr[2];
        jrow = (int)nr[6];
    }
}

// Pade pair function u(r) = (A r + B r^2)/(1 + b r) from the squared distance.
__device__ __forceinline__ double pade_u2(const double* p, double r2)
{
    const double r = r2 * rsqrt_nr(r2);
    return r * (p[0] + p[1] * r) * recip(1.0 + p[2] * r);
}

// u, u'/r and u'' + 2u'/r from the squared distance r2 and ir = 1/r.
__device__ __forceinline__ void pade_derivs2(const double* p, double r2, double ir, double& u,
                                             double& du_r, double& lap)
{
    const double A = p[0], B = p[1], b = p[2];
    const double r = r2 * ir;
    const double iden = recip(1.0 + b * r);
    const double i2 = iden * iden;
    u = (A * r + B * r * r) * iden;
    const double du = (A + 2.0 * B * r + B * b * r * r) * i2;
    du_r = du * ir;
    lap = 2.0 * (B - A * b) * i2 * iden + 2.0 * du_r;
}

// Bare (-Z/r, and its value capped at r = a) or soft-core (-Z/sqrt(r^2 + rc^2))
// electron-nucleus potential of nucleus k at distance r (App. D potentials).
// From the squared distance r2, 1/r and 1/a.
__device__ __forceinline__ void nucleus_potential(const DevSys& s, const Walker& w, int k, double r2,
                                                  double ir, double ia, double& nu, double& nua)
{
    const double* nr = lds + w.nuc + kNucLen * (k - s.N);
    const double Z = nr[3];
    if (nr[5] == 0.0) {
        nu += -Z * ir;
        nua += -Z * (ir < ia ? ir : ia);
    } else {
        const double t = -Z * rsqrt_nr(r2 + nr[4] * nr[4]);
        nu += t; nua += t;
    }
}

// Non-local pseudopotential (App. D non-local elements under the determinant
// locality approximation).  The atom whose cutoff sphere holds r (the spheres
// do not overlap), or -1, and the distance rr to it.
__device__ __forceinline__ int nl_sphere(const DevSys& s, const Walker& w, const double* r, double& rr)
{
    rr = 0.0;
    for (int I = 0; I < s.M; ++I) {
        const double rc = gld(s.ecp_rcut + I);
        if (!(rc > 0.0)) continue;
        const double d = exact_distance(r, lds + w.nuc + kNucLen * I);
        if (d < rc) { rr = d; return I; }
    }
    return -1;
}

// Elements V_q = sum_l (2l + 1)/6 v_l(rr) P_l(cos theta_q) of electron j's six
// quadrature points (octahedral quadrature of the sphere of radius rr around
// atom I along the walker's versors; theta_q the angle between r - R_I and
// the point's direction), 0 outside every sphere.  Lanes 0..5, one point each.
__device__ void nl_elements(const DevSys& s, const Walker& w, int j, const double* r, int I,
                            double rr, int lane)
{
    if (lane < 6) {
        double V = 0.0;
        if (I >= 0) {
            const double* nr = lds + w.nuc + kNucLen * I;
            const double* uv = lds + w.ev + 9;
            const int d = lane >> 1;
            const double ud = (r[0] - nr[0]) * uv[3 * d] + (r[1] - nr[1]) * uv[3 * d + 1] +
                              (r[2] - nr[2]) * uv[3 * d + 2];
            const double cth = ((lane & 1) ? -ud : ud) / rr;
            double v0 = 0.0, v1 = 0.0, v2 = 0.0;
            for (int t = 0; t < s.necp; ++t) {
                if (gld(s.ecp_atom + t) != I) continue;
                const int l = gld(s.ecp_l + t), k = gld(s.ecp_pow + t);
                const double rp = k == 0 ? 1.0 : (k == 1 ? rr : rr * rr);
                const double v = gld(s.ecp_coef + t) * rp * exp(-gld(s.ecp_exp + t) * rr * rr);
                if (l == 0) v0 += v;
                else if (l == 1) v1 += v;
                else v2 += v;
            }
            V = (v0 + 3.0 * v1 * cth + 5.0 * v2 * (0.5 * (3.0 * cth * cth - 1.0))) / 6.0;
        }
        lds[w.Vnl + 6 * j + lane] = V;
    }
}

// Lattice point q of r (0: r itself, 1..6: the neighbours in move order):
// fixed axes r +- a e_d, or the walker's rotated step vectors st.
template <bool kRot>
__device__ __forceinline__ void lattice_point(const double* r, int q, double a, const double* st,
                                              double* o)
{
    if constexpr (kRot) point_qv(r, q, st, o);
    else point_q(r, q, a, o);
}

// Orbital rows of electron j at position r (11 rows, columns k < n_j):
// row 0 the value at r, rows 1..6 the values at the six lattice neighbours
// r +- a e_d (move order; e_d the walker's lattice versors, the coordinate
// axes or a random orientation), rows 7..9 the gradient, row 10 the Laplacian.
//
// Basis values: one lane per function.  A Gaussian factorizes along the
// versors, so at the neighbour r + s a e_c (s = +-1)
//   exp(-alpha |d + s a e_c|^2) = exp(-alpha d^2) exp(-alpha a^2) exp(-2 s alpha a d.e_c),
// with d = r - centre: four exponentials (the per-function constant
// exp(-alpha a^2) is tabulated with the system) and three reciprocals give all
// seven values, and the value at r gives the gradient and Laplacian.  Slater
// functions take the seven points directly.  Orbitals: the 11 x Nb basis
// block times the Nb x n coefficient block on FP64 MFMA (16x16x4 tiles; rows
// 11..15 and columns >= n are padding).
// kChunk: only the functions m0 <= mu < m1, at columns mu - m0 of the block.
template <bool kRot, bool kChunk = false>
__device__ void basis_rows(const DevSys& s, const Walker& w, const double* r, double a, int lane,
                           int m0 = 0, int m1 = 0)
{
    const int Nb = kChunk ? m1 : s.Nb, ldb = s.ldb;
    const double* st = lds + w.ev;      // lattice step vectors a e_d
    for (int mu = (kChunk ? m0 : 0) + lane; mu < Nb; mu += kWave) {
        const double4_t c = gld((const double4_t*)(s.btab + 4 * mu));
        const int t = gld(s.btype + mu);
        const double al = c[3];
        const double d[3] = {r[0] - c[0], r[1] - c[1], r[2] - c[2]};
        const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double* Bm = lds + w.B + (kChunk ? mu - m0 : mu);
        double v, g[3], l;
        if (t == 4) {
            for (int q = 1; q < 7; ++q) {
                double pq[3];
                lattice_point<kRot>(r, q, a, st, pq);
                const double dx = pq[0] - c[0], dy = pq[1] - c[1], dz = pq[2] - c[2];
                Bm[q * ldb] = basis_value_d(t, al, dx, dy, dz, dx * dx + dy * dy + dz * dz);
            }
            basis_vgl_d(t, al, d[0], d[1], d[2], d2, v, g, l);
        } else {
            const double e = exp(-al * d2);
            const double K = gld(s.bK + mu);
            const double s2a = 2.0 * al * a, m2al = -2.0 * al;
            // polynomial factor: 1 (s) or the displacement along the p axis
            const int ax = t - 1;
            const double f0 = t == 0 ? 1.0 : (ax == 0 ? d[0] : (ax == 1 ? d[1] : d[2]));
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                // -2 alpha a d.e_cc, clamped: beyond +-700 the value at r has
                // underflowed; the p factor moves by the step's component
                double x;
                if constexpr (kRot) {
                    const double sd = d[0] * st[3 * cc] + d[1] * st[3 * cc + 1] + d[2] * st[3 * cc + 2];
                    x = fmin(fmax(m2al * sd, -700.0), 700.0);
                } else {
                    x = fmin(fmax(-s2a * d[cc], -700.0), 700.0);
                }
                const double tc = exp(x);
                const double ep = e * (K * tc), em = e * (K * recip(tc));
                double fp, fm;
                if constexpr (kRot) {
                    const double sp = t != 0 ? st[3 * cc + (ax < 0 ? 0 : ax)] : 0.0;
                    fp = t != 0 ? f0 + sp : f0;
                    fm = t != 0 ? f0 - sp : f0;
                } else {
                    fp = (t != 0 && ax == cc) ? f0 + a : f0;
                    fm = (t != 0 && ax == cc) ? f0 - a : f0;
                }
                Bm[(2 * cc + 1) * ldb] = fp * ep;
                Bm[(2 * cc + 2) * ldb] = fm * em;
            }
            if (t == 0) {
                v = e;
                for (int cc = 0; cc < 3; ++cc) g[cc] = -2.0 * al * d[cc] * e;
                l = (4.0 * al * al * d2 - 6.0 * al) * e;
            } else {
                v = f0 * e;
                for (int cc = 0; cc < 3; ++cc) g[cc] = ((cc == ax) ? e : 0.0) - 2.0 * al * f0 * d[cc] * e;
                l = f0 * e * (4.0 * al * al * d2 - 10.0 * al);
            }
        }
        Bm[0] = v;
        Bm[7 * ldb] = g[0];
        Bm[8 * ldb] = g[1];
        Bm[9 * ldb] = g[2];
        Bm[10 * ldb] = l;
    }
}

// Basis values at the six quadrature points of a sphere (radius nlr around
// atom nlI, along the walker's versors) in rows 0..5 of the basis block: one
// lane per function, each point formed as the non-local move forms it.
__device__ void nl_basis_rows(const DevSys& s, const Walker& w, int nlI, double nlr, int lane)
{
    const int Nb = s.Nb, ldb = s.ldb;
    const double* nr = lds + w.nuc + kNucLen * nlI;
    for (int mu = lane; mu < Nb; mu += kWave) {
        const double4_t c = gld((const double4_t*)(s.btab + 4 * mu));
        const int t = gld(s.btype + mu);
        double* Bm = lds + w.B + mu;
        for (int q = 0; q < 6; ++q) {
            double pq[3];
            nl_point(nr, nlr, lds + w.ev + 9, q, pq);
            const double dx = pq[0] - c[0], dy = pq[1] - c[1], dz = pq[2] - c[2];
            Bm[q * ldb] = basis_value_d(t, c[3], dx, dy, dz, dx * dx + dy * dy + dz * dz);
        }
    }
}

// Orbital rows O[row][col] = sum_mu B[row][mu] C[mu][col] of electron j
// (rows 0..10) on the four-block FP64 MFMA v_mfma_f64_4x4x4f64: block
// b = (lane >> 2) & 3 holds A[b][i][k] at lane 16k + 4b + i, B[b][k][c] at
// lane 16k + 4b + c and D[b][i][c] at lane 16i + 4b + c.  Blocks 2t and 2t+1
// take column tile t of the pair and the even and odd k-steps; three
// accumulators cover the row tiles 0..3, 4..7 and 8..10.  kQuad: the six
// quadrature-point rows of a pseudopotential sphere instead (rows 0..5).
// kGlobalC: the coefficient block is read from global memory (L1/L2-resident,
// shared by every walker) instead of the walker's LDS copy, each k-step's
// operand fetched one step ahead.
// kChunk: the nc functions from m0 on (block columns 0..nc-1), added to the
// rows unless first.
template <bool kQuad = false, bool kGlobalC = false, bool kChunk = false>
__device__ void orbital_rows(const DevSys& s, const Walker& w, int j, int lane, int m0 = 0, int nc = 0,
                             bool first = true)
{
    wave_sync();
    const int Nb = kChunk ? nc : s.Nb, ldb = s.ldb;
    const int n = nspin(s, spin_of(s, j));
    const int lk = lane >> 4, lb = (lane >> 2) & 3, l4 = lane & 3;
    const int par = lb & 1, cb = lb >> 1;
    for (int ct0 = 0; 4 * ct0 < n; ct0 += 2) {
        const int col = 4 * (ct0 + cb) + l4;
        const bool cok = col < n;
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        double bnext = 0.0;
        if constexpr (kGlobalC) {
            const int mu = 4 * par + lk;
            bnext = (cok && mu < Nb) ? gld(s.C + (kChunk ? m0 + mu : mu) * s.Norb + col) : 0.0;
        }
        for (int k0 = 0; k0 < Nb; k0 += 8) {
            const int mu = k0 + 4 * par + lk;
            const bool kok = mu < Nb;
            double bv;
            if constexpr (kGlobalC) {
                bv = bnext;
                const int mn = mu + 8;
                bnext = (cok && mn < Nb) ? gld(s.C + (kChunk ? m0 + mn : mn) * s.Norb + col) : 0.0;
            } else {
                bv = (cok && kok) ? lds[w.C + mu * s.ns + col] : 0.0;
            }
            const double a0 = kok ? lds[w.B + l4 * ldb + mu] : 0.0;
            const double a1 = (kok && (!kQuad || l4 < 2)) ? lds[w.B + (4 + l4) * ldb + mu] : 0.0;
            const double a2 = (!kQuad && kok && l4 < 3) ? lds[w.B + (8 + l4) * ldb + mu] : 0.0;
            acc0 = __builtin_amdgcn_mfma_f64_4x4x4f64(a0, bv, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_4x4x4f64(a1, bv, acc1, 0, 0, 0);
            if constexpr (!kQuad) acc2 = __builtin_amdgcn_mfma_f64_4x4x4f64(a2, bv, acc2, 0, 0, 0);
        }
        // odd k-steps (block 2t + 1, four lanes up) into block 2t: row_shl:4
        acc0 += dpp_mov<0x104, 0xf>(acc0);
        acc1 += dpp_mov<0x104, 0xf>(acc1);
        if constexpr (!kQuad) acc2 += dpp_mov<0x104, 0xf>(acc2);
        const int c = 4 * (ct0 + cb) + l4, i = lane >> 4;
        if (par == 0 && c < n) {
            if constexpr (kChunk) {
                if (!first) {
                    acc0 += lds[w.rows + i * s.ns + c];
                    acc1 += lds[w.rows + (4 + i) * s.ns + c];
                    if (i < 3) acc2 += lds[w.rows + (8 + i) * s.ns + c];
                }
            }
            lds[w.rows + i * s.ns + c] = acc0;
            if (!kQuad || i < 2) lds[w.rows + (4 + i) * s.ns + c] = acc1;
            if constexpr (!kQuad)
                if (i < 3) lds[w.rows + (8 + i) * s.ns + c] = acc2;
        }
    }
    wave_sync();
}

// kBig: in chunks of s.bchunk basis functions (the basis block holds one
// chunk; the orbital rows accumulate over the chunks).
template <bool kRot, bool kNl = false, bool kBig = false>
__device__ void electron_rows(const DevSys& s, const Walker& w, int j, const double* r, double a,
                              int lane)
{
    if constexpr (kBig) {
        for (int m0 = 0; m0 < s.Nb; m0 += s.bchunk) {
            const int m1 = min(m0 + s.bchunk, s.Nb);
            basis_rows<kRot, true>(s, w, r, a, lane, m0, m1);
            orbital_rows<false, true, true>(s, w, j, lane, m0, m1 - m0, m0 == 0);
        }
    } else {
        basis_rows<kRot>(s, w, r, a, lane);
        orbital_rows<false, kNl>(s, w, j, lane);
    }
}

// Store electron j's rows: Slater row, the 6 neighbour rows, derivatives.
template <bool kNl = false, bool kBig = false>
__device__ void store_rows(const DevSys& s, const Walker& w, int j, int lane, bool arow)
{
    const int n = nspin(s, spin_of(s, j));
    for (int idx = lane; idx < 11 * n; idx += kWave) {
        const int row = idx / n, k = idx - row * n;
        const double v = lds[w.rows + row * s.ns + k];
        if (row == 0) {
            if (arow) {
                if constexpr (kBig) gst(w.ArowG + j * s.ns + k, v);
                else lds[w.Arow + j * s.ns + k] = v;
            }
        } else if (row <= 6) gst(w.Phi + (6 * j + row - 1) * s.ns + k, v);
        else gst(w.dPhi + (4 * j + row - 7) * s.ns + k, v);
    }
    block_visible();
}

// Non-local part of electron j at position r (after its lattice rows have
// been stored, so that the basis block and the row buffer are free): its
// sphere, the elements V_q and the in-sphere flag, and inside a sphere the
// quadrature-point orbital rows, stored as spilled rows 6N + 6j + q.  Outside
// every sphere those rows are not written: the flag keeps every reader off
// them.
__device__ void nl_rows(const DevSys& s, const Walker& w, int j, const double* r, int lane)
{
    double rr;
    const int I = nl_sphere(s, w, r, rr);
    nl_elements(s, w, j, r, I, rr, lane);
    if (lane == 0) lds[w.nlin + j] = I >= 0 ? 1.0 : 0.0;
    if (I < 0) { wave_sync(); return; }
    nl_basis_rows(s, w, I, rr, lane);
    orbital_rows<true, true>(s, w, j, lane);
    const int n = nspin(s, spin_of(s, j));
    for (int idx = lane; idx < 6 * n; idx += kWave) {
        const int q = idx / n, k = idx - q * n;
        gst(w.Phi + (s.P + 6 * j + q) * s.ns + k, lds[w.rows + q * s.ns + k]);
    }
    block_visible();
}

// The same Gauss-Jordan elimination for the large-system kernel, whose basis
// block holds n x n but not n x 2n values: the left half of [A^T | I] in the
// basis block (or in global memory), the right half in the spin's inverse
// block itself, so that the right half ends as AinvT.  The Slater rows are
// read from global memory.  On a singular matrix the inverse block is left
// undefined (the phase reports the singular refresh as an error).
__device__ bool refresh_inverse_split(const DevSys& s, const Walker& w, int sp, int lane)
{
    const int n = nspin(s, sp), off = sp ? s.Nup : 0, n2 = 2 * n, nn = n * n2;
    if (!n) return true;
    // left half [n][n]: the basis block, or global memory with one-spin
    // residency; right half [n][ns]: the inverse block of spin sp in LDS
    // (the resident block itself with one-spin residency)
    double* Lh = s.ainv1 ? w.GJg : lds + w.B;
    double* Rh = lds + w.AinvT + (s.ainv1 ? 0 : sp * s.ns * s.ns);
    auto at = [&](int r, int c) -> double& { return c < n ? Lh[r * n + c] : Rh[r * s.ns + c - n]; };
    for (int idx = lane; idx < nn; idx += kWave) {
        const int r = idx / n2, c = idx - r * n2;
        at(r, c) = c < n ? gld(w.ArowG + (off + c) * s.ns + r) : (c - n == r ? 1.0 : 0.0);
    }
    block_visible();
    for (int j = 0; j < n; ++j) {
        // pivot: the largest |L[r][j]|, r >= j, the first such row on ties
        double best = -1.0;
        int bi = -1;
        for (int r0 = 0; r0 < n; r0 += kWave) {
            const int r = r0 + lane;
            const double v = (r >= j && r < n) ? fabs(Lh[r * n + j]) : -1.0;
            const double m = wave_max(v);
            if (m > best) {
                best = m;
                const unsigned long long hit = __ballot(v == m);
                bi = r0 + __ffsll((long long)hit) - 1;
            }
        }
        if (!(best > 0.0)) return false;
        if (bi != j) {
            for (int c = lane; c < n2; c += kWave) {
                const double t = at(j, c);
                at(j, c) = at(bi, c);
                at(bi, c) = t;
            }
            block_visible();
        }
        const double pv = Lh[j * n + j];
        block_visible();
        for (int c = lane; c < n2; c += kWave) at(j, c) = at(j, c) / pv;
        for (int r = lane; r < n; r += kWave) lds[w.tmp + r] = Lh[r * n + j];
        block_visible();
        for (int idx = lane; idx < nn; idx += kWave) {
            const int r = idx / n2, c = idx - r * n2;
            if (r != j) at(r, c) -= lds[w.tmp + r] * at(j, c);
        }
        block_visible();
    }
    return true;
}

// One-spin residency of the inverses (large-system layout): make spin sp's
// inverse the LDS block, writing the other back to global memory.  load =
// false when the block is about to be overwritten (the refresh).
__device__ void ainv_resident(const DevSys& s, const Walker& w, int sp, int lane, bool load = true)
{
    if (!s.ainv1) return;    // both inverse blocks in LDS
    const int res = (int)lds[w.scal + kScRes];
    if (res == sp) return;
    const int blk = s.ns * s.ns;
    for (int i = lane; i < blk; i += kWave) {
        const double v = lds[w.AinvT + i];
        gst(w.AinvG + (long)res * blk + i, v);
        if (load) lds[w.AinvT + i] = gld(w.AinvG + (long)sp * blk + i);
    }
    block_visible();
    if (lane == 0) lds[w.scal + kScRes] = (double)sp;
    wave_sync();
}

// The walker view whose inverse block of spin sp is the LDS block (offset
// shifted so that AinvT + sp ns^2 lands on it) under one-spin residency.
__device__ __forceinline__ Walker ainv_view(const DevSys& s, const Walker& w, int sp)
{
    Walker v = w;
    if (s.ainv1) v.AinvT = w.AinvT - sp * s.ns * s.ns;
    return v;
}

// FP64 Gauss-Jordan inverse with partial pivoting of the transposed Slater
// matrix of spin sp: AinvT[c][k] = (A^-1)[k][c].  Returns false for an
// exactly singular matrix.  The pivot of column j is the largest |M[r][j]|,
// r >= j, the first such row on ties: one lane per row and a wavefront
// maximum (n <= 64 rows).
__device__ bool refresh_inverse(const DevSys& s, const Walker& w, int sp, int lane)
{
    const int n = nspin(s, sp);
    if (!n) return true;
    const int off = sp ? s.Nup : 0, n2 = 2 * n, nn = n * n2;
    const int M = w.B;                   // [n][2n] scratch
    // (row, column) of the lane's first element of [n][2n] and the stride
    const int r0 = lane / n2, c0 = lane - r0 * n2;
    const int dr = kWave / n2, dc = kWave - dr * n2;
    {
        int r = r0, c = c0;
        for (int idx = lane; idx < nn; idx += kWave) {
            lds[M + idx] = c < n ? lds[w.Arow + (off + c) * s.ns + r] : (c - n == r ? 1.0 : 0.0);
            r += dr; c += dc;
            if (c >= n2) { c -= n2; ++r; }
        }
    }
    wave_sync();
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        const double v = (lane >= j && lane < n) ? fabs(lds[M + lane * n2 + j]) : -1.0;
        const double best = wave_max(v);
        if (!(best > 0.0)) { ok = false; break; }
        const unsigned long long hit = __ballot(v == best);
        const int bi = __ffsll((long long)hit) - 1;
        if (bi != j) {
            for (int c = lane; c < n2; c += kWave) {
                const double t = lds[M + j * n2 + c];
                lds[M + j * n2 + c] = lds[M + bi * n2 + c];
                lds[M + bi * n2 + c] = t;
            }
            wave_sync();
        }
        const double pv = lds[M + j * n2 + j];
        wave_sync();
        for (int c = lane; c < n2; c += kWave) lds[M + j * n2 + c] = lds[M + j * n2 + c] / pv;
        for (int r = lane; r < n; r += kWave) lds[w.tmp + r] = lds[M + r * n2 + j];
        wave_sync();
        int r = r0, c = c0;
        for (int idx = lane; idx < nn; idx += kWave) {
            if (r != j) lds[M + idx] -= lds[w.tmp + r] * lds[M + j * n2 + c];
            r += dr; c += dc;
            if (c >= n2) { c -= n2; ++r; }
        }
        wave_sync();
    }
    if (ok) {
        const int Ai = w.AinvT + sp * s.ns * s.ns;
        for (int idx = lane; idx < n * n; idx += kWave) {
            const int c = idx / n, k = idx - c * n;
            lds[Ai + c * s.ns + k] = lds[M + c * n2 + n + k];
        }
    }
    wave_sync();
    return ok;
}

// Ratios of the moves of spin sp (or of every spin when sp < 0), from the
// orbital rows, the inverse and the Jastrow exponent changes.  With a
// pseudopotential also the determinant ratios D(x')/D(x) of the quadrature
// points and their entries -2 a^2 V_q D(x')/D(x) (determinant locality
// approximation: no Jastrow factor), in the units of the lattice ratios.
template <bool kNl = false>
__device__ void recompute_ratios(const DevSys& s, const Walker& w, int sp, int lane, double a = 0.0)
{
    for (int p = lane; p < s.P; p += kWave) {
        const int j = p / 6, spj = spin_of(s, j);
        if (sp < 0 || spj == sp) {
            const int n = nspin(s, spj), c = col_of(s, j);
            const int ai = w.AinvT + spj * s.ns * s.ns + c * s.ns;
            const double* ph = w.Phi + p * s.ns;
            double rd = 0.0;
            for (int k = 0; k < n; ++k) rd += gld(ph + k) * lds[ai + k];
            lds[w.Rdet + p] = rd;
        }
        lds[w.R + p] = lds[w.Rdet + p] * exp(lds[w.dJ + p]);
    }
    if constexpr (kNl) {
        const double m2a2 = -2.0 * a * a;
        for (int p = s.P + lane; p < s.PT; p += kWave) {
            const int j = (p - s.P) / 6, spj = spin_of(s, j);
            if (sp < 0 || spj == sp) {
                const int n = nspin(s, spj), c = col_of(s, j);
                const int ai = w.AinvT + spj * s.ns * s.ns + c * s.ns;
                const double* ph = w.Phi + p * s.ns;
                double rd = 0.0;
                if (lds[w.nlin + j] != 0.0)
                    for (int k = 0; k < n; ++k) rd += gld(ph + k) * lds[ai + k];
                lds[w.Rdet + p] = rd;
            }
            lds[w.R + p] = m2a2 * lds[w.Vnl + p - s.P] * lds[w.Rdet + p];
        }
    }
    wave_sync();
}

// Determinant gradient and Laplacian of the electrons of spin sp (every spin
// when sp < 0): gd[4j + c] = sum_k dPhi_c[j][k] (A^-1)[k][col j], component c
// = x, y, z, Laplacian; one lane per (electron, component).
__device__ void recompute_gd(const DevSys& s, const Walker& w, int sp, int lane)
{
    const int N4 = 4 * s.N;
    const int it0 = sp == 1 ? 4 * s.Nup : 0, it1 = sp == 0 ? 4 * s.Nup : N4;
    for (int it = it0 + lane; it < it1; it += kWave) {
        const int j = it >> 2, spj = spin_of(s, j), n = nspin(s, spj), c = col_of(s, j);
        const int ai = w.AinvT + spj * s.ns * s.ns + c * s.ns;
        double val = 0.0;
        for (int k = 0; k < n; ++k) val += gld(w.dPhi + it * s.ns + k) * lds[ai + k];
        lds[w.gd + it] = val;
    }
    wave_sync();
}

// Jastrow caches of every electron from scratch, without cross-lane sums:
// one lane per (electron, point) pair accumulates over all partners, then one
// lane per electron accumulates its gradient, Laplacian and potentials.
// Returns V_ee.
template <bool kRot>
__device__ double jastrow_all(const DevSys& s, const Walker& w, double a, int lane)
{
    const int K = s.N + s.M;
    const int Kj = s.has_en ? K : s.N;
    const double ia = 1.0 / a;
    const int S = w.B;                            // [N][7] point sums
    for (int it = lane; it < 7 * s.N; it += kWave) {
        const int j = it / 7, q = it - 7 * j;
        const double rj[3] = {lds[w.pos + 3 * j], lds[w.pos + 3 * j + 1], lds[w.pos + 3 * j + 2]};
        double pq[3];
        lattice_point<kRot>(rj, q, a, lds + w.ev, pq);
        double acc = 0.0;
        #pragma unroll 1
        for (int k = 0; k < Kj; ++k) {
            if (k == j) continue;
            double pk[3];
            int jr;
            partner(s, w, j, k, pk, jr);
            const double e0 = pq[0] - pk[0], e1 = pq[1] - pk[1], e2 = pq[2] - pk[2];
            acc += pade_u2(lds + w.jas + 3 * jr, e0 * e0 + e1 * e1 + e2 * e2);
        }
        lds[S + it] = acc;
    }
    double vee = 0.0;
    for (int j = lane; j < s.N; j += kWave) {
        const double rj[3] = {lds[w.pos + 3 * j], lds[w.pos + 3 * j + 1], lds[w.pos + 3 * j + 2]};
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0, nu = 0.0, nua = 0.0;
        #pragma unroll 1
        for (int k = 0; k < K; ++k) {
            if (k == j) continue;
            const bool isel = k < s.N;
            double pk[3];
            int jr;
            partner(s, w, j, k, pk, jr);
            const double d0 = rj[0] - pk[0], d1 = rj[1] - pk[1], d2 = rj[2] - pk[2];
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double ir = rsqrt_nr(r2);
            if (isel || s.has_en) {
                double u, dur, lp;
                pade_derivs2(lds + w.jas + 3 * jr, r2, ir, u, dur, lp);
                g0 += dur * d0; g1 += dur * d1; g2 += dur * d2;
                l += lp;
                if (isel && k > j) vee += ir;
            }
            if (!isel) nucleus_potential(s, w, k, r2, ir, ia, nu, nua);
        }
        lds[w.Jg + 3 * j] = g0; lds[w.Jg + 3 * j + 1] = g1; lds[w.Jg + 3 * j + 2] = g2;
        lds[w.Jl + j] = l; lds[w.nue + j] = nu; lds[w.nua + j] = nua;
    }
    vee = wave_sum(vee);
    wave_sync();
    for (int p = lane; p < s.P; p += kWave) {
        const int j = p / 6, q = p - 6 * j;
        lds[w.dJ + p] = lds[S + 7 * j + q + 1] - lds[S + 7 * j];
    }
    wave_sync();
    return vee;
}

// FP64 refresh: inverses and log-determinants from the exact orbital rows,
// Jastrow caches and V_ee from scratch, all ratios.
template <bool kRot, bool kNl = false, bool kBig = false>
__device__ bool refresh_all(const DevSys& s, const Walker& w, double a, int lane)
{
    bool ok;
    if constexpr (kBig) {
        // with one-spin residency each spin's block is made resident first
        // (not loaded: the elimination overwrites it); spin 1 ends resident
        if (s.ainv1) ainv_resident(s, w, 0, lane, false);
        ok = refresh_inverse_split(s, w, 0, lane);
        if (s.ainv1) ainv_resident(s, w, 1, lane, false);
        ok = refresh_inverse_split(s, w, 1, lane) && ok;
    } else {
        ok = refresh_inverse(s, w, 0, lane);
        ok = refresh_inverse(s, w, 1, lane) && ok;
    }
    const double vee = jastrow_all<kRot>(s, w, a, lane);
    if (lane == 0) lds[w.scal + kScVee] = vee;
    wave_sync();
    if constexpr (kBig) {
        if (s.ainv1) {
            for (int sp = 1; sp >= 0; --sp) {
                ainv_resident(s, w, sp, lane);
                const Walker v = ainv_view(s, w, sp);
                recompute_ratios<kNl>(s, v, sp, lane, a);
                recompute_gd(s, v, sp, lane);
            }
            return ok;
        }
    }
    recompute_ratios<kNl>(s, w, -1, lane, a);
    recompute_gd(s, w, -1, lane);
    return ok;
}

// Lattice-regularized diagonal and local energy at the current configuration
// (App. D; Sec. II.C e_L = W - bbar).
// inc: the lane's inclusive prefix of the positive-ratio sums of the lane
// chunks (lane l owns moves [l per, (l + 1) per)), reused by the heat bath
struct Local { double bbar, W, eL, inc; };

// With a pseudopotential the entries of the quadrature points join the sums:
// positive ones are move rates (bbar), negative ones spin-flip terms (V_sf);
// a quadrature point crosses the node when its determinant ratio is negative.
template <bool kNl = false>
__device__ Local evaluate(const DevSys& s, const Walker& w, double a, int nu_mode, int lane)
{
    const double inv2a2 = 1.0 / (2.0 * a * a), ia2 = 2.0 * inv2a2;
    double loc = 0.0, vs = 0.0;
    int anyneg = 0;
    const int PT = n_prop<kNl>(s);
    const int per = (PT + kWave - 1) / kWave;
    const int p0 = lane * per, p1 = min(p0 + per, PT);
    for (int p = p0; p < p1; ++p) {
        const double r = lds[w.R + p];
        if constexpr (kNl) {
            if (r > 0) loc += r;
            else if (r < 0) vs += -r;
            if (p < s.P ? r < 0 : lds[w.Rdet + p] < 0) anyneg = 1;
        } else {
            if (r > 0) loc += r;
            else if (r < 0) { vs += -r; anyneg = 1; }
        }
    }
    const double inc = wave_incl_scan(loc, lane);
    const double bs = lane63(inc);
    vs = wave_sum(vs);
    const bool anynode = __ballot(anyneg) != 0;
    double sum_opt = 0.0;
    for (int j = lane; j < s.N; j += kWave) {
        const double g0 = lds[w.gd + 4 * j], g1 = lds[w.gd + 4 * j + 1];
        const double g2 = lds[w.gd + 4 * j + 2], ld = lds[w.gd + 4 * j + 3];
        const double j0 = lds[w.Jg + 3 * j], j1 = lds[w.Jg + 3 * j + 1], j2 = lds[w.Jg + 3 * j + 2];
        const double lap = ld + 2.0 * (g0 * j0 + g1 * j1 + g2 * j2) + lds[w.Jl + j] +
                           j0 * j0 + j1 * j1 + j2 * j2;
        double lapA = 0.0;
        int nd = 0;
        for (int q = 0; q < 6; ++q) {
            const double r = lds[w.R + 6 * j + q];
            lapA += r - 1.0;
            if (r < 0) nd = 1;
        }
        if constexpr (kNl)
            for (int q = 0; q < 6; ++q)
                if (lds[w.Rdet + s.P + 6 * j + q] < 0) nd = 1;
        lapA *= ia2;
        if (nu_mode == 1) nd = anynode;
        if (nu_mode == 2) nd = 1;
        const double nuzv = lds[w.nue + j] + 0.5 * (lapA - lap);
        const double nua = lds[w.nua + j];
        const double numax = nuzv > nua ? nuzv : nua;
        sum_opt += nd ? numax : nuzv;
    }
    sum_opt = wave_sum(sum_opt);
    Local L;
    L.bbar = bs * inv2a2;
    const double vsf = vs * inv2a2;
    L.W = 3.0 * s.N / (a * a) + sum_opt + lds[w.scal + kScVee] + vsf + s.vii;
    L.eL = L.W - L.bbar;
    L.inc = inc;
    return L;
}

// Heat-bath choice: first p with cumulative positive ratio > xi * total, from
// the chunk prefix sums of the evaluation at the same configuration.
template <bool kNl = false>
__device__ int heat_bath(const DevSys& s, const Walker& w, double xi, double inc, int lane)
{
    const int PT = n_prop<kNl>(s);
    const int per = (PT + kWave - 1) / kWave;
    const int p0 = lane * per, p1 = min(p0 + per, PT);
    const double tot = lane63(inc);
    if (!(tot > 0)) return -1;
    const double t = xi * tot;
    double c = dpp_mov<0x138, 0xf>(inc);   // wave_shr:1, lane 0 receives 0
    int found = -1, lastpos = -1;
    for (int p = p0; p < p1; ++p) {
        const double r = lds[w.R + p];
        if (r > 0) {
            c += r;
            lastpos = p;
            if (found < 0 && c > t) found = p;
        }
    }
    const unsigned long long m = __ballot(found >= 0);
    if (m) return __builtin_amdgcn_readlane(found, __ffsll((long long)m) - 1);
    const unsigned long long mp = __ballot(lastpos >= 0);
    return __builtin_amdgcn_readlane(lastpos, 63 - __clzll((long long)mp));
}

// Apply move p: position, Sherman-Morrison inverse update of the moved spin,
// new orbital rows of the moved electron, Jastrow / potential caches, ratios.
// Returns true when the determinant ratio was tiny (a refresh is forced).
// A move p >= 6N (with a pseudopotential) takes electron (p - 6N) / 6 to
// quadrature point (p - 6N) % 6 of the atom whose sphere holds it.
#ifdef LRDMC_SECTION_TIMERS
template <bool kRot, bool kNl = false, bool kBig = false>
__device__ bool apply_move(const DevSys& s, const Walker& w, double a, int p, int lane,
                           unsigned long long* sect, unsigned long long& t_mark_)
#else
template <bool kRot, bool kNl = false, bool kBig = false>
__device__ bool apply_move(const DevSys& s, const Walker& w, double a, int p, int lane)
#endif
{
    const bool nlm = kNl && p >= s.P;
    const int pk = nlm ? p - s.P : p;
    const int i = pk / 6, d = (pk / 2) % 3, sg = pk % 2;
    const int sp = spin_of(s, i), c = col_of(s, i), n = nspin(s, sp);
    const double Rd = lds[w.Rdet + p], iRd = 1.0 / Rd;
    const double rold[3] = {lds[w.pos + 3 * i], lds[w.pos + 3 * i + 1], lds[w.pos + 3 * i + 2]};
    const double* st = lds + w.ev;
    double rnew[3] = {rold[0], rold[1], rold[2]};
    if (nlm) {
        double rr;
        const int I = nl_sphere(s, w, rold, rr);
        nl_point(lds + w.nuc + kNucLen * (I < 0 ? 0 : I), rr, lds + w.ev + 9, pk % 6, rnew);
    } else if constexpr (kRot) {
        point_qv(rold, 2 * d + sg + 1, st, rnew);
    } else {
        rnew[d] = rnew[d] + (sg ? -a : a);
    }

    // The accepted orbital row u is fetched first and the basis values at
    // the new position are computed while it is in flight (in the
    // large-system layout they follow the Sherman-Morrison update, chunk by
    // chunk with the orbital rows).
    double u0 = 0.0;
    if (lane < n) u0 = gld(w.Phi + p * s.ns + lane);
    if constexpr (!kBig) basis_rows<kRot>(s, w, rnew, a, lane);
    LRDMC_T(3);

    // Sherman-Morrison on AinvT of spin sp with the accepted orbital row u
    if constexpr (kBig) ainv_resident(s, w, sp, lane);
    const int Ai = w.AinvT + ((kBig && s.ainv1) ? 0 : sp * s.ns * s.ns);
    const int u = w.tmp, rowc = w.tmp + s.ns, beta = w.tmp + 2 * s.ns;
    for (int k = lane; k < n; k += kWave) {
        lds[u + k] = k < kWave ? u0 : gld(w.Phi + p * s.ns + k);
        lds[rowc + k] = lds[Ai + c * s.ns + k];
    }
    wave_sync();
    if (n <= 8) {
        // lane (cc, k) = (lane >> 3, lane & 7): one product, a sum over the 8 lanes
        const int cc = lane >> 3, k = lane & 7;
        double v = (cc < n && k < n) ? lds[u + k] * lds[Ai + cc * s.ns + k] : 0.0;
        v += dpp_mov<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
        v += dpp_mov<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
        v += dpp_mov<0x114, 0xf>(v);   // row_shr:4: lane 8cc + 7 holds the group sum
        if (k == 7 && cc < n) lds[beta + cc] = v;
    } else {
        for (int cc = lane; cc < n; cc += kWave) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += lds[u + k] * lds[Ai + cc * s.ns + k];
            lds[beta + cc] = acc;
        }
    }
    wave_sync();
    for (int idx = lane; idx < n * n; idx += kWave) {
        const int cc = idx / n, k = idx - cc * n;
        if (cc == c) lds[Ai + cc * s.ns + k] = lds[rowc + k] * iRd;
        else lds[Ai + cc * s.ns + k] -= lds[rowc + k] * (lds[beta + cc] * iRd);
    }
    for (int k = lane; k < n; k += kWave) {
        if constexpr (kBig) gst(w.ArowG + i * s.ns + k, lds[u + k]);
        else lds[w.Arow + i * s.ns + k] = lds[u + k];
    }
    wave_sync();

    LRDMC_T(2);
    // new orbital rows of electron i at rnew
    if constexpr (kBig) electron_rows<kRot, false, true>(s, w, i, rnew, a, lane);
    else orbital_rows<false, kNl>(s, w, i, lane);
    store_rows<kNl, kBig>(s, w, i, lane, false);
    if constexpr (kNl) nl_rows(s, w, i, rnew, lane);
    LRDMC_T(4);

    // Orbital rows of the moves of spin sp and orbital derivatives of its
    // electrons (first kPre values of the first pass) are fetched now; the
    // Jastrow updates run while they are in flight.
    const int off = sp ? s.Nup : 0;
    double pre_r[kPre], pre_g[kPre];
    const bool rv = lane < 6 * n, gv = lane < 4 * n;
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        pre_r[k] = (rv && k < n) ? gld(w.Phi + (6 * off + lane) * s.ns + k) : 0.0;
        pre_g[k] = (gv && k < n) ? gld(w.dPhi + (4 * off + lane) * s.ns + k) : 0.0;
    }

    // Jastrow and potential caches: pairs (i, k) change from rold to rnew.
    // The 7 points of the moved electron (its new position and neighbours):
    // with at most 32 partners, each point takes one or two rows of 16 lanes,
    // so 4 or 2 points share a pass and a row reduction; otherwise one point
    // per pass with a wave reduction.
    const double ia = 1.0 / a;
    const int K = s.N + s.M;
    const int Kj = s.has_en ? K : s.N;
    const int dJi = w.tmp + 3 * s.ns;            // 6 new exponent changes of electron i
    const int Sq = w.tmp + 3 * s.ns + 8;         // 7 point sums
    const int rpp = (Kj + 15) >> 4;              // rows of 16 lanes per point
    if (rpp <= 2) {
        // lane = (point group, partner): the two passes of points q and
        // q + ppp are evaluated together, then reduced over the row(s)
        const int ppp = 4 / rpp, row = lane >> 4;
        const int k = (row % rpp) * 16 + (lane & 15);
        double pk[3] = {0.0, 0.0, 0.0};
        int jr = 0;
        const bool kval = k < Kj && k != i;
        if (kval) partner(s, w, i, k, pk, jr);
        const double* prm = lds + w.jas + 3 * jr;
        // displaced coordinates of each point, formed as in the move itself
        const double rp[3] = {rnew[0] + a, rnew[1] + a, rnew[2] + a};
        const double rm[3] = {rnew[0] + (-a), rnew[1] + (-a), rnew[2] + (-a)};
        for (int q0 = 0; q0 < 7; q0 += 2 * ppp) {
            const int qa = q0 + row / rpp, qb = qa + ppp;
            double va, vb;
            double pa[3], pb[3];
            if constexpr (kRot) {
                point_qv(rnew, qa, st, pa);
                point_qv(rnew, qb < 7 ? qb : 0, st, pb);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pa[c] = qa == 2 * c + 1 ? rp[c] : rnew[c];
                    pa[c] = qa == 2 * c + 2 ? rm[c] : pa[c];
                    pb[c] = qb == 2 * c + 1 ? rp[c] : rnew[c];
                    pb[c] = qb == 2 * c + 2 ? rm[c] : pb[c];
                }
            }
            const double a0 = pa[0] - pk[0], a1 = pa[1] - pk[1], a2 = pa[2] - pk[2];
            const double b0 = pb[0] - pk[0], b1 = pb[1] - pk[1], b2 = pb[2] - pk[2];
            const double ua = pade_u2(prm, a0 * a0 + a1 * a1 + a2 * a2);
            const double ub = pade_u2(prm, b0 * b0 + b1 * b1 + b2 * b2);
            va = kval ? ua : 0.0;
            vb = (kval && qb < 7) ? ub : 0.0;
            if (rpp == 1) { va = row16_sum(va); vb = row16_sum(vb); }
            else { va = row32_sum(va); vb = row32_sum(vb); }
            if ((lane & (16 * rpp - 1)) == 16 * rpp - 1) {
                lds[Sq + qa] = va;
                if (qb < 7) lds[Sq + qb] = vb;
            }
        }
        wave_sync();
    } else {
#pragma unroll 1
        for (int q = 0; q < 7; ++q) {
            double pq[3];
            lattice_point<kRot>(rnew, q, a, st, pq);
            double acc = 0.0;
            #pragma unroll 1
            for (int k = lane; k < Kj; k += kWave) {
                if (k == i) continue;
                double pk[3];
                int jr;
                partner(s, w, i, k, pk, jr);
                const double e0 = pq[0] - pk[0], e1 = pq[1] - pk[1], e2 = pq[2] - pk[2];
                acc += pade_u2(lds + w.jas + 3 * jr, e0 * e0 + e1 * e1 + e2 * e2);
            }
            acc = wave_sum(acc);
            if (lane == 0) lds[Sq + q] = acc;
        }
        wave_sync();
    }
    if (lane < 6) lds[dJi + lane] = lds[Sq + lane + 1] - lds[Sq];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0, dvee = 0.0, nu = 0.0, nua = 0.0;
    #pragma unroll 1
    for (int k = lane; k < K; k += kWave) {
        if (k == i) continue;
        const bool isel = k < s.N;
        double pk[3];
        int jr;
        partner(s, w, i, k, pk, jr);
        const double n0 = rnew[0] - pk[0], n1 = rnew[1] - pk[1], n2 = rnew[2] - pk[2];
        const double rn2 = n0 * n0 + n1 * n1 + n2 * n2;
        const double irn = rsqrt_nr(rn2);
        if (isel || s.has_en) {
            double un, dnr, lpn;
            pade_derivs2(lds + w.jas + 3 * jr, rn2, irn, un, dnr, lpn);
            g0 += dnr * n0; g1 += dnr * n1; g2 += dnr * n2;
            l += lpn;
            if (isel) {
                const double o0 = rold[0] - pk[0], o1 = rold[1] - pk[1], o2 = rold[2] - pk[2];
                const double ro2 = o0 * o0 + o1 * o1 + o2 * o2, iro = rsqrt_nr(ro2);
                double uo, dor, lpo;
                pade_derivs2(lds + w.jas + 3 * jr, ro2, iro, uo, dor, lpo);
                lds[w.dje + k] = un - uo;
                // electron k sees the pair through r_k - r_i = -(r_i - r_k)
                lds[w.Jg + 3 * k] += -(dnr * n0) + dor * o0;
                lds[w.Jg + 3 * k + 1] += -(dnr * n1) + dor * o1;
                lds[w.Jg + 3 * k + 2] += -(dnr * n2) + dor * o2;
                lds[w.Jl + k] += lpn - lpo;
                dvee += irn - iro;
            }
        }
        if (!isel) nucleus_potential(s, w, k, rn2, irn, ia, nu, nua);
    }
    g0 = wave_sum(g0); g1 = wave_sum(g1); g2 = wave_sum(g2);
    l = wave_sum(l); dvee = wave_sum(dvee); nu = wave_sum(nu); nua = wave_sum(nua);
    wave_sync();
    LRDMC_T(4);
    // Jastrow exponent changes of the other electrons' moves: moves q and
    // q + 64 of a lane are evaluated together
    for (int qa = lane; qa < s.P; qa += 2 * kWave) {
        const int qb = qa + kWave < s.P ? qa + kWave : qa;
        const int ja = qa / 6, jb = qb / 6;
        double dv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = h ? qb : qa, j = h ? jb : ja;
            const double* prm = lds + w.jas + 3 * ee_row(s, i, j);
            double r2[3] = {lds[w.pos + 3 * j], lds[w.pos + 3 * j + 1], lds[w.pos + 3 * j + 2]};
            if constexpr (kRot) {
                const double rj[3] = {r2[0], r2[1], r2[2]};
                point_qv(rj, q - 6 * j + 1, st, r2);
            } else {
                const int dd = (q >> 1) % 3, s2 = q & 1;
                r2[dd] = r2[dd] + (s2 ? -a : a);
            }
            const double n0 = r2[0] - rnew[0], n1 = r2[1] - rnew[1], n2 = r2[2] - rnew[2];
            const double o0 = r2[0] - rold[0], o1 = r2[1] - rold[1], o2 = r2[2] - rold[2];
            const double un = pade_u2(prm, n0 * n0 + n1 * n1 + n2 * n2);
            const double uo = pade_u2(prm, o0 * o0 + o1 * o1 + o2 * o2);
            dv[h] = (un - uo) - lds[w.dje + j];
        }
        if (ja != i) lds[w.dJ + qa] += dv[0];
        if (qb != qa && jb != i) lds[w.dJ + qb] += dv[1];
    }
    if (lane == 0) {
        for (int q = 0; q < 6; ++q) lds[w.dJ + 6 * i + q] = lds[dJi + q];
        lds[w.Jg + 3 * i] = g0; lds[w.Jg + 3 * i + 1] = g1; lds[w.Jg + 3 * i + 2] = g2;
        lds[w.Jl + i] = l; lds[w.nue + i] = nu; lds[w.nua + i] = nua;
        lds[w.scal + kScVee] += dvee;
        if (kRot || nlm) {
            lds[w.pos + 3 * i] = rnew[0]; lds[w.pos + 3 * i + 1] = rnew[1]; lds[w.pos + 3 * i + 2] = rnew[2];
        } else {
            lds[w.pos + 3 * i + d] = rnew[d];
        }
    }
    wave_sync();
    LRDMC_T(5);
    // ratios of the moves of spin sp, derivatives of its electrons
    for (int pp = lane; pp < 6 * n; pp += kWave) {
        const int q = 6 * off + pp, cj = col_of(s, q / 6);
        const int ai = Ai + cj * s.ns;
        double rd = 0.0;
        if (pp < kWave) {
#pragma unroll
            for (int k = 0; k < kPre; ++k)
                if (k < n) rd += pre_r[k] * lds[ai + k];
            for (int k = kPre; k < n; ++k) rd += gld(w.Phi + q * s.ns + k) * lds[ai + k];
        } else {
            for (int k = 0; k < n; ++k) rd += gld(w.Phi + q * s.ns + k) * lds[ai + k];
        }
        lds[w.Rdet + q] = rd;
    }
    if constexpr (kNl) {
        // determinant ratios and entries of spin sp's quadrature points
        const double m2a2 = -2.0 * a * a;
        for (int pp = lane; pp < 6 * n; pp += kWave) {
            const int q = s.P + 6 * off + pp, cj = col_of(s, off + pp / 6);
            const int ai = Ai + cj * s.ns;
            double rd = 0.0;
            if (lds[w.nlin + off + pp / 6] != 0.0)
                for (int k = 0; k < n; ++k) rd += gld(w.Phi + q * s.ns + k) * lds[ai + k];
            lds[w.Rdet + q] = rd;
            lds[w.R + q] = m2a2 * lds[w.Vnl + q - s.P] * rd;
        }
    }
    for (int gg = lane; gg < 4 * n; gg += kWave) {
        const int it = 4 * off + gg, cj = col_of(s, it >> 2);
        const int ai = Ai + cj * s.ns;
        double val = 0.0;
        if (gg < kWave) {
#pragma unroll
            for (int k = 0; k < kPre; ++k)
                if (k < n) val += pre_g[k] * lds[ai + k];
            for (int k = kPre; k < n; ++k) val += gld(w.dPhi + it * s.ns + k) * lds[ai + k];
        } else {
            for (int k = 0; k < n; ++k) val += gld(w.dPhi + it * s.ns + k) * lds[ai + k];
        }
        lds[w.gd + it] = val;
    }
    wave_sync();
    for (int qa = lane; qa < s.P; qa += 2 * kWave) {
        const int qb = qa + kWave;
        const double xa = lds[w.dJ + qa], xb = qb < s.P ? lds[w.dJ + qb] : 0.0;
        const double ea = exp(xa), eb = exp(xb);
        lds[w.R + qa] = lds[w.Rdet + qa] * ea;
        if (qb < s.P) lds[w.R + qb] = lds[w.Rdet + qb] * eb;
    }
    wave_sync();
    LRDMC_T(6);
    return fabs(Rd) < 1e-6;
}

// ---------------------------------------------------------------------------
// the phase kernel: one workgroup = one wavefront = one walker
// ---------------------------------------------------------------------------
// Occupancy target of the phase kernel (waves per SIMD); the compiler caps
// the register budget accordingly.
#ifndef LRDMC_PHASE_WAVES
#define LRDMC_PHASE_WAVES 2
#endif

// The phase kernel, one instantiation per lattice geometry -- fixed axes
// (kRot = false, the cheaper axis-aligned moves) or a random orientation per
// walker and phase (kRot = true) -- and per Hamiltonian: local potentials
// only, or with the non-local pseudopotential (kNl = true: 6N more proposals).
// kBig: the large-system layout for walkers whose coefficient block and
// Slater rows do not fit the LDS with the rest of their state (both read from
// global memory, the refresh's augmented matrix split over the basis block and
// the inverse block); local potentials only.
template <bool kRot, bool kNl, bool kBig>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(LRDMC_PHASE_WAVES)))
void phase_fp64(const DevSys* __restrict__ sys, PhaseArgs pa)
{
    const DevSys& s = *sys;
    const int wid = blockIdx.x;
    if (wid >= s.nw) return;
    const int lane = threadIdx.x;
    const Walker w = walker_view(s);
    const int jb = *s.jp;
    const double E0 = *s.e0p;

    for (int q = lane; q < 3 * s.N; q += kWave) lds[w.pos + q] = s.pos[(long)wid * 3 * s.N + q];
    // the coefficient block in LDS (the pseudopotential and large-system
    // kernels read it from global memory: their LDS blocks are larger)
    if constexpr (!kNl && !kBig)
        for (int q = lane; q < s.Nb * s.ns; q += kWave) {
            const int mu = q / s.ns, k = q - mu * s.ns;
            lds[w.C + q] = gld(s.C + mu * s.Norb + k);
        }
    const double a = pa.a;
    // nucleus records and Pade parameter rows
    for (int I = lane; I < s.M; I += kWave) {
        double* nr = lds + w.nuc + kNucLen * I;
        nr[0] = gld(s.R + 3 * I); nr[1] = gld(s.R + 3 * I + 1); nr[2] = gld(s.R + 3 * I + 2);
        nr[3] = gld(s.Z + I);
        nr[4] = gld(s.rc + I);
        nr[5] = gld(s.core + I) == 0 ? 0.0 : 1.0;
        nr[6] = (double)(2 + gld(s.spec + I));
    }
    for (int q = lane; q < 3 * (2 + s.nspec); q += kWave) lds[w.jas + q] = gld(s.jas + q);
    // lattice step vectors of this walker for this phase: the coordinate axes,
    // or a random orientation drawn from its own Philox stream
    if (lane == 0) {
        double st[9], uv[9];
        if constexpr (kRot)
            lattice_steps(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb, pa.a, st, kNl ? uv : nullptr);
        else lattice_steps_fixed(pa.a, st, kNl ? uv : nullptr);
        for (int q = 0; q < 9; ++q) lds[w.ev + q] = st[q];
        if constexpr (kBig) lds[w.scal + kScRes] = 0.0;   // spin 0's inverse block resident
        if constexpr (kNl)
            for (int q = 0; q < 9; ++q) lds[w.ev + 9 + q] = uv[q];
    }
    wave_sync();
    // orbital rows of every electron, then the FP64 refresh
    for (int j = 0; j < s.N; ++j) {
        const double r[3] = {lds[w.pos + 3 * j], lds[w.pos + 3 * j + 1], lds[w.pos + 3 * j + 2]};
        electron_rows<kRot, kNl, kBig>(s, w, j, r, a, lane);
        store_rows<kNl, kBig>(s, w, j, lane, true);
        if constexpr (kNl) nl_rows(s, w, j, r, lane);
    }
    unsigned long long n_neg = 0, n_nomove = 0, n_refresh = 1, n_small = 0, n_sing = 0,
                       n_capped = 0;
    if (!refresh_all<kRot, kNl, kBig>(s, w, a, lane)) n_sing++;

    double lw = s.lw[wid];
    // load-balanced weight factors bbar / (W - E_0) multiplied in blocks
    // (lw_block_update): one logarithm per 32 steps instead of one per step
    double wprod = 1.0;
    double tau_left = pa.tau;
    int it = 0, since = 0;
    Local L;
    int32_t* tr = s.trace ? s.trace + (long)wid * s.trace_cap : nullptr;
#ifdef LRDMC_SECTION_TIMERS
    unsigned long long sect[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#endif
    // uniforms of 64 consecutive iterations, lane l holding iteration m0 + l
    // (the draws are counter-based, so drawing ahead changes nothing)
    double xmove = 0.0, xpers = 0.0;
    LRDMC_T0();
    for (;;) {
        if (pa.scheme == 0 && it >= pa.nproj) break;
        if ((it & (kWave - 1)) == 0) {
            xmove = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb,
                                   (uint64_t)(it + lane), kMove);
            if (pa.scheme == 1)
                xpers = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)jb,
                                       (uint64_t)(it + lane), kPersist);
        }
        const int slot = it & (kWave - 1);
        L = evaluate<kNl>(s, w, a, pa.nu_mode, lane);
        LRDMC_T(0);
        int q;
        if (pa.scheme == 0) {
            const double den = L.W - E0;
            if (!(den > 0)) { lw = -INFINITY; n_neg++; }
            else if (!(L.bbar > 0)) { lw = -INFINITY; n_nomove++; }
            else {
                lw_block_update(lw, wprod, L.bbar, den, it + 1);
            }
            q = heat_bath<kNl>(s, w, lane_value(xmove, slot), L.inc, lane);
            if (tr && it < s.trace_cap && lane == 0) tr[it] = q;
            ++it;
        } else {
            const double xt = lane_value(xpers, slot);
            const double t = (L.bbar > 0) ? -log1p(-xt) / L.bbar : INFINITY;
            if (!(L.bbar > 0)) n_nomove++;
            // the iteration cap only guarantees termination; it is never
            // reached by a walker whose rate bbar stays finite
            const bool capped = it + 1 >= pa.conv_cap;
            if (capped && t < tau_left) n_capped++;
            const bool stop = !(t < tau_left) || capped;
            const double tx = stop ? tau_left : t;
            lw -= tx * L.eL;
            tau_left = stop ? 0.0 : tau_left - tx;
            ++it;
            if (stop) {
                if (tr && it - 1 < s.trace_cap && lane == 0) tr[it - 1] = -1;
                break;
            }
            q = heat_bath<kNl>(s, w, lane_value(xmove, slot), L.inc, lane);
            if (tr && it - 1 < s.trace_cap && lane == 0) tr[it - 1] = q;
        }
        LRDMC_T(1);
        if (q >= 0) {
#ifdef LRDMC_SECTION_TIMERS
            const bool small = apply_move<kRot, kNl, kBig>(s, w, a, q, lane, sect, t_mark_);
#else
            const bool small = apply_move<kRot, kNl, kBig>(s, w, a, q, lane);
#endif
            ++since;
            if (small) n_small++;
            if (small || since >= pa.refresh_every) {
                if (!refresh_all<kRot, kNl, kBig>(s, w, a, lane)) n_sing++;
                n_refresh++;
                since = 0;
            }
            LRDMC_T(7);
        }
    }
#ifdef LRDMC_SECTION_TIMERS
    if (lane == 0 && pa.timers)
        for (int k = 0; k < 8; ++k) pa.timers[(long)wid * 8 + k] = sect[k];
#endif
    lw += log(wprod);
    if (pa.scheme == 0) {
        L = evaluate<kNl>(s, w, a, pa.nu_mode, lane);
        // the estimator weight w / (W - E_0) at the final configuration needs
        // W - E_0 > 0 as every step's factor does: otherwise the walker dies
        if (pa.nproj > 0 && !(L.W - E0 > 0)) { lw = -INFINITY; n_neg++; }
    }
    const bool nonfinite = !(isfinite(L.eL) && isfinite(L.W)) || isnan(lw) || lw == INFINITY;

    for (int q = lane; q < 3 * s.N; q += kWave) s.pos[(long)wid * 3 * s.N + q] = lds[w.pos + q];
    if (lane == 0) {
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

template __global__ void phase_fp64<false, false, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
template __global__ void phase_fp64<true, false, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
template __global__ void phase_fp64<false, true, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
template __global__ void phase_fp64<true, true, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
template __global__ void phase_fp64<false, false, true>(const DevSys* __restrict__ sys, PhaseArgs pa);
template __global__ void phase_fp64<true, false, true>(const DevSys* __restrict__ sys, PhaseArgs pa);

// ---------------------------------------------------------------------------
// reconfiguration (Sec. II.A): one workgroup computes max log-weight, the
// FP64 inclusive prefix of exp(lw - max) in slot order, and the weighted
// local-energy sums; then one thread per new walker runs the comb search
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBranchBlock) void branch_scan(BranchView s, int scheme,
                                                               double* cum, double* out,
                                                               int* n_distinct)
{
    __shared__ double sh[kMaxBranchBlock];
    __shared__ int shi[kMaxBranchBlock];
    const int t = threadIdx.x, nt = blockDim.x, nw = s.nw;
    const double E0 = *s.e0p;
    if (t == 0) *n_distinct = 0;
    const int per = (nw + nt - 1) / nt, b0 = t * per, b1 = min(b0 + per, nw);
    double mx = -INFINITY;
    int last = -1;
    for (int b = b0; b < b1; ++b) {
        const double v = s.lw[b];
        if (v > mx || isnan(v)) mx = isnan(mx) ? mx : v;   // a NaN log-weight propagates
        if (v > -INFINITY) last = b;
    }
    sh[t] = mx; shi[t] = last;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
        if (t < o) {
            const double x = sh[t], y = sh[t + o];
            sh[t] = (isnan(x) || isnan(y)) ? NAN : fmax(x, y);
            shi[t] = max(shi[t], shi[t + o]);
        }
        __syncthreads();
    }
    mx = sh[0];
    last = shi[0];
    __syncthreads();
    double loc = 0.0, se = 0.0, so = 0.0;
    for (int b = b0; b < b1; ++b) {
        const double wv = exp(s.lw[b] - mx);
        loc += wv;
        cum[b] = loc;
        if (wv > 0.0) {   // dead walkers (weight zero) carry no W - E_0 factor
            const double om = scheme == 0 ? wv / (s.Wd[b] - E0) : wv;
            se += om * s.eL[b];
            so += om;
        }
    }
    // exclusive scan of the per-thread totals (Hillis-Steele, fixed order)
    sh[t] = loc;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        const double v = (t >= o) ? sh[t - o] : 0.0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    const double excl = sh[t] - loc;
    const double tot = sh[nt - 1];
    for (int b = b0; b < b1; ++b) cum[b] += excl;
    __syncthreads();
    sh[t] = se;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    se = sh[0];
    __syncthreads();
    sh[t] = so;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    so = sh[0];
    if (t == 0) {
        out[0] = mx; out[1] = tot; out[2] = se; out[3] = so; out[4] = (double)last;
    }
}

__global__ void branch_comb(BranchView s, uint64_t seed, const double* cum, const double* out,
                            int32_t* sel)
{
    const int al = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = s.nw;
    if (al >= nw) return;
    const double xi = philox_uniform(seed, s.sysid, 0, (uint64_t)*s.jp, 0, kComb);
    const double tot = out[1];
    const double target = (xi + (double)al) * tot / (double)nw;
    int lo = 0, hi = nw;          // first index with cum > target
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] > target) hi = mid; else lo = mid + 1;
    }
    int pick = lo < nw ? lo : (int)out[4];
    if (pick < 0 || pick >= nw) pick = 0;   // all weights zero: the host reports it
    sel[al] = pick;
}

__global__ void branch_count(const int32_t* sel, int nw, int* n_distinct)
{
    const int al = blockIdx.x * blockDim.x + threadIdx.x;
    if (al >= nw) return;
    if (al == 0 || sel[al] != sel[al - 1]) atomicAdd(n_distinct, 1);
}

__global__ void branch_gather(BranchView s, const int32_t* sel, const double* pos_old,
                              const double* eL_old, const double* W_old)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int per = 3 * s.N;
    if (idx >= (long)s.nw * per) return;
    const int al = (int)(idx / per), q = (int)(idx - (long)al * per);
    const int b = sel[al];
    s.pos[idx] = pos_old[(long)b * per + q];
    if (q == 0) {
        s.lw[al] = 0.0;
        s.eL[al] = eL_old[b];
        s.Wd[al] = W_old[b];
    }
}

// After the gather: the walker-averaged local energy and log wbar of this
// branching appended to the device history ring, and E_0 updated to the mean
// of the last `window` e_bar (Algorithm 2).  A branching in which every
// weight is zero appends nothing and is counted in n_dead[0]; one whose
// largest log-weight, weight sum or walker average is not finite (a NaN or
// +inf log-weight) appends nothing and is counted in n_dead[1].  bump_j
// (non-null for the last system of a handle) advances the branching index.
__global__ void branch_finish(int nw, const double* out, const int* n_distinct, double* hist,
                              long long* n_hist, double* e0p, int* n_dead, int window, int cap,
                              int* bump_j)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double mx = out[0], tot = out[1], se = out[2], so = out[3];
    const bool all_dead = mx == -INFINITY;
    const bool finite = isfinite(mx) && isfinite(tot) && tot > 0.0 && isfinite(se) &&
                        isfinite(so) && so != 0.0 && isfinite(se / so);
    if (all_dead) {
        n_dead[0] += 1;
    } else if (!finite) {
        n_dead[1] += 1;
    } else {
        const long long n = *n_hist;
        double* e = hist + (n % cap) * kHistLen;
        e[kHistLogW] = log(tot / (double)nw) + mx;
        e[kHistEbar] = se / so;
        e[kHistMaxLw] = mx;
        e[kHistDistinct] = (double)*n_distinct;
        const long long n1 = n + 1, k0 = n1 > window ? n1 - window : 0;
        double acc = 0.0;
        for (long long q = k0; q < n1; ++q) acc += hist[(q % cap) * kHistLen + kHistEbar];
        const double e0 = acc / (double)(n1 - k0);
        e[kHistE0] = e0;
        *e0p = e0;
        *n_hist = n1;
    }
    if (bump_j) *bump_j += 1;
}

// counters of a phase to their initial values (a kernel, so that it can sit
// inside a captured graph)
__global__ void reset_counters_kernel(unsigned long long* c)
{
    const int k = threadIdx.x;
    if (k < kCntLen) c[k] = (k == kCntMinIters) ? ~0ull : 0ull;
}

}  // namespace lrdmc
