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

namespace lrdmc {

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

// ---------------------------------------------------------------------------
// wavefront collectives; every lane receives lane 0's value so that all
// lanes hold bit-identical results and control flow stays uniform
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return __shfl(v, 0);
}

__device__ __forceinline__ double wave_incl_scan(double v, int lane)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Pade pair function u(r) = (A r + B r^2)/(1 + b r) with u' and u''.
__device__ __forceinline__ double pade_u(const double* p, double r)
{
    return (p[0] * r + p[1] * r * r) / (1.0 + p[2] * r);
}
__device__ __forceinline__ void pade_all(const double* p, double r, double& u, double& du,
                                         double& d2u)
{
    const double A = p[0], B = p[1], b = p[2], den = 1.0 + b * r;
    u = (A * r + B * r * r) / den;
    du = (A + 2.0 * B * r + B * b * r * r) / (den * den);
    d2u = 2.0 * (B - A * b) / (den * den * den);
}

__device__ __forceinline__ double norm3(double x, double y, double z)
{
    return sqrt(x * x + y * y + z * z);
}

// Value of basis function mu at point r.
__device__ __forceinline__ double basis_value(const DevSys& s, int mu, const double* r)
{
    const double* Ra = s.R + 3 * s.batom[mu];
    const double dx = r[0] - Ra[0], dy = r[1] - Ra[1], dz = r[2] - Ra[2];
    const double d2 = dx * dx + dy * dy + dz * dz, al = s.bexp[mu];
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
    const double* Ra = s.R + 3 * s.batom[mu];
    const double d[3] = {r[0] - Ra[0], r[1] - Ra[1], r[2] - Ra[2]};
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], al = s.bexp[mu];
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

// ---------------------------------------------------------------------------
// per-walker state views
// ---------------------------------------------------------------------------
struct Walker {
    double *pos, *R, *Rdet, *dJ, *Arow, *AinvT, *Jg, *Jl, *nue, *nua, *dje, *scal, *B, *rows,
        *tmp;
    double *Phi, *dPhi;   // global spill
};

__device__ __forceinline__ int spin_of(const DevSys& s, int i) { return i >= s.Nup; }
__device__ __forceinline__ int col_of(const DevSys& s, int i) { return i >= s.Nup ? i - s.Nup : i; }
__device__ __forceinline__ int nspin(const DevSys& s, int sp) { return sp ? s.Ndn : s.Nup; }
__device__ __forceinline__ const double* ee_par(const DevSys& s, int i, int k)
{
    return s.jas + 3 * ((i >= s.Nup) == (k >= s.Nup) ? 0 : 1);
}

// Orbital rows of electron j at position r (11 rows, columns k < n_j):
// row 0 the value at r, rows 1..6 the values at the six lattice neighbours
// r +- a e_d (move order), rows 7..9 the gradient, row 10 the Laplacian.
__device__ void electron_rows(const DevSys& s, const Walker& w, int j, const double* r,
                              double a, int lane)
{
    for (int mu = lane; mu < s.Nb; mu += kWave) {
        double v, g[3], l;
        basis_vgl(s, mu, r, v, g, l);
        w.B[0 * s.Nb + mu] = v;
        for (int d = 0; d < 3; ++d)
            for (int sg = 0; sg < 2; ++sg) {
                double q[3] = {r[0], r[1], r[2]};
                q[d] = q[d] + (sg ? -a : a);
                w.B[(1 + 2 * d + sg) * s.Nb + mu] = basis_value(s, mu, q);
            }
        w.B[7 * s.Nb + mu] = g[0];
        w.B[8 * s.Nb + mu] = g[1];
        w.B[9 * s.Nb + mu] = g[2];
        w.B[10 * s.Nb + mu] = l;
    }
    __syncthreads();
    const int n = nspin(s, spin_of(s, j));
    for (int idx = lane; idx < 11 * n; idx += kWave) {
        const int row = idx / n, k = idx - row * n;
        const double* b = w.B + row * s.Nb;
        double acc = 0.0;
        for (int mu = 0; mu < s.Nb; ++mu) acc += s.C[mu * s.Norb + k] * b[mu];
        w.rows[row * s.ns + k] = acc;
    }
    __syncthreads();
}

// Store electron j's rows: Slater row, the 6 neighbour rows, derivatives.
__device__ void store_rows(const DevSys& s, const Walker& w, int j, int lane, bool arow)
{
    const int n = nspin(s, spin_of(s, j));
    for (int idx = lane; idx < 11 * n; idx += kWave) {
        const int row = idx / n, k = idx - row * n;
        const double v = w.rows[row * s.ns + k];
        if (row == 0) { if (arow) w.Arow[j * s.ns + k] = v; }
        else if (row <= 6) w.Phi[(6 * j + row - 1) * s.ns + k] = v;
        else w.dPhi[(4 * j + row - 7) * s.ns + k] = v;
    }
    __syncthreads();
}

// FP64 Gauss-Jordan inverse with partial pivoting of the transposed Slater
// matrix of spin sp: AinvT[c][k] = (A^-1)[k][c].  Accumulates log|det| and
// sign.  Returns false for an exactly singular matrix.
__device__ bool refresh_inverse(const DevSys& s, const Walker& w, int sp, int lane)
{
    const int n = nspin(s, sp);
    if (!n) return true;
    const int off = sp ? s.Nup : 0, n2 = 2 * n;
    double* M = w.B;                     // [n][2n]
    for (int idx = lane; idx < n * n2; idx += kWave) {
        const int r = idx / n2, c = idx - r * n2;
        M[idx] = c < n ? w.Arow[(off + c) * s.ns + r] : (c - n == r ? 1.0 : 0.0);
    }
    __syncthreads();
    double logdet = 0.0, sign = 1.0;
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        // pivot: largest |M[r][j]| for r >= j, first one on ties
        double best = -1.0;
        int bi = n;
        for (int r = j + lane; r < n; r += kWave) {
            const double v = fabs(M[r * n2 + j]);
            if (v > best) { best = v; bi = r; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o);
            const int oi = __shfl_xor(bi, o);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        best = __shfl(best, 0); bi = __shfl(bi, 0);
        if (!(best > 0.0)) { ok = false; break; }
        if (bi != j) {
            for (int c = lane; c < n2; c += kWave) {
                const double t = M[j * n2 + c];
                M[j * n2 + c] = M[bi * n2 + c];
                M[bi * n2 + c] = t;
            }
            sign = -sign;
            __syncthreads();
        }
        const double pv = M[j * n2 + j];
        logdet += log(fabs(pv));
        if (pv < 0) sign = -sign;
        __syncthreads();
        for (int c = lane; c < n2; c += kWave) M[j * n2 + c] = M[j * n2 + c] / pv;
        for (int r = lane; r < n; r += kWave) w.tmp[r] = M[r * n2 + j];
        __syncthreads();
        for (int idx = lane; idx < n * n2; idx += kWave) {
            const int r = idx / n2, c = idx - r * n2;
            if (r != j) M[idx] -= w.tmp[r] * M[j * n2 + c];
        }
        __syncthreads();
    }
    if (ok) {
        double* Ai = w.AinvT + sp * s.ns * s.ns;
        for (int idx = lane; idx < n * n; idx += kWave) {
            const int c = idx / n, k = idx - c * n;
            Ai[c * s.ns + k] = M[c * n2 + n + k];
        }
        if (lane == 0) {
            w.scal[kScLogdet0 + sp] = logdet;
            w.scal[kScSign0 + sp] = sign;
        }
    }
    __syncthreads();
    return ok;
}

// Full Jastrow / potential pieces of electron j from scratch: the Jastrow
// exponent change of its 6 moves, grad_j J, lap_j J, nu_ei(r_j), nu^a_ei(r_j),
// and its pair contribution to V_ee (pairs k > j).  Returns the V_ee part.
__device__ double electron_jastrow(const DevSys& s, const Walker& w, int j, double a, int lane)
{
    const double* rj = w.pos + 3 * j;
    double pts[7][3];
    for (int q = 0; q < 7; ++q) {
        pts[q][0] = rj[0]; pts[q][1] = rj[1]; pts[q][2] = rj[2];
    }
    for (int d = 0; d < 3; ++d)
        for (int sg = 0; sg < 2; ++sg) pts[1 + 2 * d + sg][d] = rj[d] + (sg ? -a : a);
    double S[7] = {0, 0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0}, l = 0.0, vee = 0.0, nu = 0.0,
           nua = 0.0;
    const int K = s.N + s.M;
    for (int k = lane; k < K; k += kWave) {
        if (k == j) continue;
        const double* pk;
        const double* prm;
        const bool isel = k < s.N;
        if (isel) { pk = w.pos + 3 * k; prm = ee_par(s, j, k); }
        else { pk = s.R + 3 * (k - s.N); prm = s.jas + 3 * (2 + s.spec[k - s.N]); }
        const bool jas_on = isel || s.has_en;
        if (jas_on) {
            for (int q = 0; q < 7; ++q)
                S[q] += pade_u(prm, norm3(pts[q][0] - pk[0], pts[q][1] - pk[1], pts[q][2] - pk[2]));
            const double d[3] = {rj[0] - pk[0], rj[1] - pk[1], rj[2] - pk[2]};
            const double r = norm3(d[0], d[1], d[2]);
            double u, du, d2u;
            pade_all(prm, r, u, du, d2u);
            for (int c = 0; c < 3; ++c) g[c] += du * d[c] / r;
            l += d2u + 2.0 * du / r;
            if (isel && k > j) vee += 1.0 / r;
        }
        if (!isel) {
            const int I = k - s.N;
            const double r = norm3(rj[0] - pk[0], rj[1] - pk[1], rj[2] - pk[2]);
            if (s.core[I] == 0) {
                nu += -s.Z[I] / r;
                nua += -s.Z[I] / (r > a ? r : a);
            } else {
                const double t = -s.Z[I] * erf(r / s.rc[I]) / r;
                nu += t; nua += t;
            }
        }
    }
    for (int q = 0; q < 7; ++q) S[q] = wave_sum(S[q]);
    for (int c = 0; c < 3; ++c) g[c] = wave_sum(g[c]);
    l = wave_sum(l); vee = wave_sum(vee); nu = wave_sum(nu); nua = wave_sum(nua);
    if (lane == 0) {
        for (int q = 0; q < 6; ++q) w.dJ[6 * j + q] = S[q + 1] - S[0];
        for (int c = 0; c < 3; ++c) w.Jg[3 * j + c] = g[c];
        w.Jl[j] = l; w.nue[j] = nu; w.nua[j] = nua;
    }
    return vee;
}

// Ratios of the moves of spin sp (or of every spin when sp < 0), from the
// orbital rows, the inverse and the Jastrow exponent changes.
__device__ void recompute_ratios(const DevSys& s, const Walker& w, int sp, int lane)
{
    for (int p = lane; p < s.P; p += kWave) {
        const int j = p / 6, spj = spin_of(s, j);
        if (sp < 0 || spj == sp) {
            const int n = nspin(s, spj), c = col_of(s, j);
            const double* ai = w.AinvT + spj * s.ns * s.ns + c * s.ns;
            const double* ph = w.Phi + p * s.ns;
            double rd = 0.0;
            for (int k = 0; k < n; ++k) rd += ph[k] * ai[k];
            w.Rdet[p] = rd;
        }
        w.R[p] = w.Rdet[p] * exp(w.dJ[p]);
    }
    __syncthreads();
}

// FP64 refresh: inverses and log-determinants from the exact orbital rows,
// Jastrow caches and V_ee from scratch, all ratios.
__device__ bool refresh_all(const DevSys& s, const Walker& w, double a, int lane)
{
    bool ok = refresh_inverse(s, w, 0, lane);
    ok = refresh_inverse(s, w, 1, lane) && ok;
    double vee = 0.0;
    for (int j = 0; j < s.N; ++j) vee += electron_jastrow(s, w, j, a, lane);
    if (lane == 0) w.scal[kScVee] = vee;
    __syncthreads();
    recompute_ratios(s, w, -1, lane);
    return ok;
}

// Lattice-regularized diagonal and local energy at the current configuration
// (App. D; Sec. II.C e_L = W - bbar).
struct Local { double bbar, W, eL; };

__device__ Local evaluate(const DevSys& s, const Walker& w, const PhaseArgs& pa, int lane)
{
    const double a = pa.a, ia2 = 1.0 / (a * a), inv2a2 = 1.0 / (2.0 * a * a);
    double bs = 0.0, vs = 0.0;
    int anyneg = 0;
    for (int p = lane; p < s.P; p += kWave) {
        const double r = w.R[p];
        if (r > 0) bs += r;
        else if (r < 0) { vs += -r; anyneg = 1; }
    }
    bs = wave_sum(bs);
    vs = wave_sum(vs);
    const bool anynode = __ballot(anyneg) != 0;
    double sum_opt = 0.0;
    for (int j = lane; j < s.N; j += kWave) {
        const int sp = spin_of(s, j), n = nspin(s, sp), c = col_of(s, j);
        const double* ai = w.AinvT + sp * s.ns * s.ns + c * s.ns;
        const double* dp = w.dPhi + 4 * j * s.ns;
        double g0 = 0, g1 = 0, g2 = 0, ld = 0;
        for (int k = 0; k < n; ++k) {
            const double x = ai[k];
            g0 += dp[k] * x;
            g1 += dp[s.ns + k] * x;
            g2 += dp[2 * s.ns + k] * x;
            ld += dp[3 * s.ns + k] * x;
        }
        const double* jg = w.Jg + 3 * j;
        const double lap = ld + 2.0 * (g0 * jg[0] + g1 * jg[1] + g2 * jg[2]) + w.Jl[j] +
                           jg[0] * jg[0] + jg[1] * jg[1] + jg[2] * jg[2];
        double lapA = 0.0;
        int nd = 0;
        for (int q = 0; q < 6; ++q) {
            const double r = w.R[6 * j + q];
            lapA += (r - 1.0) / (a * a);
            if (r < 0) nd = 1;
        }
        (void)ia2;
        if (pa.nu_mode == 1) nd = anynode;
        if (pa.nu_mode == 2) nd = 1;
        const double nuzv = w.nue[j] + 0.5 * (lapA - lap);
        const double numax = nuzv > w.nua[j] ? nuzv : w.nua[j];
        sum_opt += nd ? numax : nuzv;
    }
    sum_opt = wave_sum(sum_opt);
    Local L;
    L.bbar = bs * inv2a2;
    const double vsf = vs * inv2a2;
    L.W = 3.0 * s.N / (a * a) + sum_opt + w.scal[kScVee] + vsf + s.vii;
    L.eL = L.W - L.bbar;
    return L;
}

// Heat-bath choice: first p with cumulative positive ratio > xi * total.
__device__ int heat_bath(const DevSys& s, const Walker& w, double xi, int lane)
{
    const int per = (s.P + kWave - 1) / kWave;
    const int p0 = lane * per, p1 = min(p0 + per, s.P);
    double loc = 0.0;
    for (int p = p0; p < p1; ++p) {
        const double r = w.R[p];
        if (r > 0) loc += r;
    }
    const double inc = wave_incl_scan(loc, lane);
    const double tot = __shfl(inc, kWave - 1);
    if (!(tot > 0)) return -1;
    const double t = xi * tot;
    double c = __shfl_up(inc, 1);
    if (lane == 0) c = 0.0;
    int found = -1, lastpos = -1;
    for (int p = p0; p < p1; ++p) {
        const double r = w.R[p];
        if (r > 0) {
            c += r;
            lastpos = p;
            if (found < 0 && c > t) found = p;
        }
    }
    const unsigned long long m = __ballot(found >= 0);
    if (m) return __shfl(found, __ffsll((long long)m) - 1);
    const unsigned long long mp = __ballot(lastpos >= 0);
    return __shfl(lastpos, 63 - __clzll((long long)mp));
}

// Apply move p: position, Sherman-Morrison inverse update of the moved spin,
// new orbital rows of the moved electron, Jastrow / potential caches, ratios.
// Returns true when the determinant ratio was tiny (a refresh is forced).
__device__ bool apply_move(const DevSys& s, const Walker& w, const PhaseArgs& pa, int p,
                           int lane)
{
    const double a = pa.a;
    const int i = p / 6, d = (p / 2) % 3, sg = p % 2;
    const int sp = spin_of(s, i), c = col_of(s, i), n = nspin(s, sp);
    const double Rd = w.Rdet[p];
    double rold[3] = {w.pos[3 * i], w.pos[3 * i + 1], w.pos[3 * i + 2]};
    double rnew[3] = {rold[0], rold[1], rold[2]};
    rnew[d] = rnew[d] + (sg ? -a : a);

    // Sherman-Morrison on AinvT of spin sp with the accepted orbital row u
    double* Ai = w.AinvT + sp * s.ns * s.ns;
    double* u = w.tmp;                  // [ns]
    double* rowc = w.tmp + s.ns;        // [ns]
    double* beta = w.tmp + 2 * s.ns;    // [ns]
    for (int k = lane; k < n; k += kWave) {
        u[k] = w.Phi[p * s.ns + k];
        rowc[k] = Ai[c * s.ns + k];
    }
    __syncthreads();
    for (int cc = lane; cc < n; cc += kWave) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += u[k] * Ai[cc * s.ns + k];
        beta[cc] = acc;
    }
    __syncthreads();
    for (int idx = lane; idx < n * n; idx += kWave) {
        const int cc = idx / n, k = idx - cc * n;
        if (cc == c) Ai[cc * s.ns + k] = rowc[k] / Rd;
        else Ai[cc * s.ns + k] -= rowc[k] * (beta[cc] / Rd);
    }
    for (int k = lane; k < n; k += kWave) w.Arow[i * s.ns + k] = u[k];
    if (lane == 0) {
        w.scal[kScLogdet0 + sp] += log(fabs(Rd));
        if (Rd < 0) w.scal[kScSign0 + sp] = -w.scal[kScSign0 + sp];
    }
    __syncthreads();

    // new orbital rows of electron i at rnew
    electron_rows(s, w, i, rnew, a, lane);
    store_rows(s, w, i, lane, false);

    // Jastrow and potential caches: pairs (i, k) change from rold to rnew
    double pts[7][3];
    for (int q = 0; q < 7; ++q) { pts[q][0] = rnew[0]; pts[q][1] = rnew[1]; pts[q][2] = rnew[2]; }
    for (int dd = 0; dd < 3; ++dd)
        for (int s2 = 0; s2 < 2; ++s2) pts[1 + 2 * dd + s2][dd] = rnew[dd] + (s2 ? -a : a);
    double S[7] = {0, 0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0}, l = 0.0, dvee = 0.0, nu = 0.0,
           nua = 0.0;
    const int K = s.N + s.M;
    for (int k = lane; k < K; k += kWave) {
        if (k == i) continue;
        const bool isel = k < s.N;
        const double* pk;
        const double* prm;
        if (isel) { pk = w.pos + 3 * k; prm = ee_par(s, i, k); }
        else { pk = s.R + 3 * (k - s.N); prm = s.jas + 3 * (2 + s.spec[k - s.N]); }
        if (isel || s.has_en) {
            for (int q = 0; q < 7; ++q)
                S[q] += pade_u(prm, norm3(pts[q][0] - pk[0], pts[q][1] - pk[1], pts[q][2] - pk[2]));
            const double dn[3] = {rnew[0] - pk[0], rnew[1] - pk[1], rnew[2] - pk[2]};
            const double rn = norm3(dn[0], dn[1], dn[2]);
            double un, dun, d2un;
            pade_all(prm, rn, un, dun, d2un);
            for (int cc = 0; cc < 3; ++cc) g[cc] += dun * dn[cc] / rn;
            l += d2un + 2.0 * dun / rn;
            if (isel) {
                const double dol[3] = {rold[0] - pk[0], rold[1] - pk[1], rold[2] - pk[2]};
                const double ro = norm3(dol[0], dol[1], dol[2]);
                double uo, duo, d2uo;
                pade_all(prm, ro, uo, duo, d2uo);
                w.dje[k] = un - uo;
                // electron k sees the pair through r_k - r_i = -(r_i - r_k)
                for (int cc = 0; cc < 3; ++cc)
                    w.Jg[3 * k + cc] += -(dun * dn[cc] / rn) + duo * dol[cc] / ro;
                w.Jl[k] += (d2un + 2.0 * dun / rn) - (d2uo + 2.0 * duo / ro);
                dvee += 1.0 / rn - 1.0 / ro;
            }
        }
        if (!isel) {
            const int I = k - s.N;
            const double r = norm3(rnew[0] - pk[0], rnew[1] - pk[1], rnew[2] - pk[2]);
            if (s.core[I] == 0) {
                nu += -s.Z[I] / r;
                nua += -s.Z[I] / (r > a ? r : a);
            } else {
                const double t = -s.Z[I] * erf(r / s.rc[I]) / r;
                nu += t; nua += t;
            }
        }
    }
    for (int q = 0; q < 7; ++q) S[q] = wave_sum(S[q]);
    for (int cc = 0; cc < 3; ++cc) g[cc] = wave_sum(g[cc]);
    l = wave_sum(l); dvee = wave_sum(dvee); nu = wave_sum(nu); nua = wave_sum(nua);
    __syncthreads();
    // Jastrow exponent changes of the other electrons' moves
    for (int q = lane; q < s.P; q += kWave) {
        const int j = q / 6;
        if (j == i) continue;
        const int dd = (q / 2) % 3, s2 = q % 2;
        const double* prm = ee_par(s, i, j);
        double r2[3] = {w.pos[3 * j], w.pos[3 * j + 1], w.pos[3 * j + 2]};
        r2[dd] = r2[dd] + (s2 ? -a : a);
        const double un = pade_u(prm, norm3(r2[0] - rnew[0], r2[1] - rnew[1], r2[2] - rnew[2]));
        const double uo = pade_u(prm, norm3(r2[0] - rold[0], r2[1] - rold[1], r2[2] - rold[2]));
        w.dJ[q] += (un - uo) - w.dje[j];
    }
    if (lane == 0) {
        for (int q = 0; q < 6; ++q) w.dJ[6 * i + q] = S[q + 1] - S[0];
        for (int cc = 0; cc < 3; ++cc) w.Jg[3 * i + cc] = g[cc];
        w.Jl[i] = l; w.nue[i] = nu; w.nua[i] = nua;
        w.scal[kScVee] += dvee;
        w.pos[3 * i + d] = rnew[d];
    }
    __syncthreads();
    recompute_ratios(s, w, sp, lane);
    return fabs(Rd) < 1e-6;
}

// ---------------------------------------------------------------------------
// the phase kernel: one workgroup = one wavefront = one walker
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void phase_fp64(DevSys s, PhaseArgs pa)
{
    extern __shared__ double lds[];
    const int wid = blockIdx.x;
    if (wid >= s.nw) return;
    const int lane = threadIdx.x;
    Walker w;
    w.pos = lds + s.o_pos; w.R = lds + s.o_R; w.Rdet = lds + s.o_Rdet; w.dJ = lds + s.o_dJ;
    w.Arow = lds + s.o_Arow; w.AinvT = lds + s.o_AinvT; w.Jg = lds + s.o_Jg; w.Jl = lds + s.o_Jl;
    w.nue = lds + s.o_nue; w.nua = lds + s.o_nua; w.dje = lds + s.o_dje; w.scal = lds + s.o_scal;
    w.B = lds + s.o_B; w.rows = lds + s.o_rows; w.tmp = lds + s.o_tmp;
    double* sp_base = s.spill + (long)wid * s.spill_stride;
    w.Phi = sp_base + s.s_Phi;
    w.dPhi = sp_base + s.s_dPhi;

    for (int q = lane; q < 3 * s.N; q += kWave) w.pos[q] = s.pos[(long)wid * 3 * s.N + q];
    __syncthreads();
    const double a = pa.a;
    // orbital rows of every electron, then the FP64 refresh
    for (int j = 0; j < s.N; ++j) {
        double r[3] = {w.pos[3 * j], w.pos[3 * j + 1], w.pos[3 * j + 2]};
        electron_rows(s, w, j, r, a, lane);
        store_rows(s, w, j, lane, true);
    }
    unsigned long long n_neg = 0, n_nomove = 0, n_refresh = 1, n_small = 0, n_sing = 0,
                       n_capped = 0;
    if (!refresh_all(s, w, a, lane)) n_sing++;

    double lw = s.lw[wid];
    double tau_left = pa.tau;
    int it = 0, since = 0;
    Local L;
    int32_t* tr = s.trace ? s.trace + (long)wid * s.trace_cap : nullptr;
    for (;;) {
        if (pa.scheme == 0 && it >= pa.nproj) break;
        L = evaluate(s, w, pa, lane);
        int q;
        if (pa.scheme == 0) {
            const double den = L.W - pa.E0;
            if (!(den > 0)) { lw = -INFINITY; n_neg++; }
            else if (!(L.bbar > 0)) { lw = -INFINITY; n_nomove++; }
            else lw += log(L.bbar) - log(den);
            const double xi = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)pa.j,
                                             (uint64_t)it, kMove);
            q = heat_bath(s, w, xi, lane);
            if (tr && it < s.trace_cap && lane == 0) tr[it] = q;
            ++it;
        } else {
            const double xt = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)pa.j,
                                             (uint64_t)it, kPersist);
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
            const double xi = philox_uniform(pa.seed, s.sysid, (uint64_t)wid, (uint64_t)pa.j,
                                             (uint64_t)(it - 1), kMove);
            q = heat_bath(s, w, xi, lane);
            if (tr && it - 1 < s.trace_cap && lane == 0) tr[it - 1] = q;
        }
        if (q >= 0) {
            const bool small = apply_move(s, w, pa, q, lane);
            ++since;
            if (small) n_small++;
            if (small || since >= pa.refresh_every) {
                if (!refresh_all(s, w, a, lane)) n_sing++;
                n_refresh++;
                since = 0;
            }
        }
    }
    if (pa.scheme == 0) L = evaluate(s, w, pa, lane);

    for (int q = lane; q < 3 * s.N; q += kWave) s.pos[(long)wid * 3 * s.N + q] = w.pos[q];
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
        atomicMax(cn + kCntMaxIters, (unsigned long long)it);
        atomicMin(cn + kCntMinIters, (unsigned long long)it);
    }
}

// ---------------------------------------------------------------------------
// reconfiguration (Sec. II.A): one workgroup computes max log-weight, the
// FP64 inclusive prefix of exp(lw - max) in slot order, and the weighted
// local-energy sums; then one thread per new walker runs the comb search
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBranchBlock) void branch_scan(DevSys s, int scheme, double E0,
                                                               double* cum, double* out)
{
    __shared__ double sh[kMaxBranchBlock];
    __shared__ int shi[kMaxBranchBlock];
    const int t = threadIdx.x, nt = blockDim.x, nw = s.nw;
    const int per = (nw + nt - 1) / nt, b0 = t * per, b1 = min(b0 + per, nw);
    double mx = -INFINITY;
    int last = -1;
    for (int b = b0; b < b1; ++b) {
        const double v = s.lw[b];
        if (v > mx) mx = v;
        if (v > -INFINITY) last = b;
    }
    sh[t] = mx; shi[t] = last;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
        if (t < o) {
            sh[t] = fmax(sh[t], sh[t + o]);
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
        const double om = scheme == 0 ? wv / (s.Wd[b] - E0) : wv;
        if (om != 0.0) { se += om * s.eL[b]; so += om; }
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

__global__ void branch_comb(DevSys s, uint64_t seed, int j, const double* cum, const double* out,
                            int32_t* sel)
{
    const int al = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = s.nw;
    if (al >= nw) return;
    const double xi = philox_uniform(seed, s.sysid, 0, (uint64_t)j, 0, kComb);
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

__global__ void branch_gather(DevSys s, const int32_t* sel, const double* pos_old,
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

}  // namespace lrdmc
