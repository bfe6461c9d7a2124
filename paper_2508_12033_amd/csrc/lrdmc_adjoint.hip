// Per-walker derivatives of the lattice-regularized local energy e_L and of
// log|Psi_G| with respect to the nuclear coordinates and the Pade Jastrow
// parameters, at a fixed configuration, by a hand-written reverse (adjoint)
// pass.  One 256-thread workgroup per walker, FP64 throughout, all per-walker
// data in LDS.
//
// Forward (at fixed x, the inverse recomputed by FP64 Gauss-Jordan rather than
// carried by rank-one updates):
//   A_s[c][k] = phi_k(r_c), Ainv_s;  R_p = Rdet_p exp(dJ_p) for the 6N moves;
//   L_i = lapD_i + 2 gD_i.gJ_i + lapJ_i + |gJ_i|^2  (continuum lap Psi / Psi);
//   lapA_i = sum_{q in i} (R_q - 1)/a^2;  nu_zv,i = nu_i + (lapA_i - L_i)/2;
//   d_i = [electron i regularized (nu_opt mode) and nu^a_i > nu_zv,i];
//   e_L = sum_i (-L_i/2 + nu_i + d_i (nu^a_i - nu_zv,i)) + V_ee + V_ii
// (App. D; e_L = W - bbar), log|Psi| = sum_s log|det A_s| + J.
// Reverse: with d_i held fixed (the active branch of the max),
//   de_L/dL_i = -(1 - d_i)/2 =: alpha_i, de_L/dR_q = -d_i/(2 a^2) =: beta_i,
//   de_L/dnu_i = 1 - d_i, de_L/dnu^a_i = d_i;
// determinant quantities Q_c = sum_k Y_c[k] Ainv[k][c] pass their adjoints to
// the Slater matrix as Abar = -Ainv^T Ybar Ainv^T (d Ainv = -Ainv dA Ainv), and
// every basis function moves with its nucleus (d chi / dR = -grad chi), which
// needs its gradient, Hessian and the gradient of its Laplacian.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lrdmc_dev.hpp"
#include "lrdmc_devfn.hpp"
#include "lrdmc_deriv.hpp"

namespace lrdmc {

extern __shared__ double lds[];

namespace {

constexpr int kT = kAdjThreads;

__device__ __forceinline__ double blk_sum(double v, double* red)
{
    v = wave_sum(v);
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ int aspin(const DevAdj& s, int i) { return i >= s.Nup; }
__device__ __forceinline__ int acol(const DevAdj& s, int i) { return i >= s.Nup ? i - s.Nup : i; }
__device__ __forceinline__ int ansp(const DevAdj& s, int sp) { return sp ? s.Ndn : s.Nup; }

// partner k of electron i: position and Pade row
__device__ __forceinline__ void apartner(const DevAdj& s, const double* pos, int i, int k,
                                         double* pk, int& jr)
{
    if (k < s.N) {
        pk[0] = pos[3 * k]; pk[1] = pos[3 * k + 1]; pk[2] = pos[3 * k + 2];
        jr = ((i >= s.Nup) == (k >= s.Nup)) ? 0 : 1;
    } else {
        const int I = k - s.N;
        pk[0] = s.R[3 * I]; pk[1] = s.R[3 * I + 1]; pk[2] = s.R[3 * I + 2];
        jr = 2 + s.spec[I];
    }
}

// nuclear potential of nucleus I at distance r: nu, nu^a and their r-derivatives
__device__ __forceinline__ void apot(const DevAdj& s, int I, double r, double a, double& nu,
                                     double& nua, double& dnu, double& dnua)
{
    const double Z = s.Z[I];
    if (s.core[I] == 0) {
        nu = -Z / r;
        dnu = Z / (r * r);
        if (r > a) { nua = nu; dnua = dnu; }
        else { nua = -Z / a; dnua = 0.0; }
    } else {
        const double q = r * r + s.rc[I] * s.rc[I], iq = 1.0 / sqrt(q);
        nu = nua = -Z * iq;
        dnu = dnua = Z * r * iq * iq * iq;
    }
}

// in-place Gauss-Jordan with partial pivoting of the n x n matrix G (row
// stride n) in LDS; on return G holds G^{-1}.  piv: n ints of LDS scratch,
// colk: n doubles.  Returns false if G is singular; logdet / sign of G.
__device__ bool gauss_jordan(double* G, int n, int* piv, double* colk, double& logdet, double& sign)
{
    const int tid = threadIdx.x;
    logdet = 0.0; sign = 1.0;
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = k;
        for (int r = k; r < n; ++r) {
            const double v = fabs(G[r * n + k]);
            if (v > best) { best = v; bi = r; }
        }
        if (!(best > 0.0)) return false;
        __syncthreads();   // every wave has read column k before any row moves
        if (tid == 0) piv[k] = bi;
        if (bi != k) {
            for (int c = tid; c < n; c += kT) {
                const double t = G[k * n + c];
                G[k * n + c] = G[bi * n + c];
                G[bi * n + c] = t;
            }
            sign = -sign;
            __syncthreads();
        }
        const double d = G[k * n + k];
        logdet += log(fabs(d));
        if (d < 0) sign = -sign;
        const double id = 1.0 / d;
        __syncthreads();
        for (int r = tid; r < n; r += kT) colk[r] = G[r * n + k];
        __syncthreads();
        for (int c = tid; c < n; c += kT) G[k * n + c] = (c == k ? 1.0 : G[k * n + c]) * id;
        __syncthreads();
        for (int idx = tid; idx < n * n; idx += kT) {
            const int r = idx / n, c = idx - r * n;
            if (r == k) continue;
            G[idx] = (c == k ? 0.0 : G[idx]) - colk[r] * G[k * n + c];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k)
            for (int r = tid; r < n; r += kT) {
                const double t = G[r * n + k];
                G[r * n + k] = G[r * n + p];
                G[r * n + p] = t;
            }
        __syncthreads();
    }
    return true;
}

}  // namespace

__global__ __launch_bounds__(kAdjThreads) void walker_derivs(const DevAdj* __restrict__ sys)
{
    const DevAdj& s = *sys;
    const int wid = blockIdx.x;
    if (wid >= s.nw) return;
    const int tid = threadIdx.x;
    const int N = s.N, M = s.M, Nb = s.Nb, ns = s.ns, P = 6 * N, nth = s.nth;
    const double a = s.a, ia2 = 1.0 / (a * a);
    double* pos = lds + s.o_pos;
    double* phi = lds + s.o_phi;       // [N][ns]       phi_k(r_i)
    double* dphi = lds + s.o_dphi;     // [N][4][ns]    grad, Laplacian
    double* phi6 = lds + s.o_phi6;     // [N][6][ns]    phi_k at the 6 moves
    double* ainv = lds + s.o_ainv;     // [2][ns][ns]   Ainv_s[k][c]
    double* Zm = lds + s.o_Z;          // [2][Nb][ns]   Z_s[mu][c] = sum_k C[mu][k] Ainv_s[k][c]
    double* Tm = lds + s.o_T;          // [N][Nb]       T[i][mu] = sum_b Abar_s[c_i][b] C[mu][b]
    double* Ym = lds + s.o_Y;          // [2][ns][ns]   Ybar_s[k][c], then Abar_s[c][b]
    double* G = lds + s.o_G;           // [ns][ns] + ns Gauss-Jordan / product scratch
    double* chi = lds + s.o_chi;       // [11][Nb]      basis rows of one electron
    double* gj = lds + s.o_gj;         // [N][3]
    double* Lj = lds + s.o_Lj;         // [N]
    double* dJ = lds + s.o_dJ;         // [P]
    double* Rr = lds + s.o_R;          // [P]
    double* Rd = lds + s.o_Rdet;       // [P]
    double* gd = lds + s.o_gd;         // [N][3]
    double* Ld = lds + s.o_Ld;         // [N]
    double* nu = lds + s.o_nu;         // [N]
    double* nua = lds + s.o_nua;       // [N]
    double* al = lds + s.o_al;         // [N]     de_L/dL_i
    double* sgd = lds + s.o_sgd;       // [N][3]  de_L/dgD_i
    double* sgj = lds + s.o_sgj;       // [N][3]  de_L/dgJ_i
    double* sRd = lds + s.o_sRd;       // [P]     de_L/dRdet_p
    double* sdJ = lds + s.o_sdJ;       // [P]     de_L/ddJ_p
    double* snu = lds + s.o_snu;       // [N]     de_L/dnu_i
    double* snua = lds + s.o_snua;     // [N]     de_L/dnu^a_i
    double* GeL = lds + s.o_GeL;       // [nth]
    double* Glp = lds + s.o_Glp;       // [nth]
    double* sc = lds + s.o_sc;         // [16]    scalars, reduction scratch at sc + 8
    int* piv = reinterpret_cast<int*>(lds + s.o_piv);
    double* red = sc + 8;

    for (int q = tid; q < 3 * N; q += kT) pos[q] = s.pos[(long)wid * 3 * N + q];
    for (int q = tid; q < nth; q += kT) { GeL[q] = 0.0; Glp[q] = 0.0; }
    __syncthreads();

    // ---- orbital rows of every electron: value, 6 moves, gradient, Laplacian
    for (int i = 0; i < N; ++i) {
        const int n = ansp(s, aspin(s, i));
        for (int it = tid; it < 7 * Nb; it += kT) {
            const int q = it / Nb, mu = it - q * Nb;
            double p[3];
            point_q(pos + 3 * i, q, a, p);
            const double* rec = s.btab + 4 * mu;
            const double dx = p[0] - rec[0], dy = p[1] - rec[1], dz = p[2] - rec[2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (q == 0) {
                double v, g[3], l;
                basis_vgl_d(s.btype[mu], rec[3], dx, dy, dz, d2, v, g, l);
                chi[mu] = v;
                chi[7 * Nb + mu] = g[0]; chi[8 * Nb + mu] = g[1]; chi[9 * Nb + mu] = g[2];
                chi[10 * Nb + mu] = l;
            } else {
                chi[q * Nb + mu] = basis_value_d(s.btype[mu], rec[3], dx, dy, dz, d2);
            }
        }
        __syncthreads();
        for (int it = tid; it < 11 * n; it += kT) {
            const int row = it / n, k = it - row * n;
            double acc = 0.0;
            for (int mu = 0; mu < Nb; ++mu) acc += chi[row * Nb + mu] * s.C[mu * s.Norb + k];
            if (row == 0) phi[i * ns + k] = acc;
            else if (row <= 6) phi6[(i * 6 + row - 1) * ns + k] = acc;
            else dphi[(i * 4 + row - 7) * ns + k] = acc;
        }
        __syncthreads();
    }

    // ---- inverses (FP64 Gauss-Jordan) and log|det|
    double logdet = 0.0;
    int bad = 0;
    for (int sp = 0; sp < 2; ++sp) {
        const int n = ansp(s, sp), off = sp ? s.Nup : 0;
        if (!n) continue;
        for (int idx = tid; idx < n * n; idx += kT) {
            const int c = idx / n, k = idx - c * n;
            G[idx] = phi[(off + c) * ns + k];           // G[c][k] = A[c][k]
        }
        __syncthreads();
        double ld, sg;
        if (!gauss_jordan(G, n, piv, G + ns * ns, ld, sg)) { bad = 1; break; }
        logdet += ld;
        for (int idx = tid; idx < n * n; idx += kT) {
            const int k = idx / n, c = idx - k * n;
            ainv[sp * ns * ns + k * ns + c] = G[idx];   // G now holds A^{-1}[k][c]
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) {
            atomicAdd(s.status, 1);
            s.eL[wid] = NAN; s.lp[wid] = NAN;
        }
        for (int q = tid; q < nth; q += kT) {
            s.deL[(long)wid * nth + q] = NAN; s.dlp[(long)wid * nth + q] = NAN;
        }
        return;
    }
    // Z_s = C Ainv_s
    for (int sp = 0; sp < 2; ++sp) {
        const int n = ansp(s, sp);
        for (int idx = tid; idx < Nb * n; idx += kT) {
            const int mu = idx / n, c = idx - mu * n;
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += s.C[mu * s.Norb + k] * ainv[sp * ns * ns + k * ns + c];
            Zm[(sp * Nb + mu) * ns + c] = acc;
        }
    }

    // ---- per electron: Jastrow pieces, potentials, determinant pieces
    double Jsum = 0.0, vee = 0.0;
    for (int i = tid; i < N; i += kT) {
        double g0 = 0, g1 = 0, g2 = 0, l = 0, dj[6] = {0, 0, 0, 0, 0, 0};
        double v = 0.0, va = 0.0;
        for (int k = 0; k < N + M; ++k) {
            if (k == i) continue;
            double pk[3];
            int jr;
            apartner(s, pos, i, k, pk, jr);
            const double* pp = s.jas + 3 * jr;
            const double d0 = pos[3 * i] - pk[0], d1 = pos[3 * i + 1] - pk[1], d2 = pos[3 * i + 2] - pk[2];
            const double r = norm3(d0, d1, d2);
            double u, dur, lp;
            pade_derivs(pp, r, u, dur, lp);
            g0 += dur * d0; g1 += dur * d1; g2 += dur * d2;
            l += lp;
            for (int q = 0; q < 6; ++q) {
                double pq[3];
                point_q(pos + 3 * i, q + 1, a, pq);
                dj[q] += pade_u(pp, norm3(pq[0] - pk[0], pq[1] - pk[1], pq[2] - pk[2])) - u;
            }
            if (k >= N) {
                Jsum += u;
                double n1, n2, t1, t2;
                apot(s, k - N, r, a, n1, n2, t1, t2);
                v += n1; va += n2;
            } else if (k > i) {
                Jsum += u;
                vee += 1.0 / r;
            }
        }
        gj[3 * i] = g0; gj[3 * i + 1] = g1; gj[3 * i + 2] = g2;
        Lj[i] = l;
        for (int q = 0; q < 6; ++q) dJ[6 * i + q] = dj[q];
        nu[i] = v; nua[i] = va;
    }
    __syncthreads();
    for (int i = tid; i < N; i += kT) {
        const int sp = aspin(s, i), c = acol(s, i), n = ansp(s, sp);
        const double* Ai = ainv + sp * ns * ns;
        double q4[4] = {0, 0, 0, 0};
        for (int k = 0; k < n; ++k) {
            const double w = Ai[k * ns + c];
            for (int t = 0; t < 4; ++t) q4[t] += dphi[(i * 4 + t) * ns + k] * w;
        }
        gd[3 * i] = q4[0]; gd[3 * i + 1] = q4[1]; gd[3 * i + 2] = q4[2];
        Ld[i] = q4[3];
        for (int q = 0; q < 6; ++q) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += phi6[(i * 6 + q) * ns + k] * Ai[k * ns + c];
            Rd[6 * i + q] = acc;
            Rr[6 * i + q] = acc * exp(dJ[6 * i + q]);
        }
    }
    __syncthreads();
    int neg = 0;
    for (int p = tid; p < P; p += kT)
        if (Rr[p] < 0) neg = 1;
    const bool anynode = blk_sum(neg ? 1.0 : 0.0, red) > 0.0;
    double esum = 0.0;
    for (int i = tid; i < N; i += kT) {
        const double j0 = gj[3 * i], j1 = gj[3 * i + 1], j2 = gj[3 * i + 2];
        const double L = Ld[i] + 2.0 * (gd[3 * i] * j0 + gd[3 * i + 1] * j1 + gd[3 * i + 2] * j2) +
                         Lj[i] + j0 * j0 + j1 * j1 + j2 * j2;
        double lapA = 0.0;
        int nd = 0;
        for (int q = 0; q < 6; ++q) {
            lapA += (Rr[6 * i + q] - 1.0) * ia2;
            if (Rr[6 * i + q] < 0) nd = 1;
        }
        if (s.nu_mode == 1) nd = anynode;
        if (s.nu_mode == 2) nd = 1;
        const double nuzv = nu[i] + 0.5 * (lapA - L);
        const int di = (nd && nua[i] > nuzv) ? 1 : 0;
        esum += -0.5 * L + nu[i] + (di ? nua[i] - nuzv : 0.0);
        // adjoint seeds
        const double alpha = -0.5 * (1.0 - di), beta = -0.5 * di * ia2;
        al[i] = alpha;
        sgd[3 * i] = 2.0 * alpha * j0; sgd[3 * i + 1] = 2.0 * alpha * j1; sgd[3 * i + 2] = 2.0 * alpha * j2;
        sgj[3 * i] = 2.0 * alpha * (gd[3 * i] + j0);
        sgj[3 * i + 1] = 2.0 * alpha * (gd[3 * i + 1] + j1);
        sgj[3 * i + 2] = 2.0 * alpha * (gd[3 * i + 2] + j2);
        for (int q = 0; q < 6; ++q) {
            sRd[6 * i + q] = beta * exp(dJ[6 * i + q]);
            sdJ[6 * i + q] = beta * Rr[6 * i + q];
        }
        snu[i] = 1.0 - di;
        snua[i] = (double)di;
    }
    esum = blk_sum(esum, red);
    vee = blk_sum(vee, red);
    Jsum = blk_sum(Jsum, red);
    const double eL = esum + vee + s.vii;
    const double lpsi = logdet + Jsum;

    // ---- determinant adjoint: Ybar, Abar = -Ainv^T Ybar Ainv^T, T = Abar C^T
    for (int sp = 0; sp < 2; ++sp) {
        const int n = ansp(s, sp), off = sp ? s.Nup : 0;
        if (!n) continue;
        double* Y = Ym + sp * ns * ns;
        const double* Ai = ainv + sp * ns * ns;
        for (int idx = tid; idx < n * n; idx += kT) {
            const int k = idx / n, c = idx - k * n, i = off + c;
            double y = al[i] * dphi[(i * 4 + 3) * ns + k];
            for (int t = 0; t < 3; ++t) y += sgd[3 * i + t] * dphi[(i * 4 + t) * ns + k];
            for (int q = 0; q < 6; ++q) y += sRd[6 * i + q] * phi6[(i * 6 + q) * ns + k];
            Y[k * ns + c] = y;
        }
        __syncthreads();
        // G[k][b] = sum_c Ybar[k][c] Ainv[b][c]
        for (int idx = tid; idx < n * n; idx += kT) {
            const int k = idx / n, b = idx - k * n;
            double acc = 0.0;
            for (int c = 0; c < n; ++c) acc += Y[k * ns + c] * Ai[b * ns + c];
            G[idx] = acc;
        }
        __syncthreads();
        // Abar[a][b] = -sum_k Ainv[k][a] G[k][b]  (stored over Ybar)
        for (int idx = tid; idx < n * n; idx += kT) {
            const int aa = idx / n, b = idx - aa * n;
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Ai[k * ns + aa] * G[k * n + b];
            Y[aa * ns + b] = -acc;
        }
        __syncthreads();
        for (int idx = tid; idx < n * Nb; idx += kT) {
            const int c = idx / Nb, mu = idx - c * Nb;
            double acc = 0.0;
            for (int b = 0; b < n; ++b) acc += Y[c * ns + b] * s.C[mu * s.Norb + b];
            Tm[(off + c) * Nb + mu] = acc;
        }
        __syncthreads();
    }

    // ---- basis functions move with their nucleus: d/dR_I of chi_mu = -grad chi_mu
    for (int idx = tid; idx < N * Nb; idx += kT) {
        const int i = idx / Nb, mu = idx - i * Nb;
        const int sp = aspin(s, i), c = acol(s, i);
        const double* rec = s.btab + 4 * mu;
        const double z = Zm[(sp * Nb + mu) * ns + c], t = Tm[i * Nb + mu];
        double d[3] = {pos[3 * i] - rec[0], pos[3 * i + 1] - rec[1], pos[3 * i + 2] - rec[2]};
        double g[3], H[6], gl[3];
        basis_d3(s.btype[mu], rec[3], d, g, H, gl);
        const double* v = sgd + 3 * i;
        double e[3];
        e[0] = t * g[0] + z * (al[i] * gl[0] + H[0] * v[0] + H[1] * v[1] + H[2] * v[2]);
        e[1] = t * g[1] + z * (al[i] * gl[1] + H[1] * v[0] + H[3] * v[1] + H[4] * v[2]);
        e[2] = t * g[2] + z * (al[i] * gl[2] + H[2] * v[0] + H[4] * v[1] + H[5] * v[2]);
        for (int q = 0; q < 6; ++q) {
            double pq[3];
            point_q(pos + 3 * i, q + 1, a, pq);
            double dq[3] = {pq[0] - rec[0], pq[1] - rec[1], pq[2] - rec[2]};
            double gq[3];
            basis_grad(s.btype[mu], rec[3], dq, gq);
            const double w = z * sRd[6 * i + q];
            e[0] += w * gq[0]; e[1] += w * gq[1]; e[2] += w * gq[2];
        }
        const int I = s.batom[mu];
        for (int k = 0; k < 3; ++k) {
            atomicAdd(GeL + 3 * I + k, -e[k]);
            atomicAdd(Glp + 3 * I + k, -z * g[k]);
        }
    }

    // ---- Jastrow pairs (owner i, partner k): parameter rows and e-n nuclei
    for (int idx = tid; idx < N * (N + M); idx += kT) {
        const int i = idx / (N + M), k = idx - i * (N + M);
        if (k == i) continue;
        double pk[3];
        int jr;
        apartner(s, pos, i, k, pk, jr);
        const double* pp = s.jas + 3 * jr;
        const double d[3] = {pos[3 * i] - pk[0], pos[3 * i + 1] - pk[1], pos[3 * i + 2] - pk[2]};
        const double r = norm3(d[0], d[1], d[2]);
        PadeD f;
        pade_full(pp, r, f);
        const double* v = sgj + 3 * i;
        const double vd = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
        // parameter derivatives of this owner's e_L pieces
        double gp[3];
        for (int m = 0; m < 3; ++m)
            gp[m] = vd * f.du_p[m] / r + al[i] * (f.d2u_p[m] + 2.0 * f.du_p[m] / r);
        double gR[3] = {0, 0, 0};
        for (int q = 0; q < 6; ++q) {
            double pq[3];
            point_q(pos + 3 * i, q + 1, a, pq);
            const double dq[3] = {pq[0] - pk[0], pq[1] - pk[1], pq[2] - pk[2]};
            const double rq = norm3(dq[0], dq[1], dq[2]);
            PadeD fq;
            pade_full(pp, rq, fq);
            const double w = sdJ[6 * i + q];
            for (int m = 0; m < 3; ++m) gp[m] += w * (fq.u_p[m] - f.u_p[m]);
            for (int m = 0; m < 3; ++m) gR[m] += w * (fq.du * dq[m] / rq - f.du * d[m] / r);
        }
        for (int m = 0; m < 3; ++m) atomicAdd(GeL + 3 * M + 3 * jr + m, gp[m]);
        // log|Psi|: each e-e pair once, every e-n pair
        if (k >= N || k > i)
            for (int m = 0; m < 3; ++m) atomicAdd(Glp + 3 * M + 3 * jr + m, f.u_p[m]);
        if (k >= N) {
            const int I = k - N;
            const double c1 = f.du / r, c2 = (f.d2u - f.du / r) / (r * r);
            const double hp = f.d3u + 2.0 * f.d2u / r - 2.0 * f.du / (r * r);
            for (int m = 0; m < 3; ++m) {
                const double e = c1 * v[m] + c2 * vd * d[m] + al[i] * hp * d[m] / r + gR[m];
                atomicAdd(GeL + 3 * I + m, -e);
                atomicAdd(Glp + 3 * I + m, -f.du * d[m] / r);
            }
        }
    }

    // ---- potentials nu_i, nu^a_i and the ion-ion repulsion
    for (int idx = tid; idx < N * M; idx += kT) {
        const int i = idx / M, I = idx - i * M;
        const double d[3] = {pos[3 * i] - s.R[3 * I], pos[3 * i + 1] - s.R[3 * I + 1],
                             pos[3 * i + 2] - s.R[3 * I + 2]};
        const double r = norm3(d[0], d[1], d[2]);
        double n1, n2, t1, t2;
        apot(s, I, r, a, n1, n2, t1, t2);
        const double w = (snu[i] * t1 + snua[i] * t2) / r;
        for (int m = 0; m < 3; ++m) atomicAdd(GeL + 3 * I + m, -w * d[m]);
    }
    for (int I = tid; I < M; I += kT) {
        double f[3] = {0, 0, 0};
        for (int J = 0; J < M; ++J) {
            if (J == I) continue;
            const double d[3] = {s.R[3 * I] - s.R[3 * J], s.R[3 * I + 1] - s.R[3 * J + 1],
                                 s.R[3 * I + 2] - s.R[3 * J + 2]};
            const double r = norm3(d[0], d[1], d[2]);
            const double w = s.Z[I] * s.Z[J] / (r * r * r);
            for (int m = 0; m < 3; ++m) f[m] -= w * d[m];
        }
        for (int m = 0; m < 3; ++m) atomicAdd(GeL + 3 * I + m, f[m]);
    }
    __syncthreads();
    for (int q = tid; q < nth; q += kT) {
        s.deL[(long)wid * nth + q] = GeL[q];
        s.dlp[(long)wid * nth + q] = Glp[q];
    }
    if (tid == 0) {
        s.eL[wid] = eL;
        s.lp[wid] = lpsi;
    }
}

// Population sums for the force estimator: weights omega_w (load-balanced
// w/(W - E_0), conventional w, with w = exp(lw - max lw)), then
// out = [sum omega, sum omega e_L, sum_w omega deL[.], sum_w omega e_L dlp[.],
//        sum_w omega dlp[.]]  (3 nth + 2 values); one workgroup per column.
__global__ __launch_bounds__(256) void derivs_reduce(int nw, int nth, int scheme, const double* lw,
                                                     const double* Wd, const double* e0p,
                                                     const double* eL, const double* deL,
                                                     const double* dlp, double* out)
{
    __shared__ double sh[256];
    const int col = blockIdx.x, tid = threadIdx.x;   // col in [0, 3 nth + 2)
    double mx = -INFINITY;
    for (int w = tid; w < nw; w += 256) mx = fmax(mx, lw[w]);
    sh[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) sh[tid] = fmax(sh[tid], sh[tid + o]);
        __syncthreads();
    }
    mx = sh[0];
    __syncthreads();
    const double E0 = e0p[0];
    double acc = 0.0;
    for (int w = tid; w < nw; w += 256) {
        double om = exp(lw[w] - mx);
        if (scheme == 0) om = om / (Wd[w] - E0);
        if (!(om != 0.0)) continue;
        double v;
        if (col == 0) v = 1.0;
        else if (col == 1) v = eL[w];
        else if (col < 2 + nth) v = deL[(long)w * nth + col - 2];
        else if (col < 2 + 2 * nth) v = eL[w] * dlp[(long)w * nth + col - 2 - nth];
        else v = dlp[(long)w * nth + col - 2 - 2 * nth];
        acc += om * v;
    }
    sh[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    if (tid == 0) out[col] = sh[0];
}

}  // namespace lrdmc
