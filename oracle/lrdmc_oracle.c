/*
 * Plain FP64 CPU oracle for lattice-regularized diffusion Monte Carlo (LRDMC):
 * the conventional continuous-time scheme and the load-balanced fixed-N_proj
 * scheme of Nakano, Sorella & Casula (arXiv 2508.12033).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; its inputs come from the
 * seeded generator and the random numbers it draws come from its own copy of
 * the counter-based Philox4x64-10 generator (Salmon et al., SC'11).
 *
 * Design rule: every quantity is recomputed from the electron positions by
 * its plain definition at every step -- basis functions evaluated directly,
 * Slater matrices inverted by a fresh LU factorisation with partial pivoting,
 * Jastrow factors summed pair by pair.  Nothing is updated incrementally.
 *
 * Conventions (see the accompanying design notes for the readings taken
 * where the paper is silent):
 *   electrons 0..n_up-1 are spin up; proposal p = (3 i + d) * 2 + s moves
 *   electron i by +a (s = 0) or -a (s = 1) along axis d; with a non-local
 *   pseudopotential, proposal 6N + 6 i + q moves electron i to quadrature
 *   point q of the atom whose cutoff sphere holds it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* System description (mirrors the generator's arrays)                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int M;                    /* atoms */
    const double *R;          /* [M][3] */
    const double *Z;          /* [M] charge seen by electrons */
    const int32_t *core;      /* [M] 0 bare Coulomb, 1 softened core -Z/sqrt(r^2+rc^2) */
    const double *rc;         /* [M] */
    const int32_t *spec;      /* [M] species for e-n Jastrow */
    int Nb;
    const int32_t *batom;     /* [Nb] */
    const int32_t *btype;     /* [Nb] 0 s, 1-3 p, 4 Slater 1s */
    const double *bexp;       /* [Nb] */
    int Norb;
    const double *C;          /* [Nb][Norb] */
    int Nup, Ndn;
    int nspec;
    const double *jas;        /* [2+nspec][3] (A, B, b) */
    /* semi-local pseudopotential, non-local channels: term t belongs to atom
     * ecp_atom[t], channel l = ecp_l[t] (0, 1, 2) and contributes
     * ecp_coef[t] r^ecp_pow[t] exp(-ecp_exp[t] r^2) to v_l(r) of that atom
     * for r < ecp_rcut[atom]; necp = 0: no non-local part */
    int necp;
    const int32_t *ecp_atom;  /* [necp] */
    const int32_t *ecp_l;     /* [necp] */
    const int32_t *ecp_pow;   /* [necp] 0, 1 or 2 */
    const double *ecp_coef;   /* [necp] */
    const double *ecp_exp;    /* [necp] */
    const double *ecp_rcut;   /* [M] cutoff radius of each atom's channels, 0: none */
} orc_system;

typedef struct {
    double a;          /* lattice space */
    double tau;        /* conventional projection time between branchings */
    int nproj;         /* load-balanced steps between branchings */
    int nu_opt_mode;   /* 0: node test on electron i's own 6 proposals,
                          1: node test on any proposal, 2: nu_max always */
    uint64_t seed, sysid;
    double band;       /* relative width of the ambiguity band (1e-12) */
    int rotate;        /* 1: every walker's three lattice versors are rotated by a
                          random rotation drawn at the start of each projection
                          phase (App. D randomized lattice); 0: fixed x, y, z */
} orc_params;

enum { RNG_MOVE = 0, RNG_PERSIST = 1, RNG_COMB = 2, RNG_INIT = 3, RNG_ROTATE = 4 };

/* counters returned by the phase drivers */
enum {
    CNT_DECISIONS = 0, CNT_AMBIG_ADOPTED = 1, CNT_HARD_MISMATCH = 2,
    CNT_NODE_AMBIG = 3, CNT_NEG_WEIGHT = 4, CNT_NO_MOVE = 5, CNT_SINGULAR = 6,
    CNT_ITERS = 7, CNT_LEN = 8
};

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)                         */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in [0,1): top 53 bits of the first output word */
double orc_uniform(uint64_t seed, uint64_t sysid, uint64_t slot, uint64_t j,
                   uint64_t k, uint64_t purpose)
{
    uint64_t ctr[4] = {slot, j, k, purpose}, key[2] = {seed, sysid}, out[4];
    orc_philox4x64_10(ctr, key, out);
    return (double)(out[0] >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------ */
/* Random lattice orientation (App. D: the three versors of the discretized  */
/* Laplacian rotate with random angles along the simulation)                */
/* ------------------------------------------------------------------------ */
/* Rotation matrix R[x][d] (row-major 3x3; versor d is column d) of walker
 * slot `slot` for the projection phase after branching j.  A uniformly random
 * rotation is the rotation of a uniformly random unit quaternion; a point
 * uniform in the unit 4-ball has a uniformly random direction, so q = 2U - 1
 * componentwise (the four words of one Philox call with counter (slot, j,
 * attempt, ROTATE)) is accepted once 1e-3 <= |q|^2 <= 1, attempts 0..63
 * (identity if all are rejected, probability 0.69^64).  R is the textbook
 * rotation matrix of q divided by |q|^2; every sum and product is rounded on
 * its own, in the order written (no fused operations), so that another
 * implementation that evaluates the same expressions in the same order gets
 * the same bits. */
void orc_rotation(uint64_t seed, uint64_t sysid, uint64_t slot, uint64_t j, double R[9])
{
    for (uint64_t k = 0; k < 64; k++) {
        uint64_t ctr[4] = {slot, j, k, RNG_ROTATE}, key[2] = {seed, sysid}, out[4];
        orc_philox4x64_10(ctr, key, out);
        double q[4];
        for (int m = 0; m < 4; m++) q[m] = 2.0 * ((double)(out[m] >> 11) * 0x1.0p-53) - 1.0;
        double w = q[0], x = q[1], y = q[2], z = q[3];
        double ww = w * w, xx = x * x, yy = y * y, zz = z * z;
        double n = ((ww + xx) + yy) + zz;
        if (!(n <= 1.0 && n >= 1e-3)) continue;
        double xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
        R[0] = (((ww + xx) - yy) - zz) / n;
        R[1] = (2.0 * (xy - wz)) / n;
        R[2] = (2.0 * (xz + wy)) / n;
        R[3] = (2.0 * (xy + wz)) / n;
        R[4] = (((ww - xx) + yy) - zz) / n;
        R[5] = (2.0 * (yz - wx)) / n;
        R[6] = (2.0 * (xz - wy)) / n;
        R[7] = (2.0 * (yz + wx)) / n;
        R[8] = (((ww - xx) - yy) + zz) / n;
        return;
    }
    for (int m = 0; m < 9; m++) R[m] = (m % 4 == 0) ? 1.0 : 0.0;
}

/* Lattice step vectors st[d][x] = a * R[x][d] (each product rounded once);
 * R == NULL gives the fixed axes (a on the diagonal, zeros elsewhere). */
static void lattice_steps(const double *R, double a, double st[3][3])
{
    for (int d = 0; d < 3; d++)
        for (int x = 0; x < 3; x++)
            st[d][x] = R ? a * R[3 * x + d] : (x == d ? a : 0.0);
}

/* Proposal q (0..5 = +d0, -d0, +d1, -d1, +d2, -d2) of a point r: every
 * coordinate moved by one addition of the signed step vector (with fixed
 * axes the other two coordinates add zero and stay as they were). */
static void displaced(const double r[3], const double st[3][3], int q, double out[3])
{
    int d = q / 2, sg = q % 2;
    for (int x = 0; x < 3; x++) out[x] = r[x] + (sg ? -st[d][x] : st[d][x]);
}

/* ------------------------------------------------------------------------ */
/* Guiding function pieces                                                  */
/* ------------------------------------------------------------------------ */

/* Basis functions chi_mu at r; grad [Nb][3] and lap [Nb] optional. */
void orc_basis(const orc_system *s, const double r[3], double *val,
               double *grad, double *lap)
{
    for (int mu = 0; mu < s->Nb; mu++) {
        const double *Ra = s->R + 3 * s->batom[mu];
        double d[3] = {r[0] - Ra[0], r[1] - Ra[1], r[2] - Ra[2]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double al = s->bexp[mu];
        int t = s->btype[mu];
        if (t == 4) {                               /* exp(-zeta |r-R|) */
            double dd = sqrt(d2), g = exp(-al * dd);
            val[mu] = g;
            if (grad) for (int c = 0; c < 3; c++) grad[3 * mu + c] = -al * d[c] / dd * g;
            if (lap) lap[mu] = (al * al - 2.0 * al / dd) * g;
        } else if (t == 0) {                        /* exp(-alpha |r-R|^2) */
            double g = exp(-al * d2);
            val[mu] = g;
            if (grad) for (int c = 0; c < 3; c++) grad[3 * mu + c] = -2.0 * al * d[c] * g;
            if (lap) lap[mu] = (4.0 * al * al * d2 - 6.0 * al) * g;
        } else {                                    /* (x-X) exp(-alpha |r-R|^2) etc. */
            int q = t - 1;
            double g = exp(-al * d2);
            val[mu] = d[q] * g;
            if (grad)
                for (int c = 0; c < 3; c++)
                    grad[3 * mu + c] = ((c == q) ? g : 0.0) - 2.0 * al * d[q] * d[c] * g;
            if (lap) lap[mu] = d[q] * g * (4.0 * al * al * d2 - 10.0 * al);
        }
    }
}

/* Orbitals phi_k(r) = sum_mu C[mu][k] chi_mu(r), k < n. */
static void orbitals(const orc_system *s, const double *chi, int n, double *phi)
{
    for (int k = 0; k < n; k++) {
        double acc = 0.0;
        for (int mu = 0; mu < s->Nb; mu++) acc += s->C[mu * s->Norb + k] * chi[mu];
        phi[k] = acc;
    }
}

/* LU factorisation with partial pivoting of the n x n matrix A (row-major,
 * overwritten), returning log|det| and sign; inv (row-major) receives A^-1.
 * Returns 0 on success, -1 when a pivot is exactly zero. */
static int lu_inverse(int n, double *A, double *inv, double *logabs, double *sign)
{
    int *piv = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    double la = 0.0, sg = 1.0;
    for (int i = 0; i < n; i++) piv[i] = i;
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; i++)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        if (best == 0.0) { free(piv); return -1; }
        if (p != k) {
            for (int c = 0; c < n; c++) {
                double t = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = t;
            }
            int t = piv[k]; piv[k] = piv[p]; piv[p] = t;
            sg = -sg;
        }
        double d = A[k * n + k];
        if (d < 0) sg = -sg;
        la += log(fabs(d));
        for (int i = k + 1; i < n; i++) {
            double f = A[i * n + k] / d;
            A[i * n + k] = f;
            for (int c = k + 1; c < n; c++) A[i * n + c] -= f * A[k * n + c];
        }
    }
    /* solve A X = P^T I column by column */
    double *y = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int col = 0; col < n; col++) {
        for (int i = 0; i < n; i++) y[i] = (piv[i] == col) ? 1.0 : 0.0;
        for (int i = 0; i < n; i++)
            for (int c = 0; c < i; c++) y[i] -= A[i * n + c] * y[c];
        for (int i = n - 1; i >= 0; i--) {
            for (int c = i + 1; c < n; c++) y[i] -= A[i * n + c] * y[c];
            y[i] /= A[i * n + i];
        }
        for (int i = 0; i < n; i++) inv[i * n + col] = y[i];
    }
    free(y); free(piv);
    *logabs = la; *sign = sg;
    return 0;
}

/* Pade pair function u(r) = (A r + B r^2)/(1 + b r) and derivatives. */
static void pade(const double *p, double r, double *u, double *du, double *d2u)
{
    double A = p[0], B = p[1], b = p[2], den = 1.0 + b * r;
    *u = (A * r + B * r * r) / den;
    if (du) *du = (A + 2.0 * B * r + B * b * r * r) / (den * den);
    if (d2u) *d2u = 2.0 * (B - A * b) / (den * den * den);
}

static const double *ee_params(const orc_system *s, int i, int j)
{
    int si = i >= s->Nup, sj = j >= s->Nup;
    return s->jas + 3 * (si == sj ? 0 : 1);
}

/* Jastrow exponent J(x) = sum_{i<j} u_ee(r_ij) + sum_{i,I} u_en(|r_i - R_I|). */
double orc_jastrow(const orc_system *s, const double *pos)
{
    int N = s->Nup + s->Ndn;
    double J = 0.0, u;
    for (int i = 0; i < N; i++) {
        for (int j = i + 1; j < N; j++) {
            double dx = pos[3 * i] - pos[3 * j], dy = pos[3 * i + 1] - pos[3 * j + 1],
                   dz = pos[3 * i + 2] - pos[3 * j + 2];
            pade(ee_params(s, i, j), sqrt(dx * dx + dy * dy + dz * dz), &u, 0, 0);
            J += u;
        }
        for (int I = 0; I < s->M; I++) {
            const double *RI = s->R + 3 * I;
            double dx = pos[3 * i] - RI[0], dy = pos[3 * i + 1] - RI[1], dz = pos[3 * i + 2] - RI[2];
            pade(s->jas + 3 * (2 + s->spec[I]), sqrt(dx * dx + dy * dy + dz * dz), &u, 0, 0);
            J += u;
        }
    }
    return J;
}

/* Terms of J that involve electron i when it sits at r (other electrons at pos). */
static double jastrow_of(const orc_system *s, const double *pos, int i, const double r[3])
{
    int N = s->Nup + s->Ndn;
    double J = 0.0, u;
    for (int j = 0; j < N; j++) {
        if (j == i) continue;
        double dx = r[0] - pos[3 * j], dy = r[1] - pos[3 * j + 1], dz = r[2] - pos[3 * j + 2];
        pade(ee_params(s, i, j), sqrt(dx * dx + dy * dy + dz * dz), &u, 0, 0);
        J += u;
    }
    for (int I = 0; I < s->M; I++) {
        const double *RI = s->R + 3 * I;
        double dx = r[0] - RI[0], dy = r[1] - RI[1], dz = r[2] - RI[2];
        pade(s->jas + 3 * (2 + s->spec[I]), sqrt(dx * dx + dy * dy + dz * dz), &u, 0, 0);
        J += u;
    }
    return J;
}

/* grad_i J and lap_i J */
static void jastrow_derivs(const orc_system *s, const double *pos, int i, double g[3], double *l)
{
    int N = s->Nup + s->Ndn;
    double u, du, d2u;
    g[0] = g[1] = g[2] = 0.0; *l = 0.0;
    for (int j = 0; j < N + s->M; j++) {
        if (j == i) continue;
        const double *q; const double *prm;
        if (j < N) { q = pos + 3 * j; prm = ee_params(s, i, j); }
        else { q = s->R + 3 * (j - N); prm = s->jas + 3 * (2 + s->spec[j - N]); }
        double d[3] = {pos[3 * i] - q[0], pos[3 * i + 1] - q[1], pos[3 * i + 2] - q[2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        pade(prm, r, &u, &du, &d2u);
        for (int c = 0; c < 3; c++) g[c] += du * d[c] / r;
        *l += d2u + 2.0 * du / r;
    }
}

/* Electron-nucleus potential nu_ei(r) and its lattice bound nu^a_ei(r). */
static void nuclear_potential(const orc_system *s, const double r[3], double a,
                              double *nu, double *nua)
{
    double v = 0.0, va = 0.0;
    for (int I = 0; I < s->M; I++) {
        const double *RI = s->R + 3 * I;
        double dx = r[0] - RI[0], dy = r[1] - RI[1], dz = r[2] - RI[2];
        double d = sqrt(dx * dx + dy * dy + dz * dz);
        if (s->core[I] == 0) {
            v += -s->Z[I] / d;
            va += -s->Z[I] / (d > a ? d : a);
        } else {
            double t = -s->Z[I] / sqrt(d * d + s->rc[I] * s->rc[I]);
            v += t; va += t;
        }
    }
    *nu = v; *nua = va;
}

static double ion_ion(const orc_system *s)
{
    double v = 0.0;
    for (int I = 0; I < s->M; I++)
        for (int J = I + 1; J < s->M; J++) {
            const double *A = s->R + 3 * I, *B = s->R + 3 * J;
            double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
            v += s->Z[I] * s->Z[J] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return v;
}

/* ------------------------------------------------------------------------ */
/* Non-local pseudopotential under the determinant locality approximation   */
/* (App. D: the non-local elements V^nl_{x',x} of the FN Hamiltonian, with  */
/* the guiding-function ratio replaced by the determinant ratio D(x')/D(x))  */
/* ------------------------------------------------------------------------ */
/* The semi-local operator sum_l v_l(r) sum_m |lm><lm| of atom I acting on
 * electron i is applied with the 6-point octahedral quadrature of the sphere
 * of radius r = |r_i - R_I| around R_I: points R_I +- r u_d (u_d the walker's
 * lattice versors, column d of its rotation; the coordinate axes without
 * one), weights 1/6, exact for spherical harmonics of degree <= 3.  Point q
 * (0..5 = +u0, -u0, +u1, -u1, +u2, -u2) is the configuration x' with electron
 * i moved there, and its element is
 *   V_q = sum_l (2l + 1)/6 v_l(r) P_l(cos theta_q),
 * theta_q the angle between r_i - R_I and the point's direction. */

/* distance of r from atom I, each product and sum rounded in the order written */
static double atom_distance(const orc_system *s, int I, const double r[3], double dv[3])
{
    const double *RI = s->R + 3 * I;
    dv[0] = r[0] - RI[0]; dv[1] = r[1] - RI[1]; dv[2] = r[2] - RI[2];
    return sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
}

/* the atom whose cutoff sphere holds r (the spheres do not overlap), or -1 */
static int nl_atom(const orc_system *s, const double r[3])
{
    for (int I = 0; I < s->M; I++) {
        double rc = s->ecp_rcut ? s->ecp_rcut[I] : 0.0, dv[3];
        if (rc > 0 && atom_distance(s, I, r, dv) < rc) return I;
    }
    return -1;
}

/* quadrature point q of the sphere of radius r around atom I */
static void nl_point(const orc_system *s, int I, double r, const double *rot, int q,
                     double out[3])
{
    const double *RI = s->R + 3 * I;
    int d = q / 2, sg = q % 2;
    for (int x = 0; x < 3; x++) {
        double u = rot ? rot[3 * x + d] : (x == d ? 1.0 : 0.0);
        double t = r * u;
        out[x] = RI[x] + (sg ? -t : t);
    }
}

/* V_q from the channels of atom I at distance r and cos theta_q */
static double nl_element(const orc_system *s, int I, double r, double cth)
{
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < s->necp; t++) {
        if (s->ecp_atom[t] != I) continue;
        double rp = s->ecp_pow[t] == 0 ? 1.0 : (s->ecp_pow[t] == 1 ? r : r * r);
        v[s->ecp_l[t]] += s->ecp_coef[t] * rp * exp(-s->ecp_exp[t] * r * r);
    }
    double P1 = cth, P2 = 0.5 * (3.0 * cth * cth - 1.0);
    return (v[0] + 3.0 * v[1] * P1 + 5.0 * v[2] * P2) / 6.0;
}

/* log|Psi_G| and sign, by LU determinants and the Jastrow sum.  Returns 0 or
 * -1 for a singular Slater matrix. */
int orc_log_psi(const orc_system *s, const double *pos, double *logabs, double *sign)
{
    int ns[2] = {s->Nup, s->Ndn}, off[2] = {0, s->Nup};
    double la = 0.0, sg = 1.0;
    double *chi = (double *)malloc(sizeof(double) * s->Nb);
    for (int sp = 0; sp < 2; sp++) {
        int n = ns[sp];
        if (!n) continue;
        double *A = (double *)malloc(sizeof(double) * n * n);
        double *inv = (double *)malloc(sizeof(double) * n * n);
        for (int c = 0; c < n; c++) {
            orc_basis(s, pos + 3 * (off[sp] + c), chi, 0, 0);
            orbitals(s, chi, n, A + c * n);
        }
        double l1, s1;
        int rc = lu_inverse(n, A, inv, &l1, &s1);
        free(A); free(inv);
        if (rc) { free(chi); return -1; }
        la += l1; sg *= s1;
    }
    free(chi);
    *logabs = la + orc_jastrow(s, pos);
    *sign = sg;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-configuration evaluation (lattice-regularized FN Hamiltonian, App. D;  */
/* load-balanced split, Sec. II.C)                                           */
/* ------------------------------------------------------------------------ */
enum {
    SC_BBAR = 0, SC_VSF, SC_W, SC_EL, SC_ELCONT, SC_VEE, SC_VII, SC_LOGABS,
    SC_SIGN, SC_MINREL, SC_VNL, SC_LEN = 16
};

/* Outputs (any pointer may be NULL except scal); PT = 6N, or 12N with a
 * non-local pseudopotential:
 *   R[PT]    Psi_G(x')/Psi_G(x) for every lattice move, then
 *            -2 a^2 V_q D(x')/D(x) for every non-local proposal
 *   Rdet[PT] determinant part of the ratio, dJ[PT] Jastrow exponent change
 *            (0 for the non-local proposals)
 *   lap[N]   continuum lap_i Psi_G / Psi_G
 *   grad[N][3] grad_i Psi_G / Psi_G
 *   nu_zv[N], nu_opt[N], node[N]
 *   scal[SC_LEN]: bbar, V_sf, W, e_L, e_L(continuum), V_ee, V_ii, log|Psi|,
 *                 sign, min |R_p| / max |R_p| over the lattice moves,
 *                 non-local energy sum_{i,q} V_q D(x')/D(x)
 * Returns 0, or -1 for a singular Slater matrix. */
int orc_eval_rot(const orc_system *s, const orc_params *prm, const double *rot,
                 const double *pos, double *R, double *Rdet, double *dJ, double *lap,
                 double *grad, double *nu_zv, double *nu_opt, int32_t *node, double *scal)
{
    const int N = s->Nup + s->Ndn, P = 6 * N, PT = s->necp ? 12 * N : P, Nb = s->Nb;
    const double a = prm->a;
    double st[3][3];
    lattice_steps(rot, a, st);
    int ns[2] = {s->Nup, s->Ndn}, off[2] = {0, s->Nup};
    double *Ainv[2] = {0, 0};
    double logabs = 0.0, sign = 1.0;
    double *chi = (double *)malloc(sizeof(double) * Nb);
    double *chig = (double *)malloc(sizeof(double) * Nb * 3);
    double *chil = (double *)malloc(sizeof(double) * Nb);
    double *phi = (double *)malloc(sizeof(double) * (s->Norb + 1));
    double *Rl = (double *)malloc(sizeof(double) * PT);
    int *nlneg = (int *)calloc(N, sizeof(int));
    double *lapl = (double *)malloc(sizeof(double) * N);
    double *nuzv = (double *)malloc(sizeof(double) * N);
    double *nuop = (double *)malloc(sizeof(double) * N);
    int rc = 0;

    /* Slater matrices A_sigma[c][k] = phi_k(r_{off+c}) and their inverses */
    for (int sp = 0; sp < 2; sp++) {
        int n = ns[sp];
        if (!n) continue;
        double *A = (double *)malloc(sizeof(double) * n * n);
        Ainv[sp] = (double *)malloc(sizeof(double) * n * n);
        for (int c = 0; c < n; c++) {
            orc_basis(s, pos + 3 * (off[sp] + c), chi, 0, 0);
            orbitals(s, chi, n, A + c * n);
        }
        double l1, s1;
        if (lu_inverse(n, A, Ainv[sp], &l1, &s1)) rc = -1;
        logabs += l1; sign *= s1;
        free(A);
    }
    if (rc) goto done;
    logabs += orc_jastrow(s, pos);

    /* ratios for all 6N single-electron lattice moves */
    for (int i = 0; i < N; i++) {
        int sp = i >= s->Nup, n = ns[sp], c = i - off[sp];
        double J0 = jastrow_of(s, pos, i, pos + 3 * i);
        for (int d = 0; d < 3; d++)
            for (int sg = 0; sg < 2; sg++) {
                int p = (3 * i + d) * 2 + sg;
                double r[3];
                displaced(pos + 3 * i, st, 2 * d + sg, r);
                orc_basis(s, r, chi, 0, 0);
                orbitals(s, chi, n, phi);
                double rd = 0.0;   /* det(A with row c -> phi(r'))/det(A) = phi . Ainv[:,c] */
                for (int k = 0; k < n; k++) rd += phi[k] * Ainv[sp][k * n + c];
                double dj = jastrow_of(s, pos, i, r) - J0;
                Rl[p] = rd * exp(dj);
                if (Rdet) Rdet[p] = rd;
                if (dJ) dJ[p] = dj;
            }
    }

    /* non-local proposals (DLA): electron i moved to quadrature point q of the
     * atom whose sphere holds it, entry -2 a^2 V_q D(x')/D(x) in the units of
     * the kinetic ratios (a kinetic move weighs R_p / (2 a^2)); slots of
     * electrons outside every sphere hold 0 */
    double vnl = 0.0;
    for (int i = 0; i < N && PT > P; i++) {
        int sp = i >= s->Nup, n = ns[sp], c = i - off[sp];
        for (int q = 0; q < 6; q++) {
            Rl[P + 6 * i + q] = 0.0;
            if (Rdet) Rdet[P + 6 * i + q] = 0.0;
            if (dJ) dJ[P + 6 * i + q] = 0.0;
        }
        int I = nl_atom(s, pos + 3 * i);
        if (I < 0) continue;
        double dv[3];
        double r = atom_distance(s, I, pos + 3 * i, dv);
        for (int q = 0; q < 6; q++) {
            int d = q / 2;
            double xq[3];
            nl_point(s, I, r, rot, q, xq);
            orc_basis(s, xq, chi, 0, 0);
            orbitals(s, chi, n, phi);
            double rd = 0.0;
            for (int k = 0; k < n; k++) rd += phi[k] * Ainv[sp][k * n + c];
            double ud = rot ? dv[0] * rot[d] + dv[1] * rot[3 + d] + dv[2] * rot[6 + d] : dv[d];
            double cth = (q % 2 ? -ud : ud) / r;
            double V = nl_element(s, I, r, cth);
            Rl[P + 6 * i + q] = -2.0 * a * a * V * rd;
            if (Rdet) Rdet[P + 6 * i + q] = rd;
            vnl += V * rd;
            if (rd < 0) nlneg[i] = 1;
        }
    }

    /* continuum local energy pieces */
    double vee = 0.0, vii = ion_ion(s), elc = 0.0;
    for (int i = 0; i < N; i++)
        for (int j = i + 1; j < N; j++) {
            double dx = pos[3 * i] - pos[3 * j], dy = pos[3 * i + 1] - pos[3 * j + 1],
                   dz = pos[3 * i + 2] - pos[3 * j + 2];
            vee += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        }
    double *nua = (double *)malloc(sizeof(double) * N);
    double *nue = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; i++) {
        int sp = i >= s->Nup, n = ns[sp], c = i - off[sp];
        orc_basis(s, pos + 3 * i, chi, chig, chil);
        double gD[3] = {0, 0, 0}, lD = 0.0;
        for (int k = 0; k < n; k++) {
            double g0 = 0, g1 = 0, g2 = 0, l = 0;
            for (int mu = 0; mu < Nb; mu++) {
                double cm = s->C[mu * s->Norb + k];
                g0 += cm * chig[3 * mu]; g1 += cm * chig[3 * mu + 1]; g2 += cm * chig[3 * mu + 2];
                l += cm * chil[mu];
            }
            double w = Ainv[sp][k * n + c];
            gD[0] += g0 * w; gD[1] += g1 * w; gD[2] += g2 * w; lD += l * w;
        }
        double gJ[3], lJ;
        jastrow_derivs(s, pos, i, gJ, &lJ);
        lapl[i] = lD + 2.0 * (gD[0] * gJ[0] + gD[1] * gJ[1] + gD[2] * gJ[2]) + lJ +
                  gJ[0] * gJ[0] + gJ[1] * gJ[1] + gJ[2] * gJ[2];
        if (grad) for (int q = 0; q < 3; q++) grad[3 * i + q] = gD[q] + gJ[q];
        nuclear_potential(s, pos + 3 * i, a, &nue[i], &nua[i]);
        elc += -0.5 * lapl[i] + nue[i];
    }
    elc += vee + vii + vnl;

    /* lattice terms with the fixed-node spin-flip contributions (App. D) */
    double bsum = 0.0, vsum = 0.0, maxabs = 0.0, minabs = INFINITY;
    int anynode = 0;
    for (int p = 0; p < PT; p++) {
        if (Rl[p] > 0) bsum += Rl[p];
        else if (Rl[p] < 0) vsum += -Rl[p];
        if (p >= P) continue;
        if (Rl[p] < 0) anynode = 1;
        double m = fabs(Rl[p]);
        if (m > maxabs) maxabs = m;
        if (m < minabs) minabs = m;
    }
    /* a non-local proposal crosses the node when its determinant ratio is
     * negative (the Jastrow factor is positive) */
    for (int i = 0; i < N; i++) if (nlneg[i]) anynode = 1;
    double inv2a2 = 1.0 / (2.0 * a * a);
    double bbar = bsum * inv2a2, vsf = vsum * inv2a2;
    double sum_opt = 0.0;
    for (int i = 0; i < N; i++) {
        double lapA = 0.0;
        int nd = 0;
        for (int q = 0; q < 6; q++) {
            double r = Rl[6 * i + q];
            lapA += (r - 1.0) / (a * a);
            if (r < 0) nd = 1;
        }
        if (nlneg[i]) nd = 1;
        if (prm->nu_opt_mode == 1) nd = anynode;
        if (prm->nu_opt_mode == 2) nd = 1;
        nuzv[i] = nue[i] + 0.5 * (lapA - lapl[i]);
        double numax = nuzv[i] > nua[i] ? nuzv[i] : nua[i];
        nuop[i] = nd ? numax : nuzv[i];
        sum_opt += nuop[i];
        if (node) node[i] = nd;
    }
    double W = 3.0 * N / (a * a) + sum_opt + vee + vsf + vii;
    double eL = W - bbar;

    if (R) memcpy(R, Rl, sizeof(double) * PT);
    if (lap) memcpy(lap, lapl, sizeof(double) * N);
    if (nu_zv) memcpy(nu_zv, nuzv, sizeof(double) * N);
    if (nu_opt) memcpy(nu_opt, nuop, sizeof(double) * N);
    for (int q = 0; q < SC_LEN; q++) scal[q] = 0.0;
    scal[SC_BBAR] = bbar; scal[SC_VSF] = vsf; scal[SC_W] = W; scal[SC_EL] = eL;
    scal[SC_ELCONT] = elc; scal[SC_VEE] = vee; scal[SC_VII] = vii;
    scal[SC_LOGABS] = logabs; scal[SC_SIGN] = sign;
    scal[SC_MINREL] = maxabs > 0 ? minabs / maxabs : 0.0;
    scal[SC_VNL] = vnl;
    free(nua); free(nue);
done:
    free(Ainv[0]); free(Ainv[1]);
    free(chi); free(chig); free(chil); free(phi); free(Rl); free(nlneg); free(lapl); free(nuzv);
    free(nuop);
    return rc;
}

/* orc_eval_rot with the fixed lattice axes */
int orc_eval(const orc_system *s, const orc_params *prm, const double *pos,
             double *R, double *Rdet, double *dJ, double *lap, double *grad,
             double *nu_zv, double *nu_opt, int32_t *node, double *scal)
{
    return orc_eval_rot(s, prm, 0, pos, R, Rdet, dJ, lap, grad, nu_zv, nu_opt, node, scal);
}

/* ------------------------------------------------------------------------ */
/* Heat-bath choice among the proposals, p_{x',x} of the load-balanced split */
/* (Sec. II.C) and of Algorithm 1's move line                                */
/* ------------------------------------------------------------------------ */
/* returns the chosen proposal (or -1 if no move has positive weight) and the
 * distance of the threshold to the nearest cumulative boundary, relative to
 * the total. */
static int heat_bath(int P, const double *R, double xi, double *margin)
{
    double tot = 0.0;
    for (int p = 0; p < P; p++) if (R[p] > 0) tot += R[p];
    if (!(tot > 0)) { *margin = INFINITY; return -1; }
    double t = xi * tot, c = 0.0, m = INFINITY;
    int pick = -1, last = -1;
    for (int p = 0; p < P; p++) {
        if (R[p] > 0) {
            c += R[p];
            last = p;
            double g = fabs(c - t);
            if (g < m) m = g;
            if (pick < 0 && c > t) pick = p;
        }
    }
    if (pick < 0) pick = last;
    *margin = m / tot;
    return pick;
}

/* (for the parity harness) whether the choice q is consistent with xi up to
 * the band: the threshold lies within band*total of q's cumulative interval */
static int choice_within_band(int P, const double *R, double xi, int q, double band)
{
    if (q < 0 || q >= P || !(R[q] > 0)) return 0;
    double tot = 0.0;
    for (int p = 0; p < P; p++) if (R[p] > 0) tot += R[p];
    double t = xi * tot, lo = 0.0;
    for (int p = 0; p < q; p++) if (R[p] > 0) lo += R[p];
    double hi = lo + R[q];
    return (t >= lo - band * tot) && (t < hi + band * tot);
}

/* Move p: a lattice move (p < 6N) or a non-local move (p = 6N + 6i + q:
 * electron i to quadrature point q of the atom whose sphere holds it). */
static void apply_move(const orc_system *s, double *pos, int p, const double *rot, double a)
{
    const int N = s->Nup + s->Ndn;
    double st[3][3], r[3];
    if (p >= 6 * N) {
        int i = (p - 6 * N) / 6, I = nl_atom(s, pos + 3 * i);
        double dv[3];
        double rr = atom_distance(s, I, pos + 3 * i, dv);
        nl_point(s, I, rr, rot, (p - 6 * N) % 6, r);
        for (int x = 0; x < 3; x++) pos[3 * i + x] = r[x];
        return;
    }
    lattice_steps(rot, a, st);
    int i = p / 6;
    displaced(pos + 3 * i, st, p % 6, r);
    for (int x = 0; x < 3; x++) pos[3 * i + x] = r[x];
}

/* ------------------------------------------------------------------------ */
/* Load-balanced projection phase for one walker (Algorithm 2)                */
/* ------------------------------------------------------------------------ */
/* Runs nproj steps: evaluate at x, w <- w * bbar/(W - E0), move by p_{x',x}.
 * After the last move the estimator values e_L, W at the final x are
 * returned.  follow (optional, [nproj]) holds another implementation's
 * choices: where they differ only inside the ambiguity band the oracle adopts
 * them and counts it; otherwise a hard mismatch is counted (and adopted, so
 * the rest of the comparison stays meaningful).  moves_out [nproj] optional. */
int orc_lb_phase(const orc_system *s, const orc_params *prm, uint64_t slot, uint64_t j,
                 double E0, double *pos, double *lw, double *eL_out, double *W_out,
                 const int32_t *follow, int32_t *moves_out, int64_t *cnt)
{
    const int N = s->Nup + s->Ndn, P = s->necp ? 12 * N : 6 * N;
    double *R = (double *)malloc(sizeof(double) * P);
    double sc[SC_LEN], rotm[9];
    const double *rot = 0;
    if (prm->rotate) { orc_rotation(prm->seed, prm->sysid, slot, j, rotm); rot = rotm; }
    int rc = 0;
    for (int k = 0; k < prm->nproj; k++) {
        if (orc_eval_rot(s, prm, rot, pos, R, 0, 0, 0, 0, 0, 0, 0, sc)) { cnt[CNT_SINGULAR]++; rc = -1; break; }
        if (sc[SC_MINREL] <= prm->band) cnt[CNT_NODE_AMBIG]++;
        double bbar = sc[SC_BBAR], W = sc[SC_W];
        if (!(W - E0 > 0)) { cnt[CNT_NEG_WEIGHT]++; *lw = -INFINITY; }
        else if (!(bbar > 0)) { cnt[CNT_NO_MOVE]++; *lw = -INFINITY; }
        else *lw += log(bbar) - log(W - E0);
        double xi = orc_uniform(prm->seed, prm->sysid, slot, j, (uint64_t)k, RNG_MOVE);
        double margin;
        int q = heat_bath(P, R, xi, &margin);
        cnt[CNT_DECISIONS]++;
        if (follow && follow[k] != q) {
            if (margin <= prm->band && choice_within_band(P, R, xi, follow[k], prm->band))
                cnt[CNT_AMBIG_ADOPTED]++;
            else
                cnt[CNT_HARD_MISMATCH]++;
            q = follow[k];
        }
        if (moves_out) moves_out[k] = q;
        if (q >= 0) apply_move(s, pos, q, rot, prm->a);
    }
    if (!rc) {
        if (orc_eval_rot(s, prm, rot, pos, 0, 0, 0, 0, 0, 0, 0, 0, sc)) { cnt[CNT_SINGULAR]++; rc = -1; }
        else {
            *eL_out = sc[SC_EL]; *W_out = sc[SC_W];
            /* Sec. II.C: the walker average weights w by 1/(W - E_0) at the
             * final configuration, which needs W - E_0 > 0 there as well; a
             * walker violating it gets weight zero, like any step's factor */
            if (prm->nproj > 0 && !(sc[SC_W] - E0 > 0)) { cnt[CNT_NEG_WEIGHT]++; *lw = -INFINITY; }
        }
    }
    free(R);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Conventional continuous-time projection for one walker (Algorithm 1)       */
/* ------------------------------------------------------------------------ */
/* Each iteration: evaluate at x; tau_xi = min(-log(1-xi)/bbar, tau_left);
 * w <- w exp(-tau_xi e_L(x)); tau_left -= tau_xi; stop when tau_left = 0,
 * else move by p_{x',x}.  moves_out [cap]: proposal of each iteration, -1 for
 * the final (stopping) iteration.  follow [cap] likewise, from another
 * implementation.  Returns the iteration count in *n_iter. */
int orc_conv_phase(const orc_system *s, const orc_params *prm, uint64_t slot, uint64_t j,
                   double *pos, double *lw, double *eL_out, double *W_out,
                   const int32_t *follow, int32_t *moves_out, int cap, int *n_iter,
                   int64_t *cnt)
{
    const int N = s->Nup + s->Ndn, P = s->necp ? 12 * N : 6 * N;
    double *R = (double *)malloc(sizeof(double) * P);
    double sc[SC_LEN], rotm[9];
    const double *rot = 0;
    if (prm->rotate) { orc_rotation(prm->seed, prm->sysid, slot, j, rotm); rot = rotm; }
    double tau_left = prm->tau;
    int it = 0, rc = 0;
    for (;;) {
        if (orc_eval_rot(s, prm, rot, pos, R, 0, 0, 0, 0, 0, 0, 0, sc)) { cnt[CNT_SINGULAR]++; rc = -1; break; }
        if (sc[SC_MINREL] <= prm->band) cnt[CNT_NODE_AMBIG]++;
        double bbar = sc[SC_BBAR], eL = sc[SC_EL];
        double xt = orc_uniform(prm->seed, prm->sysid, slot, j, (uint64_t)it, RNG_PERSIST);
        double t = (bbar > 0) ? -log1p(-xt) / bbar : INFINITY;
        if (!(bbar > 0)) cnt[CNT_NO_MOVE]++;
        int stop = !(t < tau_left);
        cnt[CNT_DECISIONS]++;
        if (follow && it < cap) {
            int fstop = follow[it] < 0;
            if (fstop != stop) {
                if (fabs(t - tau_left) <= prm->band * prm->tau) cnt[CNT_AMBIG_ADOPTED]++;
                else cnt[CNT_HARD_MISMATCH]++;
                stop = fstop;
            }
        }
        double tx = stop ? tau_left : t;
        *lw -= tx * eL;
        tau_left = stop ? 0.0 : tau_left - tx;
        *eL_out = eL; *W_out = sc[SC_W];
        it++;
        if (stop) { if (moves_out && it - 1 < cap) moves_out[it - 1] = -1; break; }
        double xi = orc_uniform(prm->seed, prm->sysid, slot, j, (uint64_t)(it - 1), RNG_MOVE);
        double margin;
        int q = heat_bath(P, R, xi, &margin);
        cnt[CNT_DECISIONS]++;
        if (follow && it - 1 < cap && follow[it - 1] >= 0 && follow[it - 1] != q) {
            if (margin <= prm->band && choice_within_band(P, R, xi, follow[it - 1], prm->band))
                cnt[CNT_AMBIG_ADOPTED]++;
            else
                cnt[CNT_HARD_MISMATCH]++;
            q = follow[it - 1];
        }
        if (moves_out && it - 1 < cap) moves_out[it - 1] = q;
        if (q >= 0) apply_move(s, pos, q, rot, prm->a);
    }
    *n_iter = it;
    cnt[CNT_ITERS] += it;
    free(R);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Reconfiguration with N_w correlated numbers Z_alpha = (xi + alpha - 1)/N_w */
/* (Sec. II.A, branching equations)                                          */
/* ------------------------------------------------------------------------ */
/* sel[alpha] = min{beta : C_beta > (xi + alpha) * C_N / N_w} (0-based alpha),
 * C the inclusive running sum of exp(lw - max lw) in slot order.
 * out[0] = log of the average weight, out[1] = max lw, out[2] = C_N.
 * follow (optional) adopts another implementation's selections when they
 * differ only inside the band.  Returns -1 if every weight is zero. */
int orc_comb(int nw, const double *lw, double xi, int32_t *sel, double *out,
             const int32_t *follow, double band, int64_t *cnt)
{
    double mx = -INFINITY;
    for (int b = 0; b < nw; b++) if (lw[b] > mx) mx = lw[b];
    if (!(mx > -INFINITY)) return -1;
    double *C = (double *)malloc(sizeof(double) * nw);
    double c = 0.0;
    for (int b = 0; b < nw; b++) { c += exp(lw[b] - mx); C[b] = c; }
    double tot = C[nw - 1];
    int beta = 0, lastpos = 0;
    for (int b = 0; b < nw; b++) if (lw[b] > -INFINITY) lastpos = b;
    for (int al = 0; al < nw; al++) {
        double target = (xi + (double)al) * tot / (double)nw;
        while (beta < nw && !(C[beta] > target)) beta++;
        int pick = beta < nw ? beta : lastpos;
        if (beta >= nw) beta = nw - 1;
        if (cnt) cnt[CNT_DECISIONS]++;
        if (follow && follow[al] != pick) {
            int f = follow[al];
            double lo = (f > 0) ? C[f - 1] : 0.0, hi = (f >= 0 && f < nw) ? C[f] : -1.0;
            int ok = (f >= 0 && f < nw) && target >= lo - band * tot && target < hi + band * tot &&
                     (fabs(target - lo) <= band * tot || fabs(target - hi) <= band * tot);
            if (cnt) cnt[ok ? CNT_AMBIG_ADOPTED : CNT_HARD_MISMATCH]++;
            pick = f;
        }
        sel[al] = pick;
    }
    out[0] = log(tot / (double)nw) + mx;
    out[1] = mx;
    out[2] = tot;
    free(C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole-population phase, std threads over walkers                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_system *s; const orc_params *prm;
    int scheme, j, w0, w1, cap;
    double E0;
    double *pos, *lw, *eL, *W;
    const int32_t *follow; int32_t *moves; int32_t *iters;
    uint64_t slot0; const int64_t *slots;
    int64_t cnt[CNT_LEN];
    int rc;
} orc_job;

static void *phase_worker(void *arg)
{
    orc_job *jb = (orc_job *)arg;
    const int N = jb->s->Nup + jb->s->Ndn;
    const int stride = jb->scheme == 0 ? jb->prm->nproj : jb->cap;
    for (int w = jb->w0; w < jb->w1; w++) {
        const int32_t *f = jb->follow ? jb->follow + (size_t)w * stride : 0;
        int32_t *m = jb->moves ? jb->moves + (size_t)w * stride : 0;
        uint64_t slot = jb->slots ? (uint64_t)jb->slots[w] : jb->slot0 + w;
        int rc;
        if (jb->scheme == 0) {
            rc = orc_lb_phase(jb->s, jb->prm, slot, jb->j, jb->E0, jb->pos + (size_t)w * 3 * N,
                              jb->lw + w, jb->eL + w, jb->W + w, f, m, jb->cnt);
            if (jb->iters) jb->iters[w] = jb->prm->nproj;
        } else {
            int it = 0;
            rc = orc_conv_phase(jb->s, jb->prm, slot, jb->j, jb->pos + (size_t)w * 3 * N,
                                jb->lw + w, jb->eL + w, jb->W + w, f, m, jb->cap, &it, jb->cnt);
            if (jb->iters) jb->iters[w] = it;
        }
        if (rc) jb->rc = rc;
    }
    return 0;
}

/* scheme 0 = load-balanced, 1 = conventional.  Walker w uses Philox slot
 * slots[w] when slots is given, else slot0 + w.  follow/moves are [nw][stride] with stride nproj (LB) or cap
 * (conventional).  cnt_out[CNT_LEN] accumulates the counters. */
int orc_population_phase(const orc_system *s, const orc_params *prm, int scheme, int nw,
                         uint64_t slot0, int j, double E0, double *pos, double *lw,
                         double *eL, double *W, const int32_t *follow, int32_t *moves,
                         int cap, int32_t *iters, int nthreads, int64_t *cnt_out,
                         const int64_t *slots)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nw) nthreads = nw > 0 ? nw : 1;
    orc_job *jobs = (orc_job *)calloc(nthreads, sizeof(orc_job));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; t++) {
        orc_job *jb = &jobs[t];
        jb->s = s; jb->prm = prm; jb->scheme = scheme; jb->j = j; jb->cap = cap;
        jb->w0 = (int)((long)nw * t / nthreads); jb->w1 = (int)((long)nw * (t + 1) / nthreads);
        jb->E0 = E0; jb->pos = pos; jb->lw = lw; jb->eL = eL; jb->W = W;
        jb->follow = follow; jb->moves = moves; jb->iters = iters; jb->slot0 = slot0;
        jb->slots = slots;
        pthread_create(&th[t], 0, phase_worker, jb);
    }
    int rc = 0;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], 0);
        for (int q = 0; q < CNT_LEN; q++) cnt_out[q] += jobs[t].cnt[q];
        if (jobs[t].rc) rc = jobs[t].rc;
    }
    free(jobs); free(th);
    return rc;
}
