// Device-side descriptors shared by the host orchestration and the kernels of
// the lattice-regularized DMC library.  Everything here is plain data: the
// host fills these structs and passes them by value as kernel arguments.
#pragma once
#include <stdint.h>

namespace lrdmc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxBranchBlock = 1024;

enum : int { kMove = 0, kPersist = 1, kComb = 2, kInit = 3 };   // Philox purposes

// counters accumulated by one projection phase (device, 64-bit)
enum : int {
    kCntIters = 0, kCntNegW = 1, kCntNoMove = 2, kCntRefresh = 3, kCntSmallR = 4,
    kCntSingular = 5, kCntMaxIters = 6, kCntMinIters = 7, kCntCapped = 8,
    kCntNonfinite = 9,   // walkers ending a phase with a NaN or infinite e_L or W, or a
                         // NaN or +inf log-weight (-inf marks a dead walker)
    kCntLen = 10
};

// One molecular system, its walkers, and the per-walker state layout.
struct DevSys {
    // sizes
    int M, Nb, Norb, Nup, Ndn, N, P, ns, nspec, nw, has_en;
    double vii;              // ion-ion repulsion (host-computed constant)
    uint64_t sysid;
    const int *jp;           // branching index (Philox counter word 1), device
    const double *e0p;       // E_0 of this system, device
    // system arrays (device)
    const double *R, *Z, *rc, *bexp, *C, *jas;
    const double *btab;      // [Nb][4]: centre x, y, z and exponent of each basis function
    const double *bK;        // [Nb]: exp(-alpha a^2), the Gaussian factor of one lattice step
    const int32_t *core, *spec, *batom, *btype;
    // walker arrays (device)
    double *pos;             // [nw][N][3]
    double *lw, *eL, *Wd;    // [nw]
    double *spill;           // [nw][spill_stride]: orbital rows at the moves [PT][ns],
                             // orbital derivatives at the current positions [4N][ns] and,
                             // for the large-system kernel, the Slater rows [N][ns]
    long spill_stride;
    int32_t *iters;          // [nw]
    int32_t *trace;          // [nw][trace_cap] or null
    int trace_cap;
    // LDS layout of one walker (offsets in doubles)
    int ldb;                 // row stride (doubles) of the basis block: Nb padded to 4 mod 16
                             // so that the 16 rows of an MFMA operand read fall in distinct banks
    int o_pos, o_R, o_Rdet, o_dJ, o_Arow, o_AinvT, o_Jg, o_Jl, o_nue, o_nua, o_dje,
        o_scal, o_B, o_rows, o_tmp, o_C, o_nuc, o_jas, o_gd, o_ev, lds_doubles;
    // spill layout (offsets in doubles inside a walker's spill block)
    int s_Phi, s_dPhi;
    // systems too large for the LDS-resident layout (the large-system kernel):
    // the Slater rows [N][ns] in the spill block at s_Arow (0 otherwise), and
    // the basis functions per chunk of the orbital product (all, or 64)
    int s_Arow;
    int bchunk;
    // large-system layout with one spin's inverse in LDS (ainv1 = 1): both
    // inverses [2][ns][ns] at s_AinvG and the refresh's left half [ns][ns] at
    // s_GJ in the spill block; the moved spin's inverse is staged into LDS
    int ainv1;
    long s_AinvG, s_GJ;
    // non-local pseudopotential (App. D non-local elements, determinant
    // locality approximation): term t adds ecp_coef r^ecp_pow exp(-ecp_exp r^2)
    // to channel ecp_l of atom ecp_atom, inside radius ecp_rcut of that atom.
    // PT: proposals per configuration, the 6N lattice moves and, with a
    // pseudopotential, 6N quadrature points (zero entries for electrons outside
    // every sphere); PT is also the number of spilled orbital rows.
    int PT, necp;
    const int32_t *ecp_atom, *ecp_l, *ecp_pow;
    const double *ecp_coef, *ecp_exp, *ecp_rcut;
    int o_Vnl;               // LDS [6N]: element V_q of each quadrature point
    int o_nlin;              // LDS [N]: 1 for an electron inside a sphere, else 0
};

// Nucleus record staged in LDS per walker by the FP64 phase kernel: x, y, z,
// charge, core radius, soft-core flag, Jastrow parameter row.
constexpr int kNucLen = 7;

struct PhaseArgs {
    int scheme;              // 0 load-balanced, 1 conventional
    int nproj;
    int refresh_every;
    int nu_mode;
    int conv_cap;            // hard bound on conventional iterations per phase
    int rotate;              // 1: random lattice orientation per walker and phase
    double a, tau;
    uint64_t seed;
    unsigned long long *counters;   // [kCntLen]
    unsigned long long *timers;     // [nw][8] section cycles (instrumentation builds)
};

// Mixed-precision walker layout for large systems: one 256-thread workgroup
// per walker, orbital data in HBM (FP32), the small per-electron and
// per-move arrays in LDS, FP64 for positions, potentials, weights, sums and
// the periodic Gauss-Jordan refresh.
constexpr int kMixThreads = 256;
enum : int { kGemmFP32 = 0, kGemmBF16 = 1 };

struct DevMix {
    int M, Nb, Norb, Nup, Ndn, N, P, ns, nspec, nw, has_en, gemm;
    double vii;
    uint64_t sysid;
    const int *jp;               // branching index, device
    const double *e0p;           // E_0 of this system, device
    const double *R, *Z, *rc, *jas, *btab;
    const int32_t *core, *spec, *btype;
    const float *Cf;             // [Nb][ns] coefficients, FP32
    const uint16_t *Cbf;         // [2][tiles][Nb/32][64 lanes][8] BF16 MFMA B operands:
                                 // high part, then the BF16 residual (low part)
    int nb32;                    // Nb rounded up to a multiple of 32
    int fkc;                     // basis functions per chunk of the FP64 Slater rows
    const double *C64;           // [Nb][Norb] coefficients, FP64 (estimator evaluation)
    double *s64;                 // [nw][stride64] FP64 scratch: Slater rows, inverses
    long stride64;
    double *diag;                // [nw][4] error report of the last phase: e_L, W, bbar of
                                 // the mixed-precision step at the final configuration,
                                 // largest ratio error against the FP64 evaluation
    double *pos, *lw, *eL, *Wd;  // [nw][N][3], [nw]
    float *state;                // [nw][stride] walker blocks (current buffer)
    long stride;                 // floats per walker block
    // offsets (floats) inside a walker block
    long g_Phi;                  // [2][ns][6 ns]  orbital values at the moves, k-major per spin
    long g_dPhi;                 // [2][ns][4 ns]  gradient and Laplacian, k-major per spin
    long g_Arow;                 // [N][ns]        Slater rows
    long g_AinvT;                // [2][ns][ns]    transposed inverses
    int32_t *iters, *trace;
    int trace_cap;
    // LDS layout, byte offsets
    int l_pos, l_nue, l_nua, l_scal, l_red, l_U, l_R, l_Rdet, l_dJ, l_gD, l_Jg, l_Jl, l_dje,
        l_rows, l_tmp, l_F, l_ev, l_bytes;
    // l_ev: the walker's lattice step vectors a e_d for the phase, [3 d + x]:
    // 9 doubles, then the same 9 as floats
};
constexpr int kMixChunk = 64;   // basis functions per chunk of the FP64 estimator evaluation

// Adjoint pass (parameter derivatives of e_L and log|Psi| at fixed walkers):
// one 256-thread workgroup per walker, FP64, everything in LDS.
constexpr int kAdjThreads = 256;
struct DevAdj {
    int M, Nb, Norb, Nup, Ndn, N, ns, nspec, nw, nth, nu_mode;
    double a, vii;
    const double *R, *Z, *rc, *jas, *btab, *C;   // R, jas and btab centres follow theta
    const int32_t *core, *spec, *batom, *btype;
    const double *pos;                          // [nw][N][3]
    double *eL, *lp;                            // [nw]
    double *deL, *dlp;                          // [nw][nth]
    int *status;                                // walkers with a singular Slater matrix
    // LDS layout (offsets in doubles)
    int o_pos, o_phi, o_dphi, o_phi6, o_ainv, o_Z, o_T, o_Y, o_G, o_chi, o_gj, o_Lj, o_dJ, o_R,
        o_Rdet, o_gd, o_Ld, o_nu, o_nua, o_al, o_sgd, o_sgj, o_sRd, o_sdJ, o_snu, o_snua, o_GeL,
        o_Glp, o_sc, o_piv, lds_doubles;
};

// Systems advanced by one launch of the mixed-precision phase kernel.
constexpr int kMaxBatch = 8;
struct MixBatch {
    const DevMix *tab;            // [nsys] descriptors in launch order
    int nsys;
    int start[kMaxBatch + 1];     // first workgroup of each system, start[nsys] = total
};

// What the reconfiguration kernels see of a system (either layout).
struct BranchView {
    int nw, N;
    uint64_t sysid;
    double *pos, *lw, *eL, *Wd;   // current buffers
    const int *jp;                // branching index
    const double *e0p;            // E_0
};

// device history ring of the branchings: one record per branching
enum : int { kHistLogW = 0, kHistEbar = 1, kHistE0 = 2, kHistMaxLw = 3, kHistDistinct = 4,
             kHistLen = 8 };
constexpr int kHistCap = 4096;

// per-walker scalars stored at o_scal / l_scal: V_ee (slots 0..3 unused)
enum : int { kScVee = 4, kScRes = 5, kScLen = 8 };

}  // namespace lrdmc
