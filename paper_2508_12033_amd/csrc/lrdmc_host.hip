// Host side of the C ABI declared in include/lrdmc.h: validation, workspace
// carving, kernel launches on the caller's stream, and the host-level pieces
// of the method (E_0 update after each branching, Algorithm 2; the
// correcting-factor energy estimate and its blocking error bar, Sec. II.A).
//
// Two walker layouts: FP64 runs use the LDS-resident one-wavefront-per-walker
// phase kernel (phase_fp64, one launch per system); mixed-precision runs use
// the workgroup-per-walker kernel with orbital data in HBM (phase_mixed), one
// launch for the walkers of every system.  Both share the reconfiguration
// kernels.  E_0, the branching index and the history of the branchings live
// on the device, so that a projection phase plus its reconfiguration can be
// captured once into a graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lrdmc.h"
#include "lrdmc_dev.hpp"

namespace lrdmc {
template <bool kRot, bool kNl, bool kBig>
__global__ void phase_fp64(const DevSys* __restrict__ sys, PhaseArgs pa);
extern template __global__ void phase_fp64<false, false, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
extern template __global__ void phase_fp64<true, false, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
extern template __global__ void phase_fp64<false, true, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
extern template __global__ void phase_fp64<true, true, false>(const DevSys* __restrict__ sys, PhaseArgs pa);
extern template __global__ void phase_fp64<false, false, true>(const DevSys* __restrict__ sys, PhaseArgs pa);
extern template __global__ void phase_fp64<true, false, true>(const DevSys* __restrict__ sys, PhaseArgs pa);

// the FP64 phase kernel for a lattice geometry, Hamiltonian and layout
inline void (*phase_kernel(bool rot, bool nl, bool big))(const DevSys*, PhaseArgs)
{
    if (nl) return rot ? phase_fp64<true, true, false> : phase_fp64<false, true, false>;
    if (big) return rot ? phase_fp64<true, false, true> : phase_fp64<false, false, true>;
    return rot ? phase_fp64<true, false, false> : phase_fp64<false, false, false>;
}
__global__ void phase_mixed(MixBatch b, PhaseArgs pa, int build);
__global__ void branch_scan(BranchView s, int scheme, double* cum, double* out, int* n_distinct);
__global__ void branch_comb(BranchView s, uint64_t seed, const double* cum, const double* out,
                            int32_t* sel);
__global__ void branch_count(const int32_t* sel, int nw, int* n_distinct);
__global__ void branch_gather(BranchView s, const int32_t* sel, const double* pos_old,
                              const double* eL_old, const double* W_old);
__global__ void branch_gather_mixed(const DevMix* __restrict__ sys, const int32_t* sel,
                                    const float* old_state, const double* pos_old,
                                    const double* eL_old, const double* W_old);
__global__ void branch_finish(int nw, const double* out, const int* n_distinct, double* hist,
                              long long* n_hist, double* e0p, int* n_dead, int window, int cap,
                              int* bump_j);
__global__ void reset_counters_kernel(unsigned long long* c);
__global__ void walker_derivs(const DevAdj* __restrict__ sys);
__global__ void derivs_reduce(int nw, int nth, int scheme, const double* lw, const double* Wd,
                              const double* e0p, const double* eL, const double* deL,
                              const double* dlp, double* out);

// E_0 and the branching index of a caller-held reconfiguration, written by a
// kernel so that the whole sequence can be captured in a graph
__global__ void reconf_setup(double* ctl, double e0, int j)
{
    if (threadIdx.x == 0) {
        ctl[0] = e0;
        *reinterpret_cast<int*>(ctl + 1) = j;
        *reinterpret_cast<int*>(ctl + 2) = 0;
    }
}

// out[0] log wbar = log(C_N / N_w) + max lw, out[1] walker-averaged e_L,
// out[2] max lw, out[3] distinct parents, out[4] status: 0 ok, 1 every weight
// zero, 2 non-finite sums (a NaN or +inf log-weight, or W - E_0 = 0)
__global__ void reconf_finish(int nw, const double* bout, const int* ndist, double* out)
{
    if (threadIdx.x != 0) return;
    const double mx = bout[0], tot = bout[1], se = bout[2], so = bout[3];
    const bool all_dead = mx == -INFINITY;
    const bool finite = isfinite(mx) && isfinite(tot) && tot > 0.0 && isfinite(se) &&
                        isfinite(so) && so != 0.0 && isfinite(se / so);
    out[0] = finite ? log(tot / (double)nw) + mx : NAN;
    out[1] = finite ? se / so : NAN;
    out[2] = mx;
    out[3] = (double)*ndist;
    out[4] = all_dead ? 1.0 : (finite ? 0.0 : 2.0);
}
}  // namespace lrdmc

using namespace lrdmc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(LRDMC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxLdsBytes = 160 * 1024;
enum { kKindLds = 0, kKindMixed = 1 };

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int kind_of(const lrdmc_params& p) { return p.precision == LRDMC_FP64 ? kKindLds : kKindMixed; }

// Per-system sizes and layout, computed identically by workspace_bytes and init.
struct Layout {
    int kind, N, P, ns;
    int PT;                  // proposals: 6N, or 12N with a non-local pseudopotential
    int o_Vnl, o_nlin;
    // FP64 kernel: LDS offsets (doubles), spill layout
    int ldb;
    int o_pos, o_R, o_Rdet, o_dJ, o_Arow, o_AinvT, o_Jg, o_Jl, o_nue, o_nua, o_dje, o_scal, o_B,
        o_rows, o_tmp, o_C, o_nuc, o_jas, o_gd, o_ev, lds_doubles;
    bool big;                // large-system layout: coefficient block and Slater rows in global memory
    int bchunk;              // large-system layout: basis functions per chunk of the orbital product
    bool ainv1;              // large-system layout: one spin's inverse in LDS, both in global memory
    long s_AinvG, s_GJ;
    int s_Phi, s_dPhi, s_Arow;
    long spill_stride;
    // mixed kernel: LDS byte offsets, walker block (floats)
    int l_pos, l_nue, l_nua, l_scal, l_red, l_U, l_R, l_Rdet, l_dJ, l_gD, l_Jg, l_Jl, l_dje, l_rows,
        l_tmp, l_F, l_ev, l_bytes;
    long g_Phi, g_dPhi, g_Arow, g_AinvT, m_stride, stride64;
    int nb32, tiles;
    size_t lds_bytes;
    int fkc = 4;
    // adjoint pass: LDS offsets (doubles)
    int nth;
    int a_pos, a_phi, a_dphi, a_phi6, a_ainv, a_Z, a_T, a_Y, a_G, a_chi, a_gj, a_Lj, a_dJ, a_R,
        a_Rdet, a_gd, a_Ld, a_nu, a_nua, a_al, a_sgd, a_sgj, a_sRd, a_sdJ, a_snu, a_snua, a_GeL,
        a_Glp, a_sc, a_piv, a_doubles;
    // workspace bytes
    size_t b_sys, b_state, b_adj;
};

Layout make_layout(const lrdmc_system& s, const lrdmc_params& p)
{
    Layout L{};
    L.kind = kind_of(p);
    L.N = s.n_up + s.n_dn;
    L.P = 6 * L.N;
    L.PT = s.n_ecp > 0 ? 12 * L.N : L.P;
    L.ns = std::max(1, std::max(s.n_up, s.n_dn));
    const int M = s.n_atoms, Nb = s.n_basis, N = L.N, P = L.P, ns = L.ns, PT = L.PT;
    const bool nl = s.n_ecp > 0;
    const size_t nw = s.n_walkers;
    L.b_sys = align_up(M * 3 * 8) + 2 * align_up(M * 8) + 2 * align_up(M * 4) +
              2 * align_up(Nb * 4) + align_up(Nb * 8) + align_up((size_t)Nb * s.n_orb * 8) +
              align_up((2 + s.n_species) * 3 * 8) + align_up((size_t)Nb * 4 * 8) + align_up(Nb * 8) +
              (nl ? 3 * align_up((size_t)s.n_ecp * 4) + 2 * align_up((size_t)s.n_ecp * 8) + align_up(M * 8)
                  : 0);
    size_t common = 2 * align_up(nw * 3 * N * 8)    // positions, double-buffered
                    + align_up(nw * 8)              // lw
                    + 4 * align_up(nw * 8)          // eL, W double-buffered
                    + 2 * align_up(nw * 4)          // iters, sel
                    + align_up(nw * 8)              // cumulative weights
                    + align_up(8 * 8)               // branch outputs
                    + align_up(8)                   // distinct counter
                    + (p.trace_cap > 0 ? align_up(nw * (size_t)p.trace_cap * 4) : 0);
    if (L.kind == kKindLds) {
        // the LDS-resident layout, or (without a pseudopotential) the
        // large-system layout: coefficient block and Slater rows in global
        // memory, the basis block sized for the refresh's n x n half and for
        // one chunk of the orbital product (all functions, or 64), the
        // pair-term scratch in the basis block.  The layout that puts more
        // walkers on a CU wins (the kernel's 256 registers allow at most 8);
        // on a tie the earlier one: LDS-resident (faster coefficient reads),
        // then the large-system layout in one chunk (less overhead), in
        // chunks, and in chunks with one spin's inverse in LDS (the moved
        // spin's block staged from global memory, the refresh's left half in
        // global memory).
        Layout keep{};
        int keep_w = -1;
        for (int pass = 0; pass < 4; ++pass) {
            const bool big = pass > 0;
            L.bchunk = pass >= 2 ? std::min(Nb, 64) : Nb;
            L.ainv1 = pass == 3;
            int o = 0;
            auto take = [&](int n) { int r = o; o += (n + 1) / 2 * 2; return r; };
            L.big = big;
            L.o_pos = take(3 * N);
            L.o_R = take(PT);
            L.o_Rdet = take(PT);
            L.o_dJ = take(P);
            L.o_Arow = big ? 0 : take(N * ns);
            L.o_AinvT = take((L.ainv1 ? 1 : 2) * ns * ns);
            L.o_Jg = take(3 * N);
            L.o_Jl = take(N);
            L.o_nue = take(N);
            L.o_nua = take(N);
            L.o_dje = big ? 0 : take(N);
            L.o_scal = take(kScRes + 1);
            // basis block: one chunk of the orbital product
            const int nbb = L.bchunk;
            L.ldb = nbb + ((20 - nbb % 16) % 16);
            L.o_B = take(std::max(std::max(11 * L.ldb, L.ainv1 ? 0 : (big ? 1 : 2) * ns * ns), 7 * N));
            if (big) L.o_dje = L.o_B;
            L.o_rows = take(11 * ns);
            L.o_tmp = take(3 * ns + 16);
            L.o_C = take(nl || big ? 0 : Nb * ns);   // read from global memory otherwise
            L.o_nuc = take(kNucLen * M);
            L.o_jas = take(3 * (2 + s.n_species));
            L.o_gd = take(4 * N);
            L.o_ev = take(nl ? 18 : 9);
            L.o_Vnl = nl ? take(P) : 0;
            L.o_nlin = nl ? take(N) : 0;
            L.lds_doubles = o;
            L.lds_bytes = (size_t)o * 8;
            const int wcu = L.lds_bytes > (size_t)kMaxLdsBytes ? 0
                            : (int)std::min<size_t>(8, (size_t)kMaxLdsBytes / L.lds_bytes);
            if (wcu > keep_w) { keep = L; keep_w = wcu; }
            if (nl) break;
        }
        L = keep;
        L.s_Phi = 0;
        L.s_dPhi = PT * ns;
        {
            size_t sb = align_up((size_t)(PT * ns + 4 * N * ns) * 8);
            L.s_Arow = L.big ? (int)(sb / 8) : 0;
            if (L.big) sb += align_up((size_t)N * ns * 8);
            L.s_AinvG = L.ainv1 ? (long)(sb / 8) : 0;
            if (L.ainv1) sb += align_up((size_t)2 * ns * ns * 8);
            L.s_GJ = L.ainv1 ? (long)(sb / 8) : 0;
            if (L.ainv1) sb += align_up((size_t)ns * ns * 8);
            L.spill_stride = (long)(sb / 8);
        }
        L.b_state = common + align_up(nw * L.spill_stride * 8) + 2 * align_up(sizeof(DevSys));
    } else {
        L.nb32 = (Nb + 31) / 32 * 32;
        L.tiles = (ns + 15) / 16;
        int o = 0;
        auto take = [&](size_t bytes) { int r = o; o += (int)((bytes + 15) / 16 * 16); return r; };
        L.l_pos = take(3 * N * 8);
        L.l_nue = take(N * 8);
        L.l_nua = take(N * 8);
        L.l_scal = take(kScLen * 8);
        L.l_red = take(64 * 8);    // block sums, heat-bath picks, 13-way sums
        {
            const size_t uby = std::max(std::max(std::max((size_t)11 * (L.nb32 + 4) * 4,
                                                          (size_t)(ns * (ns + 1) + 3 * ns) * 8),
                                                 (size_t)7 * N * 8),
                                        (size_t)11 * kMixChunk * 8);
            // basis-value chunk of the FP64 Slater rows: [N rounded to 16][kc + 1] doubles,
            // kc the largest multiple of 4 (at most 32) that fits the block, at least 4
            const size_t rows16 = (size_t)(N + 15) / 16 * 16;
            int kc = (int)(uby / (rows16 * 8)) - 1;
            kc = std::min(32, kc) / 4 * 4;
            if (kc < 4) kc = 4;
            L.fkc = kc;
            L.l_U = take(std::max(uby, rows16 * (kc + 1) * 8));
        }
        L.l_R = take(P * 4);
        L.l_Rdet = take(P * 4);
        L.l_dJ = take(P * 4);
        L.l_gD = take(4 * N * 4);
        L.l_Jg = take(3 * N * 4);
        L.l_Jl = take(N * 4);
        L.l_dje = take(N * 4);
        L.l_rows = take(11 * ns * 4);
        L.l_tmp = take((3 * ns + 8) * 4);
        L.l_F = take((size_t)(2 * P + 8 * N) * 8);
        L.l_ev = take(9 * 8 + 9 * 4);
        L.l_bytes = o;
        L.lds_bytes = o;
        L.g_Phi = 0;
        L.g_dPhi = L.g_Phi + 2L * ns * 6 * ns;
        L.g_Arow = L.g_dPhi + 2L * ns * 4 * ns;
        L.g_AinvT = L.g_Arow + (long)N * ns;
        L.m_stride = (L.g_AinvT + 2L * ns * ns + 63) / 64 * 64;
        L.stride64 = (long)N * ns + 2L * ns * ns + 2L * Nb * ns;
        L.b_sys += align_up((size_t)Nb * ns * 4) +
                   align_up((size_t)2 * L.tiles * (L.nb32 / 32) * 64 * 8 * 2);
        L.b_state = common + 2 * align_up(nw * L.m_stride * 4) + align_up(nw * L.stride64 * 8) +
                    align_up(nw * 4 * 8) + 2 * align_up(sizeof(DevMix));
    }
    {
        int o = 0;
        auto take = [&](int n) { int r = o; o += (n + 1) / 2 * 2; return r; };
        L.nth = 3 * M + 3 * (2 + s.n_species);
        L.a_pos = take(3 * N); L.a_phi = take(N * ns); L.a_dphi = take(4 * N * ns);
        L.a_phi6 = take(6 * N * ns); L.a_ainv = take(2 * ns * ns); L.a_Z = take(2 * Nb * ns);
        L.a_T = take(N * Nb); L.a_Y = take(2 * ns * ns); L.a_G = take(ns * ns + ns);
        L.a_chi = take(11 * Nb); L.a_gj = take(3 * N); L.a_Lj = take(N); L.a_dJ = take(P);
        L.a_R = take(P); L.a_Rdet = take(P); L.a_gd = take(3 * N); L.a_Ld = take(N);
        L.a_nu = take(N); L.a_nua = take(N); L.a_al = take(N); L.a_sgd = take(3 * N);
        L.a_sgj = take(3 * N); L.a_sRd = take(P); L.a_sdJ = take(P); L.a_snu = take(N);
        L.a_snua = take(N); L.a_GeL = take(L.nth); L.a_Glp = take(L.nth); L.a_sc = take(16);
        L.a_piv = take(ns / 2 + 1);
        L.a_doubles = o;
        const int nspec = s.n_species;
        L.b_adj = align_up(M * 3 * 8) + align_up((2 + nspec) * 3 * 8) + align_up((size_t)Nb * 4 * 8) +
                  2 * align_up(nw * 8) + 2 * align_up(nw * (size_t)L.nth * 8) + align_up(8) +
                  align_up((3 * (size_t)L.nth + 2) * 8) + align_up(8) + align_up(sizeof(DevAdj));
    }
    return L;
}

std::string validate(const lrdmc_system* sys, int n_sys, const lrdmc_params* prm)
{
    if (!sys || n_sys < 1) return "no systems";
    if (!prm) return "null params";
    if (prm->scheme != LRDMC_SCHEME_LB && prm->scheme != LRDMC_SCHEME_CONV) return "bad scheme";
    if (prm->precision != LRDMC_FP64 && prm->precision != LRDMC_MIXED_FP32 &&
        prm->precision != LRDMC_MIXED_BF16)
        return "bad precision";
    if (!(prm->a > 0)) return "lattice space a must be > 0";
    if (prm->scheme == LRDMC_SCHEME_CONV && !(prm->tau > 0)) return "tau must be > 0";
    if (prm->scheme == LRDMC_SCHEME_LB && prm->n_proj < 1) return "n_proj must be >= 1";
    if (prm->refresh_every < 1) return "refresh_every must be >= 1";
    if (prm->nu_opt_mode < 0 || prm->nu_opt_mode > 2) return "bad nu_opt_mode";
    if (prm->trace_cap < 0) return "bad trace_cap";
    if (prm->strict != 0 && prm->strict != 1) return "strict must be 0 or 1";
    if (prm->rotate != 0 && prm->rotate != 1) return "rotate must be 0 or 1";
    if (prm->n_therm < 0) return "n_therm must be >= 0";
    if (prm->e0_window < 0 || prm->e0_window > kHistCap) return "e0_window out of range";
    if (n_sys > kMaxBatch) return "at most 8 systems per handle";
    for (int k = 0; k < n_sys; ++k) {
        const lrdmc_system& s = sys[k];
        if (s.n_atoms < 1 || s.n_basis < 1 || s.n_up < 0 || s.n_dn < 0 || s.n_up + s.n_dn < 1)
            return "bad system sizes";
        if (s.n_orb < std::max(s.n_up, s.n_dn)) return "n_orb < max(n_up, n_dn)";
        if (s.n_walkers < 1) return "n_walkers must be >= 1";
        if (!s.atom_pos || !s.atom_charge || !s.atom_core || !s.core_rc || !s.atom_species ||
            !s.basis_atom || !s.basis_type || !s.basis_exp || !s.mo_coeff || !s.jastrow)
            return "null system array";
        for (int i = 0; i < s.n_atoms; ++i) {
            if (s.atom_core[i] != LRDMC_CORE_BARE && s.atom_core[i] != LRDMC_CORE_SOFT)
                return "bad atom_core";
            if (s.atom_core[i] == LRDMC_CORE_SOFT && !(s.core_rc[i] > 0)) return "core_rc <= 0";
            if (s.atom_species[i] < 0 || s.atom_species[i] >= s.n_species) return "bad species";
        }
        for (int mu = 0; mu < s.n_basis; ++mu) {
            if (s.basis_atom[mu] < 0 || s.basis_atom[mu] >= s.n_atoms) return "bad basis_atom";
            if (s.basis_type[mu] < 0 || s.basis_type[mu] > 4) return "bad basis_type";
            if (!(s.basis_exp[mu] > 0)) return "basis exponent <= 0";
        }
        if (s.n_ecp < 0) return "bad n_ecp";
        if (s.n_ecp > 0) {
            if (prm->precision != LRDMC_FP64)
                return "non-local pseudopotential: not supported by the mixed-precision kinds";
            if (!s.ecp_atom || !s.ecp_l || !s.ecp_pow || !s.ecp_coef || !s.ecp_exp || !s.ecp_rcut)
                return "null pseudopotential array";
            for (int I = 0; I < s.n_atoms; ++I)
                if (!(s.ecp_rcut[I] >= 0)) return "bad ecp_rcut";
            for (int t = 0; t < s.n_ecp; ++t) {
                if (s.ecp_atom[t] < 0 || s.ecp_atom[t] >= s.n_atoms) return "bad ecp_atom";
                if (s.ecp_l[t] < 0 || s.ecp_l[t] > 2) return "ecp_l must be 0, 1 or 2";
                if (s.ecp_pow[t] < 0 || s.ecp_pow[t] > 2) return "ecp_pow must be 0, 1 or 2";
                if (!(s.ecp_exp[t] >= 0) || !std::isfinite(s.ecp_coef[t])) return "bad ecp term";
                if (!(s.ecp_rcut[s.ecp_atom[t]] > 0)) return "ecp term on an atom without a cutoff radius";
            }
            for (int I = 0; I < s.n_atoms; ++I)
                for (int J = I + 1; J < s.n_atoms; ++J) {
                    if (!(s.ecp_rcut[I] > 0 && s.ecp_rcut[J] > 0)) continue;
                    const double* A = s.atom_pos + 3 * I;
                    const double* B = s.atom_pos + 3 * J;
                    const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
                    if (std::sqrt(dx * dx + dy * dy + dz * dz) <= s.ecp_rcut[I] + s.ecp_rcut[J])
                        return "pseudopotential cutoff spheres overlap";
                }
        }
        if (std::max(s.n_up, s.n_dn) > 64)
            return prm->precision != LRDMC_FP64
                       ? "mixed-precision layout: at most 64 electrons per spin (too large)"
                       : "FP64 layouts: at most 64 electrons per spin (too large)";
        const Layout L = make_layout(s, *prm);
        if (L.lds_bytes > (size_t)kMaxLdsBytes)
            return L.kind == kKindLds ? "system too large for the FP64 walker layouts "
                                        "(use a mixed precision)"
                                      : "system too large for the mixed-precision walker layout";
        if (s.n_walkers > (1 << 24)) return "too many walkers";
    }
    return "";
}

uint16_t to_bf16(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    const uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);                // nearest even
    return (uint16_t)((u + rounding) >> 16);
}

struct SysRun {
    int kind;
    bool nl = false;                     // non-local pseudopotential (FP64 kernel)
    Layout L;
    int nw, N;
    uint64_t sysid;
    // walker buffers by slot; the current slot is the handle's parity, the
    // other one receives the gather of the next reconfiguration
    double *pos[2], *eL[2], *Wd[2];
    float* state[2];                     // mixed layout walker blocks
    double* lw;
    int32_t *iters, *trace, *sel;
    double *cum, *bout;
    int* ndist;
    // device control: E_0, history ring of the branchings, dead-population count
    double* d_e0;
    double* d_hist;
    long long* d_nhist;
    int* d_dead;
    long long h_nhist;
    int h_dead;
    int h_nonfinite = 0;
    // descriptors per slot
    DevSys hsys[2];
    DevSys* dsys[2];
    DevMix hmix[2];
    DevMix* dmix[2];
    bool need_build;
    double e0;
    std::vector<double> hist_lwb, hist_e, hist_e0, hist_mx, hist_nd;
    std::vector<double> btab_host;
    // adjoint pass: theta-dependent copies of the system arrays, outputs
    DevAdj ad;
    DevAdj* dadj;
    double *R_t, *jas_t, *btab_t, *a_eL, *a_lp, *a_deL, *a_dlp, *a_out;
    int* a_status;
    std::vector<double> h_R, h_Z, h_bexp, h_jas;
    std::vector<int32_t> h_batom;
    std::vector<float> cf_host;
    std::vector<uint16_t> cbf_host;
};

BranchView view_of(const SysRun& r, int slot, const int* jp)
{
    BranchView v;
    v.nw = r.nw; v.N = r.N; v.sysid = r.sysid;
    v.pos = r.pos[slot]; v.lw = r.lw; v.eL = r.eL[slot]; v.Wd = r.Wd[slot];
    v.jp = jp; v.e0p = r.d_e0;
    return v;
}

size_t handle_bytes(int n_sys)
{
    return align_up(kCntLen * 8) + align_up(8) + 2 * align_up((size_t)n_sys * sizeof(DevMix));
}

size_t control_bytes()
{
    return align_up(8) + align_up((size_t)kHistCap * kHistLen * 8) + align_up(8) + align_up(8);
}

}  // namespace

struct lrdmc_handle {
    std::vector<SysRun> sys;
    lrdmc_params prm;
    hipStream_t stream;
    int j;                                  // host mirror of the branching index
    int parity;                             // current walker slot
    int* d_j;
    unsigned long long* counters;           // [kCntLen] device
    hipEvent_t ev0, ev1;
    unsigned long long* timers = nullptr;   // instrumentation builds: [nw][8]
    // one launch advances every mixed-precision system (batched), or one
    // launch per system with its own workgroup size and LDS block (separate)
    std::vector<int> mix_order;             // system indices in launch order
    DevMix* mix_tab[2];                     // device descriptor tables per slot
    int mix_threads = kMixThreads;
    size_t mix_lds = 0;
    int mix_separate = 0;
    std::vector<int> mix_sys_threads;       // [system] workgroup size when separate
    // captured step + reconfiguration per slot
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::vector<lrdmc_tune_entry> tune_log;
};

namespace {

int maxN_all(const lrdmc_handle* h)
{
    int m = 1;
    for (int k : h->mix_order) m = std::max(m, h->sys[k].N);
    return m;
}

int upload_mix_tables(lrdmc_handle* h)
{
    const int n = (int)h->mix_order.size();
    if (!n) return LRDMC_OK;
    for (int p = 0; p < 2; ++p) {
        std::vector<DevMix> t(n);
        for (int k = 0; k < n; ++k) t[k] = h->sys[h->mix_order[k]].hmix[p];
        HIPCHK(hipMemcpyAsync(h->mix_tab[p], t.data(), n * sizeof(DevMix), hipMemcpyHostToDevice,
                              h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return LRDMC_OK;
}

void drop_graphs(lrdmc_handle* h)
{
    for (int p = 0; p < 2; ++p)
        if (h->gexec[p]) { (void)hipGraphExecDestroy(h->gexec[p]); h->gexec[p] = nullptr; }
}

// Termination bound of the conventional loop: 1000 times the mean number of
// moves tau * 3N/a^2 (plus a floor).  Reaching it is counted and reported.
int conv_cap(const lrdmc_params& p, int N)
{
    const double mean = p.tau * 3.0 * N / (p.a * p.a);
    const double cap = 1000.0 * mean + 10000.0;
    return cap > 2e9 ? 2000000000 : (int)cap;
}

PhaseArgs phase_args(const lrdmc_handle* h, int N, int nproj_override)
{
    PhaseArgs pa{};
    pa.scheme = nproj_override >= 0 ? 0 : h->prm.scheme;
    pa.nproj = nproj_override >= 0 ? nproj_override : h->prm.n_proj;
    pa.refresh_every = h->prm.refresh_every;
    pa.nu_mode = h->prm.nu_opt_mode;
    pa.conv_cap = conv_cap(h->prm, N);
    pa.rotate = h->prm.rotate;
    pa.a = h->prm.a;
    pa.tau = h->prm.tau;
    pa.seed = h->prm.seed;
    pa.counters = h->counters;
    pa.timers = h->timers;
    return pa;
}

// The mixed-precision phase of the systems in launch order, walkers in slot p:
// one launch for all of them (workgroup b of system k when start[k] <= b <
// start[k+1]; every system gets the largest LDS block and one workgroup size),
// or with separate = 1 one launch per system with its own LDS block and
// workgroup size.  only >= 0: that system alone (the autotuner's timing runs),
// with workgroup size threads_only.
int launch_mixed(lrdmc_handle* h, hipStream_t st, int p, int nproj_override, int build, int separate,
                 int only, int threads_only = 0)
{
    const int n = (int)h->mix_order.size();
    if (!separate && only < 0) {
        MixBatch b{};
        b.tab = h->mix_tab[p];
        b.nsys = n;
        int tot = 0, maxN = 1;
        for (int k = 0; k < n; ++k) {
            SysRun& r = h->sys[h->mix_order[k]];
            b.start[k] = tot;
            tot += r.nw;
            maxN = std::max(maxN, r.N);
        }
        b.start[n] = tot;
        const PhaseArgs pa = phase_args(h, maxN, nproj_override);
        hipLaunchKernelGGL(phase_mixed, dim3(tot), dim3(h->mix_threads), h->mix_lds, st, b, pa, build);
        HIPCHK(hipGetLastError());
        return LRDMC_OK;
    }
    for (int k = 0; k < n; ++k) {
        const int isys = h->mix_order[k];
        if (only >= 0 && isys != only) continue;
        SysRun& r = h->sys[isys];
        MixBatch b{};
        b.tab = h->mix_tab[p] + k;
        b.nsys = 1;
        b.start[0] = 0;
        b.start[1] = r.nw;
        const int thr = only >= 0 ? threads_only : h->mix_sys_threads[isys];
        const PhaseArgs pa = phase_args(h, r.N, nproj_override);
        hipLaunchKernelGGL(phase_mixed, dim3(r.nw), dim3(thr), r.L.lds_bytes, st, b, pa, build);
        HIPCHK(hipGetLastError());
    }
    return LRDMC_OK;
}

// One projection phase for every system on stream st with walkers in slot p.
// nproj_override >= 0: a load-balanced phase of that many steps (0 = evaluate
// only).  FP64 systems: one launch each; mixed systems: launch_mixed.
int launch_phases(lrdmc_handle* h, hipStream_t st, int p, int nproj_override, bool allow_build)
{
    for (auto& r : h->sys) {
        if (r.kind != kKindLds) continue;
        const PhaseArgs pa = phase_args(h, r.N, nproj_override);
        hipLaunchKernelGGL(phase_kernel(pa.rotate != 0, r.nl, r.L.big), dim3(r.nw), dim3(kWave),
                           r.L.lds_bytes, st,
                           (const DevSys*)r.dsys[p], pa);
        HIPCHK(hipGetLastError());
    }
    const int n = (int)h->mix_order.size();
    if (n) {
        int build = 0;
        for (int k = 0; k < n; ++k)
            if (h->sys[h->mix_order[k]].need_build) build = 1;
        if (build && !allow_build) return fail(LRDMC_ERR_INVALID_ARG, "rebuild pending in a capture");
        const int rc = launch_mixed(h, st, p, nproj_override, build, h->mix_separate, -1);
        if (rc) return rc;
        for (int k = 0; k < n; ++k) h->sys[h->mix_order[k]].need_build = false;
    }
    return LRDMC_OK;
}

// Reconfiguration of every system on stream st, walkers in slot p gathered
// into slot p ^ 1; device-side history and E_0 update; branching index + 1.
int enqueue_branch(lrdmc_handle* h, hipStream_t st, int p)
{
    const int nsys = (int)h->sys.size();
    for (int k = 0; k < nsys; ++k) {
        SysRun& r = h->sys[k];
        const int nw = r.nw;
        const BranchView bv = view_of(r, p, h->d_j);
        const int nt = std::min(kMaxBranchBlock, std::max(64, 1 << (int)std::ceil(std::log2((double)nw))));
        hipLaunchKernelGGL(branch_scan, dim3(1), dim3(nt), 0, st, bv, h->prm.scheme, r.cum, r.bout,
                           r.ndist);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(branch_comb, dim3((nw + 255) / 256), dim3(256), 0, st, bv, h->prm.seed,
                           (const double*)r.cum, (const double*)r.bout, r.sel);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(branch_count, dim3((nw + 255) / 256), dim3(256), 0, st,
                           (const int32_t*)r.sel, nw, r.ndist);
        HIPCHK(hipGetLastError());
        if (r.kind == kKindLds) {
            const BranchView dn = view_of(r, p ^ 1, h->d_j);
            const long tot = (long)nw * 3 * r.N;
            hipLaunchKernelGGL(branch_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                               dn, (const int32_t*)r.sel, (const double*)r.pos[p],
                               (const double*)r.eL[p], (const double*)r.Wd[p]);
        } else {
            hipLaunchKernelGGL(branch_gather_mixed, dim3(nw), dim3(256), 0, st,
                               (const DevMix*)r.dmix[p ^ 1], (const int32_t*)r.sel,
                               (const float*)r.state[p], (const double*)r.pos[p],
                               (const double*)r.eL[p], (const double*)r.Wd[p]);
        }
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(branch_finish, dim3(1), dim3(64), 0, st, nw, (const double*)r.bout,
                           (const int*)r.ndist, r.d_hist, r.d_nhist, r.d_e0, r.d_dead,
                           std::max(1, h->prm.e0_window), kHistCap, k == nsys - 1 ? h->d_j : nullptr);
        HIPCHK(hipGetLastError());
    }
    return LRDMC_OK;
}

// Copy the branchings recorded on the device since the last drain into the
// host history (synchronises).
int drain(lrdmc_handle* h)
{
    HIPCHK(hipStreamSynchronize(h->stream));
    int rc = LRDMC_OK;
    for (auto& r : h->sys) {
        long long n = 0;
        int dead[2] = {0, 0};   // all-dead and non-finite reconfigurations
        HIPCHK(hipMemcpy(&n, r.d_nhist, 8, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(dead, r.d_dead, 8, hipMemcpyDeviceToHost));
        if (n - r.h_nhist > kHistCap) rc = fail(LRDMC_ERR_INVALID_ARG, "branching history overflow");
        const long long q0 = std::max(r.h_nhist, n - kHistCap);
        std::vector<double> buf((size_t)kHistCap * kHistLen);
        for (long long q = q0; q < n;) {   // contiguous pieces of the ring
            const long long at = q % kHistCap, cnt = std::min(n - q, (long long)kHistCap - at);
            HIPCHK(hipMemcpy(buf.data() + at * kHistLen, r.d_hist + at * kHistLen,
                             (size_t)cnt * kHistLen * 8, hipMemcpyDeviceToHost));
            q += cnt;
        }
        for (long long q = q0; q < n; ++q) {
            const double* e = buf.data() + (q % kHistCap) * kHistLen;
            r.hist_lwb.push_back(e[kHistLogW]);
            r.hist_e.push_back(e[kHistEbar]);
            r.hist_e0.push_back(e[kHistE0]);
            r.hist_mx.push_back(e[kHistMaxLw]);
            r.hist_nd.push_back(e[kHistDistinct]);
            r.e0 = e[kHistE0];
        }
        r.h_nhist = n;
        if (dead[0] > r.h_dead) {
            r.h_dead = dead[0];
            rc = fail(LRDMC_ERR_ALL_DEAD, "every walker weight is zero");
        }
        if (dead[1] > r.h_nonfinite) {
            r.h_nonfinite = dead[1];
            rc = fail(LRDMC_ERR_NONFINITE, "non-finite weight sum or walker average at a reconfiguration");
        }
    }
    return rc;
}

int capture_graphs(lrdmc_handle* h)
{
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    for (int p = 0; p < 2; ++p) {
        if (h->gexec[p]) continue;
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = launch_phases(h, h->cap_stream, p, -1, false);
        if (!rc) rc = enqueue_branch(h, h->cap_stream, p);
        const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
        if (rc) { if (e == hipSuccess) (void)hipGraphDestroy(g); return rc; }
        HIPCHK(e);
        const hipError_t ei = hipGraphInstantiate(&h->gexec[p], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ei);
    }
    return LRDMC_OK;
}

int reset_counters(lrdmc_handle* h, hipStream_t st)
{
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, h->counters);
    HIPCHK(hipGetLastError());
    return LRDMC_OK;
}

int read_counters(lrdmc_handle* h, lrdmc_step_stats* st, float ms)
{
    unsigned long long cnt[kCntLen];
    HIPCHK(hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    st->walker_iters = (int64_t)cnt[kCntIters];
    st->max_iters = (int32_t)cnt[kCntMaxIters];
    st->min_iters = (int32_t)cnt[kCntMinIters];
    st->n_neg_weight = (int64_t)cnt[kCntNegW];
    st->n_no_move = (int64_t)cnt[kCntNoMove];
    st->n_refresh = (int64_t)cnt[kCntRefresh];
    st->n_small_ratio = (int64_t)cnt[kCntSmallR];
    st->n_capped = (int64_t)cnt[kCntCapped];
    st->n_nonfinite = (int64_t)cnt[kCntNonfinite];
    st->elapsed_ms = ms;
    if (cnt[kCntSingular]) return fail(LRDMC_ERR_SINGULAR, "singular Slater matrix in a refresh");
    if (cnt[kCntNonfinite])
        return fail(LRDMC_ERR_NONFINITE, std::to_string(cnt[kCntNonfinite]) +
                                             " walkers ended the phase with a non-finite e_L, W or log-weight");
    if (h->prm.strict && cnt[kCntNegW])
        return fail(LRDMC_ERR_NEG_WEIGHT, std::to_string(cnt[kCntNegW]) + " walker-steps with W - E_0 <= 0");
    if (h->prm.strict && cnt[kCntNoMove])
        return fail(LRDMC_ERR_NO_MOVE, std::to_string(cnt[kCntNoMove]) + " walker-steps with no allowed move");
    const unsigned long long warn = cnt[kCntNegW] + cnt[kCntNoMove];
    return warn > 0x7fffffffull ? 0x7fffffff : (int)warn;
}

void fill_branch_stats(const lrdmc_handle* h, lrdmc_branch_stats* st, float ms)
{
    const SysRun& r = h->sys[0];
    const size_t n = r.hist_e.size();
    st->elapsed_ms = ms;
    if (!n) { st->log_wbar = NAN; st->e_bar = NAN; st->e0 = r.e0; st->max_lw = NAN; st->n_distinct = 0; return; }
    st->log_wbar = r.hist_lwb[n - 1];
    st->e_bar = r.hist_e[n - 1];
    st->e0 = r.hist_e0[n - 1];
    st->max_lw = r.hist_mx[n - 1];
    st->n_distinct = (int)r.hist_nd[n - 1];
}

// ---------------------------------------------------------------------------
// Scratch of lrdmc_reconfigure_noalloc: a fixed device array, one copy per GPU
// that the library runs on, held until the process ends (8 MiB).  In host code
// `scratch` is only a host-side stand-in for the symbol; its device address on
// each GPU comes from hipGetSymbolAddress, called once per device with that
// device current, and only that address is passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[((LRDMC_NOALLOC_MAX_WALKERS + 31) / 32) * 32 + 16];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on first use)
int noalloc_scratch(double** out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LRDMC_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LRDMC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return LRDMC_OK;
}

// ---------------------------------------------------------------------------
// Reconfiguration of a caller-held population (lrdmc_reconfigure): the comb
// kernels of lrdmc_branch on device arrays passed by the caller, with their
// prefix sums and sums in a scratch block of reconf_scratch_doubles(nw)
// doubles: cum [nw] (padded to 32), the scan results [8], then E_0, the
// branching index and the distinct-parent count.
// ---------------------------------------------------------------------------
long reconf_scratch_doubles(int nw) { return ((long)nw + 31) / 32 * 32 + 16; }

int check_reconf_args(int scheme, int nw, const double* lw, const double* eL, const double* W,
                      const int32_t* sel, const double* out)
{
    if (scheme != LRDMC_SCHEME_LB && scheme != LRDMC_SCHEME_CONV)
        return fail(LRDMC_ERR_INVALID_ARG, "scheme must be LRDMC_SCHEME_LB or LRDMC_SCHEME_CONV");
    if (nw < 1) return fail(LRDMC_ERR_INVALID_ARG, "nw must be positive");
    if (!lw || !eL || !sel || !out || (scheme == LRDMC_SCHEME_LB && !W))
        return fail(LRDMC_ERR_INVALID_ARG, "null device pointer");
    return LRDMC_OK;
}

int enqueue_reconfigure(int scheme, int nw, const double* lw, const double* eL, const double* W,
                        double e0, uint64_t seed, uint64_t sysid, int j, int32_t* sel, double* out,
                        double* scr, hipStream_t st)
{
    double* cum = scr;
    double* bout = scr + (reconf_scratch_doubles(nw) - 16);
    double* ctl = bout + 8;
    int* jp = reinterpret_cast<int*>(ctl + 1);
    int* ndist = reinterpret_cast<int*>(ctl + 2);
    BranchView bv{};
    bv.nw = nw; bv.N = 0; bv.sysid = sysid;
    bv.pos = nullptr; bv.lw = const_cast<double*>(lw); bv.eL = const_cast<double*>(eL);
    bv.Wd = const_cast<double*>(W ? W : eL);
    bv.jp = jp; bv.e0p = ctl;
    hipLaunchKernelGGL(reconf_setup, dim3(1), dim3(64), 0, st, ctl, e0, j);
    HIPCHK(hipGetLastError());
    const int nt = std::min(kMaxBranchBlock, std::max(64, 1 << (int)std::ceil(std::log2((double)nw))));
    hipLaunchKernelGGL(branch_scan, dim3(1), dim3(nt), 0, st, bv, scheme, cum, bout, ndist);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(branch_comb, dim3((nw + 255) / 256), dim3(256), 0, st, bv, seed,
                       (const double*)cum, (const double*)bout, sel);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(branch_count, dim3((nw + 255) / 256), dim3(256), 0, st, (const int32_t*)sel, nw,
                       ndist);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(reconf_finish, dim3(1), dim3(64), 0, st, nw, (const double*)bout,
                       (const int*)ndist, out);
    HIPCHK(hipGetLastError());
    return LRDMC_OK;
}

}  // namespace

extern "C" {

const char* lrdmc_last_error(void) { return g_err.c_str(); }

size_t lrdmc_workspace_bytes(const lrdmc_system* sys, int n_sys, const lrdmc_params* prm)
{
    const std::string v = validate(sys, n_sys, prm);
    if (!v.empty()) { g_err = v; return 0; }
    size_t tot = handle_bytes(n_sys);
    for (int k = 0; k < n_sys; ++k) {
        const Layout L = make_layout(sys[k], *prm);
        tot += L.b_sys + L.b_state + L.b_adj + control_bytes();
    }
    return tot;
}

static int run_derivs(lrdmc_handle* h, int isys, const double* theta, double* eL, double* lp,
                      double* deL, double* dlp);

int lrdmc_init_system(const lrdmc_system* sys, int n_sys, const lrdmc_params* prm,
                      const double* init_pos, void* dev_workspace, size_t ws_bytes, void* stream,
                      lrdmc_handle** out)
{
    if (!out) return fail(LRDMC_ERR_INVALID_ARG, "null handle pointer");
    *out = nullptr;
    const std::string v = validate(sys, n_sys, prm);
    if (!v.empty()) return fail(v.find("too large") != std::string::npos ||
                                        v.find("not supported") != std::string::npos
                                    ? LRDMC_ERR_UNSUPPORTED
                                                                           : LRDMC_ERR_INVALID_ARG,
                                v);
    if (!init_pos) return fail(LRDMC_ERR_INVALID_ARG, "null init_pos");
    if (!dev_workspace) return fail(LRDMC_ERR_INVALID_ARG, "null workspace");
    const size_t need = lrdmc_workspace_bytes(sys, n_sys, prm);
    if (ws_bytes < need)
        return fail(LRDMC_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) +
                                             " bytes, got " + std::to_string(ws_bytes));
    if (((uintptr_t)dev_workspace) % kAlign)
        return fail(LRDMC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");

    lrdmc_handle* h = new lrdmc_handle();
    h->prm = *prm;
    h->stream = (hipStream_t)stream;
    h->j = 0;
    h->parity = 0;
    h->sys.reserve(n_sys);
    char* base = (char*)dev_workspace;
    size_t off = 0;
    auto carve = [&](size_t bytes) { void* p = base + off; off += align_up(bytes); return p; };
    h->counters = (unsigned long long*)carve(kCntLen * 8);
    h->d_j = (int*)carve(8);
    h->mix_tab[0] = (DevMix*)carve((size_t)n_sys * sizeof(DevMix));
    h->mix_tab[1] = (DevMix*)carve((size_t)n_sys * sizeof(DevMix));
    hipError_t e1 = hipEventCreate(&h->ev0), e2 = hipEventCreate(&h->ev1);
    if (e1 != hipSuccess || e2 != hipSuccess) { delete h; return fail(LRDMC_ERR_HIP, "hipEventCreate"); }

    auto up = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream);
    };
    const int zero4[2] = {0, 0};
    const long long zero8 = 0;
    int rc = up(h->d_j, zero4, 4) == hipSuccess ? LRDMC_OK : fail(LRDMC_ERR_HIP, "upload failed");
    const double* ip = init_pos;
    for (int k = 0; k < n_sys && rc == LRDMC_OK; ++k) {
        const lrdmc_system& s = sys[k];
        h->sys.emplace_back();
        SysRun& r = h->sys.back();
        r.L = make_layout(s, *prm);
        r.kind = r.L.kind;
        r.nl = s.n_ecp > 0;
        const Layout& L = r.L;
        r.nw = s.n_walkers;
        r.N = L.N;
        r.sysid = s.system_id;
        int has_en = 0;
        for (int q = 0; q < s.n_species; ++q)
            if (s.jastrow[3 * (2 + q)] != 0.0 || s.jastrow[3 * (2 + q) + 1] != 0.0) has_en = 1;
        double vii = 0.0;
        for (int I = 0; I < s.n_atoms; ++I)
            for (int J = I + 1; J < s.n_atoms; ++J) {
                const double* A = s.atom_pos + 3 * I;
                const double* B = s.atom_pos + 3 * J;
                const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
                vii += s.atom_charge[I] * s.atom_charge[J] / std::sqrt(dx * dx + dy * dy + dz * dz);
            }
        const int M = s.n_atoms, Nb = s.n_basis, ns = L.ns;
        double* R = (double*)carve(M * 3 * 8);
        double* Z = (double*)carve(M * 8);
        double* rcs = (double*)carve(M * 8);
        int32_t* core = (int32_t*)carve(M * 4);
        int32_t* spec = (int32_t*)carve(M * 4);
        int32_t* batom = (int32_t*)carve(Nb * 4);
        int32_t* btype = (int32_t*)carve(Nb * 4);
        double* bexp = (double*)carve(Nb * 8);
        double* C = (double*)carve((size_t)Nb * s.n_orb * 8);
        double* jas = (double*)carve((2 + s.n_species) * 3 * 8);
        double* btab = (double*)carve((size_t)Nb * 4 * 8);
        double* bK = (double*)carve(Nb * 8);
        std::vector<double> bK_host(Nb);
        for (int mu = 0; mu < Nb; ++mu) bK_host[mu] = std::exp(-s.basis_exp[mu] * prm->a * prm->a);
        r.btab_host.resize((size_t)Nb * 4);
        for (int mu = 0; mu < Nb; ++mu) {
            const int at = s.basis_atom[mu];
            for (int c = 0; c < 3; ++c) r.btab_host[4 * mu + c] = s.atom_pos[3 * at + c];
            r.btab_host[4 * mu + 3] = s.basis_exp[mu];
        }
        if (up(R, s.atom_pos, M * 24) || up(Z, s.atom_charge, M * 8) || up(rcs, s.core_rc, M * 8) ||
            up(core, s.atom_core, M * 4) || up(spec, s.atom_species, M * 4) ||
            up(batom, s.basis_atom, Nb * 4) || up(btype, s.basis_type, Nb * 4) ||
            up(bexp, s.basis_exp, Nb * 8) || up(C, s.mo_coeff, (size_t)Nb * s.n_orb * 8) ||
            up(jas, s.jastrow, (2 + s.n_species) * 24) ||
            up(btab, r.btab_host.data(), (size_t)Nb * 32) || up(bK, bK_host.data(), Nb * 8)) {
            rc = fail(LRDMC_ERR_HIP, "upload of system arrays failed");
            break;
        }
        int32_t *e_atom = nullptr, *e_l = nullptr, *e_pow = nullptr;
        double *e_coef = nullptr, *e_exp = nullptr, *e_rcut = nullptr;
        if (r.nl) {
            const size_t ne = s.n_ecp;
            e_atom = (int32_t*)carve(ne * 4);
            e_l = (int32_t*)carve(ne * 4);
            e_pow = (int32_t*)carve(ne * 4);
            e_coef = (double*)carve(ne * 8);
            e_exp = (double*)carve(ne * 8);
            e_rcut = (double*)carve(M * 8);
            if (up(e_atom, s.ecp_atom, ne * 4) || up(e_l, s.ecp_l, ne * 4) || up(e_pow, s.ecp_pow, ne * 4) ||
                up(e_coef, s.ecp_coef, ne * 8) || up(e_exp, s.ecp_exp, ne * 8) ||
                up(e_rcut, s.ecp_rcut, M * 8)) {
                rc = fail(LRDMC_ERR_HIP, "upload of pseudopotential arrays failed");
                break;
            }
        }
        float* Cf = nullptr;
        uint16_t* Cbf = nullptr;
        if (r.kind == kKindMixed) {
            Cf = (float*)carve((size_t)Nb * ns * 4);
            Cbf = (uint16_t*)carve((size_t)2 * L.tiles * (L.nb32 / 32) * 64 * 8 * 2);
            r.cf_host.resize((size_t)Nb * ns);
            for (int mu = 0; mu < Nb; ++mu)
                for (int c = 0; c < ns; ++c)
                    r.cf_host[(size_t)mu * ns + c] = (float)s.mo_coeff[(size_t)mu * s.n_orb + c];
            // BF16 B operands of v_mfma_f32_16x16x32_bf16: lane l of k-block kb holds
            // C[32 kb + 8 (l / 16) + e][16 t + l % 16], e = 0..7; the high part
            // bf16(c) and the low part bf16(c - bf16(c)) in two planes
            const size_t plane = (size_t)L.tiles * (L.nb32 / 32) * 64 * 8;
            r.cbf_host.assign(2 * plane, 0);
            for (int t = 0; t < L.tiles; ++t)
                for (int kb = 0; kb < L.nb32 / 32; ++kb)
                    for (int l = 0; l < 64; ++l)
                        for (int e = 0; e < 8; ++e) {
                            const int mu = 32 * kb + 8 * (l / 16) + e, col = 16 * t + l % 16;
                            const float x = (mu < Nb && col < ns)
                                                ? (float)s.mo_coeff[(size_t)mu * s.n_orb + col]
                                                : 0.0f;
                            const uint16_t hi = to_bf16(x);
                            uint32_t hb = (uint32_t)hi << 16;
                            float hf;
                            std::memcpy(&hf, &hb, 4);
                            const size_t at = (((size_t)t * (L.nb32 / 32) + kb) * 64 + l) * 8 + e;
                            r.cbf_host[at] = hi;
                            r.cbf_host[plane + at] = to_bf16(x - hf);
                        }
            if (up(Cf, r.cf_host.data(), r.cf_host.size() * 4) ||
                up(Cbf, r.cbf_host.data(), r.cbf_host.size() * 2)) {
                rc = fail(LRDMC_ERR_HIP, "upload of coefficients failed");
                break;
            }
        }
        const size_t nw = s.n_walkers;
        for (int p = 0; p < 2; ++p) {
            r.pos[p] = (double*)carve(nw * 3 * L.N * 8);
            r.eL[p] = (double*)carve(nw * 8);
            r.Wd[p] = (double*)carve(nw * 8);
            r.state[p] = nullptr;
        }
        r.lw = (double*)carve(nw * 8);
        r.iters = (int32_t*)carve(nw * 4);
        r.sel = (int32_t*)carve(nw * 4);
        r.cum = (double*)carve(nw * 8);
        r.bout = (double*)carve(8 * 8);
        r.ndist = (int*)carve(8);
        r.trace = prm->trace_cap > 0 ? (int32_t*)carve(nw * (size_t)prm->trace_cap * 4) : nullptr;
        r.d_e0 = (double*)carve(8);
        r.d_hist = (double*)carve((size_t)kHistCap * kHistLen * 8);
        r.d_nhist = (long long*)carve(8);
        r.d_dead = (int*)carve(8);
        r.h_nhist = 0;
        r.h_dead = 0;
        r.need_build = false;
        if (up(r.d_nhist, &zero8, 8) || up(r.d_dead, zero4, 8)) {
            rc = fail(LRDMC_ERR_HIP, "upload failed");
            break;
        }
        {   // adjoint pass buffers and descriptor
            const int nth = L.nth, nsp = s.n_species;
            r.R_t = (double*)carve(M * 3 * 8);
            r.jas_t = (double*)carve((2 + nsp) * 3 * 8);
            r.btab_t = (double*)carve((size_t)Nb * 4 * 8);
            r.a_eL = (double*)carve(nw * 8);
            r.a_lp = (double*)carve(nw * 8);
            r.a_deL = (double*)carve(nw * (size_t)nth * 8);
            r.a_dlp = (double*)carve(nw * (size_t)nth * 8);
            r.a_status = (int*)carve(8);
            r.a_out = (double*)carve((3 * (size_t)nth + 2) * 8);
            (void)carve(8);
            r.dadj = (DevAdj*)carve(sizeof(DevAdj));
            r.h_R.assign(s.atom_pos, s.atom_pos + 3 * M);
            r.h_Z.assign(s.atom_charge, s.atom_charge + M);
            r.h_bexp.assign(s.basis_exp, s.basis_exp + Nb);
            r.h_batom.assign(s.basis_atom, s.basis_atom + Nb);
            r.h_jas.assign(s.jastrow, s.jastrow + 3 * (2 + nsp));
            DevAdj& ad = r.ad;
            ad.M = M; ad.Nb = Nb; ad.Norb = s.n_orb; ad.Nup = s.n_up; ad.Ndn = s.n_dn; ad.N = L.N;
            ad.ns = ns; ad.nspec = nsp; ad.nw = r.nw; ad.nth = nth; ad.nu_mode = prm->nu_opt_mode;
            ad.a = prm->a; ad.vii = vii;
            ad.R = r.R_t; ad.Z = Z; ad.rc = rcs; ad.jas = r.jas_t; ad.btab = r.btab_t; ad.C = C;
            ad.core = core; ad.spec = spec; ad.batom = batom; ad.btype = btype;
            ad.pos = r.pos[0];
            ad.eL = r.a_eL; ad.lp = r.a_lp; ad.deL = r.a_deL; ad.dlp = r.a_dlp;
            ad.status = r.a_status;
            ad.o_pos = L.a_pos; ad.o_phi = L.a_phi; ad.o_dphi = L.a_dphi; ad.o_phi6 = L.a_phi6;
            ad.o_ainv = L.a_ainv; ad.o_Z = L.a_Z; ad.o_T = L.a_T; ad.o_Y = L.a_Y; ad.o_G = L.a_G;
            ad.o_chi = L.a_chi; ad.o_gj = L.a_gj; ad.o_Lj = L.a_Lj; ad.o_dJ = L.a_dJ; ad.o_R = L.a_R;
            ad.o_Rdet = L.a_Rdet; ad.o_gd = L.a_gd; ad.o_Ld = L.a_Ld; ad.o_nu = L.a_nu;
            ad.o_nua = L.a_nua; ad.o_al = L.a_al; ad.o_sgd = L.a_sgd; ad.o_sgj = L.a_sgj;
            ad.o_sRd = L.a_sRd; ad.o_sdJ = L.a_sdJ; ad.o_snu = L.a_snu; ad.o_snua = L.a_snua;
            ad.o_GeL = L.a_GeL; ad.o_Glp = L.a_Glp; ad.o_sc = L.a_sc; ad.o_piv = L.a_piv;
            ad.lds_doubles = L.a_doubles;
        }
        if (r.kind == kKindLds) {
            DevSys d{};
            d.M = M; d.Nb = Nb; d.Norb = s.n_orb; d.Nup = s.n_up; d.Ndn = s.n_dn;
            d.N = L.N; d.P = L.P; d.ns = ns; d.nspec = s.n_species; d.nw = r.nw;
            d.has_en = has_en; d.vii = vii; d.sysid = s.system_id;
            d.jp = h->d_j; d.e0p = r.d_e0;
            d.R = R; d.Z = Z; d.rc = rcs; d.core = core; d.spec = spec; d.batom = batom;
            d.btype = btype; d.bexp = bexp; d.C = C; d.jas = jas; d.btab = btab;
            d.lw = r.lw;
            d.spill = (double*)carve(nw * L.spill_stride * 8);
            d.spill_stride = L.spill_stride;
            d.iters = r.iters; d.trace = r.trace; d.trace_cap = prm->trace_cap;
            d.o_pos = L.o_pos; d.o_R = L.o_R; d.o_Rdet = L.o_Rdet; d.o_dJ = L.o_dJ;
            d.o_Arow = L.o_Arow; d.o_AinvT = L.o_AinvT; d.o_Jg = L.o_Jg; d.o_Jl = L.o_Jl;
            d.o_nue = L.o_nue; d.o_nua = L.o_nua; d.o_dje = L.o_dje; d.o_scal = L.o_scal;
            d.ldb = L.ldb; d.o_B = L.o_B; d.o_rows = L.o_rows; d.o_tmp = L.o_tmp; d.o_C = L.o_C;
            d.bK = bK; d.o_nuc = L.o_nuc; d.o_jas = L.o_jas; d.o_gd = L.o_gd; d.o_ev = L.o_ev;
            d.lds_doubles = L.lds_doubles;
            d.s_Phi = L.s_Phi; d.s_dPhi = L.s_dPhi; d.s_Arow = L.s_Arow; d.bchunk = L.bchunk;
            d.ainv1 = L.ainv1 ? 1 : 0; d.s_AinvG = L.s_AinvG; d.s_GJ = L.s_GJ;
            d.PT = L.PT; d.necp = r.nl ? s.n_ecp : 0;
            d.ecp_atom = e_atom; d.ecp_l = e_l; d.ecp_pow = e_pow;
            d.ecp_coef = e_coef; d.ecp_exp = e_exp; d.ecp_rcut = e_rcut; d.o_Vnl = L.o_Vnl;
            d.o_nlin = L.o_nlin;
            for (int p = 0; p < 2; ++p) {
                r.dsys[p] = (DevSys*)carve(sizeof(DevSys));
                r.hsys[p] = d;
                r.hsys[p].pos = r.pos[p]; r.hsys[p].eL = r.eL[p]; r.hsys[p].Wd = r.Wd[p];
            }
        } else {
            DevMix m{};
            m.M = M; m.Nb = Nb; m.Norb = s.n_orb; m.Nup = s.n_up; m.Ndn = s.n_dn;
            m.N = L.N; m.P = L.P; m.ns = ns; m.nspec = s.n_species; m.nw = r.nw;
            m.has_en = has_en; m.vii = vii; m.sysid = s.system_id;
            m.jp = h->d_j; m.e0p = r.d_e0;
            m.gemm = prm->precision == LRDMC_MIXED_BF16 ? kGemmBF16 : kGemmFP32;
            m.R = R; m.Z = Z; m.rc = rcs; m.jas = jas; m.btab = btab;
            m.core = core; m.spec = spec; m.btype = btype;
            m.Cf = Cf; m.Cbf = Cbf; m.nb32 = L.nb32; m.fkc = L.fkc;
            m.C64 = C;
            m.s64 = (double*)carve(nw * L.stride64 * 8);
            m.stride64 = L.stride64;
            m.diag = (double*)carve(nw * 4 * 8);
            m.lw = r.lw;
            r.state[0] = (float*)carve(nw * L.m_stride * 4);
            r.state[1] = (float*)carve(nw * L.m_stride * 4);
            m.stride = L.m_stride;
            m.g_Phi = L.g_Phi; m.g_dPhi = L.g_dPhi; m.g_Arow = L.g_Arow; m.g_AinvT = L.g_AinvT;
            m.iters = r.iters; m.trace = r.trace; m.trace_cap = prm->trace_cap;
            m.l_pos = L.l_pos; m.l_nue = L.l_nue; m.l_nua = L.l_nua; m.l_scal = L.l_scal;
            m.l_red = L.l_red; m.l_U = L.l_U; m.l_R = L.l_R; m.l_Rdet = L.l_Rdet; m.l_dJ = L.l_dJ;
            m.l_gD = L.l_gD; m.l_Jg = L.l_Jg; m.l_Jl = L.l_Jl; m.l_dje = L.l_dje;
            m.l_rows = L.l_rows; m.l_tmp = L.l_tmp; m.l_F = L.l_F; m.l_ev = L.l_ev; m.l_bytes = L.l_bytes;
            for (int p = 0; p < 2; ++p) {
                r.dmix[p] = (DevMix*)carve(sizeof(DevMix));
                r.hmix[p] = m;
                r.hmix[p].pos = r.pos[p]; r.hmix[p].eL = r.eL[p]; r.hmix[p].Wd = r.Wd[p];
                r.hmix[p].state = r.state[p];
            }
            r.need_build = true;
            h->mix_order.push_back(k);
            h->mix_lds = std::max(h->mix_lds, L.lds_bytes);
            if (h->mix_sys_threads.empty()) h->mix_sys_threads.assign(n_sys, kMixThreads);
        }
        if (up(r.pos[0], ip, nw * 3 * L.N * 8) != hipSuccess ||
            hipMemsetAsync(r.lw, 0, nw * 8, h->stream) != hipSuccess) {
            rc = fail(LRDMC_ERR_HIP, "upload of walkers failed");
            break;
        }
        if (r.trace && hipMemsetAsync(r.trace, 0xfe, nw * (size_t)prm->trace_cap * 4, h->stream)) {
            rc = fail(LRDMC_ERR_HIP, "trace init failed");
            break;
        }
        ip += nw * 3 * L.N;
    }
    if (rc == LRDMC_OK && off > ws_bytes) rc = fail(LRDMC_ERR_WORKSPACE, "workspace layout overflow");
    for (auto& r : h->sys) {
        if (rc) break;
        bool bad = false;
        for (int p = 0; p < 2; ++p)
            bad = bad || (r.kind == kKindLds ? up(r.dsys[p], &r.hsys[p], sizeof(DevSys))
                                             : up(r.dmix[p], &r.hmix[p], sizeof(DevMix))) != hipSuccess;
        if (bad) rc = fail(LRDMC_ERR_HIP, "upload of system descriptors failed");
    }
    if (rc == LRDMC_OK && !h->mix_order.empty()) {
        // larger systems first: their walkers take longest
        std::stable_sort(h->mix_order.begin(), h->mix_order.end(), [&](int x, int y) {
            return h->sys[x].N > h->sys[y].N;
        });
        rc = upload_mix_tables(h);
    }
    if (rc == LRDMC_OK) {
        // allow each phase kernel the LDS that its static allocation leaves free
        // (kernel kinds: 0, 1 the FP64 kernel without and with the non-local
        // pseudopotential, 2 the FP64 large-system kernel, 3 the mixed-precision
        // kernel)
        for (int kind = 0; kind < 4 && !rc; ++kind) {
            const void* fn = kind < 3 ? (const void*)phase_kernel(h->prm.rotate != 0, kind == 1, kind == 2)
                                      : (const void*)phase_mixed;
            size_t need_lds = 0;
            for (auto& r : h->sys) {
                const int rk = r.kind != kKindLds ? 3 : (r.nl ? 1 : (r.L.big ? 2 : 0));
                if (rk == kind) need_lds = std::max(need_lds, r.L.lds_bytes);
            }
            if (!need_lds) continue;
            hipFuncAttributes fa;
            if (hipFuncGetAttributes(&fa, fn) != hipSuccess) { rc = fail(LRDMC_ERR_HIP, "hipFuncGetAttributes failed"); break; }
            const size_t dyn_max = (size_t)kMaxLdsBytes - fa.sharedSizeBytes;
            if (need_lds > dyn_max) { rc = fail(LRDMC_ERR_UNSUPPORTED, "system too large for the LDS of one workgroup"); break; }
            if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_max) != hipSuccess)
                rc = fail(LRDMC_ERR_HIP, "hipFuncSetAttribute failed");
        }
    }
    if (rc == LRDMC_OK) {
        // initial local energies: a zero-step load-balanced phase (E_0 is not
        // read by it); E_0 = their unweighted mean
        for (auto& r : h->sys) r.e0 = 0.0;
        for (auto& r : h->sys) if (!rc && up(r.d_e0, &r.e0, 8)) rc = fail(LRDMC_ERR_HIP, "upload failed");
        if (!rc) rc = reset_counters(h, h->stream);
        if (!rc) rc = launch_phases(h, h->stream, 0, 0, true);
        for (auto& r : h->sys) {
            if (rc) break;
            std::vector<double> eL(r.nw);
            if (hipMemcpyAsync(eL.data(), r.eL[0], r.nw * 8, hipMemcpyDeviceToHost, h->stream) ||
                hipStreamSynchronize(h->stream)) {
                rc = fail(LRDMC_ERR_HIP, "init evaluation failed");
                break;
            }
            double acc = 0.0;
            int nbad = 0, first = -1;
            for (int w = 0; w < r.nw; ++w) {
                acc += eL[w];
                if (!std::isfinite(eL[w])) { if (first < 0) first = w; ++nbad; }
            }
            r.e0 = acc / r.nw;
#ifdef LRDMC_DEBUG_KEEP_NONFINITE
            if (nbad) { std::fprintf(stderr, "debug: system %d: %d non-finite, first %d\n", (int)(&r - h->sys.data()), nbad, first); nbad = 0; r.e0 = eL[0]; }
#endif
            if (nbad)
                rc = fail(LRDMC_ERR_SINGULAR,
                          "non-finite initial local energy: system " +
                              std::to_string(&r - h->sys.data()) + ", " + std::to_string(nbad) +
                              " walkers, first " + std::to_string(first));
            else if (up(r.d_e0, &r.e0, 8)) rc = fail(LRDMC_ERR_HIP, "upload failed");
        }
        unsigned long long cnt[kCntLen];
        if (!rc && (hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream) !=
                        hipSuccess ||
                    hipStreamSynchronize(h->stream) != hipSuccess))
            rc = fail(LRDMC_ERR_HIP, "counter readback failed");
        if (!rc && cnt[kCntSingular]) rc = fail(LRDMC_ERR_SINGULAR, "singular Slater matrix at init");
    }
    if (rc) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipEventDestroy(h->ev0); (void)hipEventDestroy(h->ev1);
        delete h;
        return rc;
    }
#ifdef LRDMC_SECTION_TIMERS
    if (hipMalloc((void**)&h->timers, (size_t)h->sys[0].nw * 8 * 8) != hipSuccess) h->timers = nullptr;
#endif
    *out = h;
    return LRDMC_OK;
}

#ifdef LRDMC_SECTION_TIMERS
// instrumentation builds only: per-walker section cycle counts of the last phase
int lrdmc_section_timers(lrdmc_handle* h, unsigned long long* out)
{
    if (!h || !h->timers) return fail(LRDMC_ERR_INVALID_ARG, "no timers");
    HIPCHK(hipMemcpy(out, h->timers, (size_t)h->sys[0].nw * 64, hipMemcpyDeviceToHost));
    return LRDMC_OK;
}
#endif

int lrdmc_step(lrdmc_handle* h, lrdmc_step_stats* st)
{
    if (!h) return fail(LRDMC_ERR_INVALID_ARG, "null handle");
    int rc = reset_counters(h, h->stream);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    if ((rc = launch_phases(h, h->stream, h->parity, -1, true))) return rc;
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    if (st) {
        HIPCHK(hipStreamSynchronize(h->stream));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        return read_counters(h, st, ms);
    }
    return LRDMC_OK;
}

int lrdmc_branch(lrdmc_handle* h, lrdmc_branch_stats* st)
{
    if (!h) return fail(LRDMC_ERR_INVALID_ARG, "null handle");
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    int rc = enqueue_branch(h, h->stream, h->parity);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    h->parity ^= 1;
    h->j++;
    rc = drain(h);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    if (st) fill_branch_stats(h, st, ms);
    return rc;
}

int lrdmc_run(lrdmc_handle* h, int n_branchings, lrdmc_step_stats* st, lrdmc_branch_stats* bst)
{
    if (!h || n_branchings < 1) return fail(LRDMC_ERR_INVALID_ARG, "bad arguments");
    bool pending = false;
    for (auto& r : h->sys) pending = pending || r.need_build;
    int rc = reset_counters(h, h->stream);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    int done = 0;
    if (pending) {   // a rebuild of the orbital data is not part of the captured cycle
        if ((rc = launch_phases(h, h->stream, h->parity, -1, true))) return rc;
        if ((rc = enqueue_branch(h, h->stream, h->parity))) return rc;
        h->parity ^= 1; h->j++; done = 1;
    }
    if (done < n_branchings && (rc = capture_graphs(h))) return rc;
    for (; done < n_branchings; ++done) {
        HIPCHK(hipGraphLaunch(h->gexec[h->parity], h->stream));
        h->parity ^= 1;
        h->j++;
        if ((done + 1) % (kHistCap / 2) == 0 && (rc = drain(h))) return rc;
    }
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    rc = drain(h);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    if (st) { const int rc2 = read_counters(h, st, ms); if (!rc) rc = rc2; }
    if (bst) fill_branch_stats(h, bst, ms);
    return rc;
}

// Autotuner of the mixed-precision launch: workgroup size (64, 128 or 256
// threads per walker) x order of the systems in the launch, each candidate timed on a
// copy of the current walkers (the other slot) for n_steps and 2 n_steps
// load-balanced steps; the one with the shortest projected full phase is
// kept.  Stream-synchronous.
int lrdmc_autotune(lrdmc_handle* h, int n_steps, lrdmc_tune_entry* log, int log_cap, int* n_log)
{
    if (!h || n_steps < 1) return fail(LRDMC_ERR_INVALID_ARG, "bad arguments");
    if (n_log) *n_log = 0;
    if (h->mix_order.empty()) return LRDMC_OK;
    for (auto& r : h->sys)
        if (r.need_build) return fail(LRDMC_ERR_INVALID_ARG, "run one phase before tuning");
    const int p = h->parity, q = p ^ 1;
    // candidate orders: largest systems first, smallest first
    std::vector<int> big = h->mix_order, small;
    std::stable_sort(big.begin(), big.end(), [&](int x, int y) { return h->sys[x].N > h->sys[y].N; });
    small.assign(big.rbegin(), big.rend());
    const std::vector<std::vector<int>> orders = big.size() > 1 ? std::vector<std::vector<int>>{big, small}
                                                                : std::vector<std::vector<int>>{big};
    const int threads[3] = {256, 128, 64};
    const std::vector<int> keep_order = h->mix_order;
    const int keep_threads = h->mix_threads, keep_sep = h->mix_separate;
    const std::vector<int> keep_sys_threads = h->mix_sys_threads;
    float best = 1e30f;
    int best_t = keep_threads;
    std::vector<int> best_o = keep_order;
    h->tune_log.clear();
    int rc = LRDMC_OK;
    const int steps_full = h->prm.scheme == LRDMC_SCHEME_LB
                               ? h->prm.n_proj
                               : std::max(1, (int)(h->prm.tau * 3.0 * maxN_all(h) / (h->prm.a * h->prm.a)));
    // the tuning phases update the log-weights in place: keep them
    for (int k : h->mix_order) {
        SysRun& r = h->sys[k];
        HIPCHK(hipMemcpyAsync(r.cum, r.lw, (size_t)r.nw * 8, hipMemcpyDeviceToDevice, h->stream));
    }
    // projected time of a full phase of one launch configuration: two tuning
    // phases of n_steps and 2 n_steps on copies of the walkers in the other
    // slot; the difference is the per-step cost, the rest the fixed cost of a
    // phase (refresh, FP64 estimator evaluation)
    auto project = [&](int only, int thr, float& ms_full) -> int {
        float tms[2] = {0.f, 0.f};
        for (int rep = 0; rep < 2; ++rep) {
            for (int k : h->mix_order) {
                if (only >= 0 && k != only) continue;
                SysRun& r = h->sys[k];
                const size_t nw = r.nw;
                if (hipMemcpyAsync(r.pos[q], r.pos[p], nw * 3 * r.N * 8, hipMemcpyDeviceToDevice, h->stream) ||
                    hipMemcpyAsync(r.state[q], r.state[p], nw * r.L.m_stride * 4, hipMemcpyDeviceToDevice, h->stream))
                    return fail(LRDMC_ERR_HIP, "tuning copy failed");
            }
            HIPCHK(hipEventRecord(h->ev0, h->stream));
            int rc1 = launch_mixed(h, h->stream, q, n_steps * (rep + 1), 0, 0, only, thr);
            if (rc1) return rc1;
            HIPCHK(hipEventRecord(h->ev1, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            HIPCHK(hipEventElapsedTime(&tms[rep], h->ev0, h->ev1));
        }
        const float per_step = std::max(0.f, (tms[1] - tms[0]) / n_steps);
        const float fixed = std::max(0.f, tms[0] - per_step * n_steps);
        ms_full = fixed + per_step * steps_full;
        return LRDMC_OK;
    };
    // one launch for all systems: workgroup size x order
    for (size_t oi = 0; oi < orders.size() && !rc; ++oi)
        for (int ti = 0; ti < 3 && !rc; ++ti) {
            h->mix_order = orders[oi];
            h->mix_threads = threads[ti];
            if ((rc = upload_mix_tables(h))) break;
            float ms_full = 0.f;
            if ((rc = project(-1, 0, ms_full))) break;
            lrdmc_tune_entry e;
            e.threads = h->mix_threads;
            e.order_big_first = (oi == 0) ? 1 : 0;
            e.ms = ms_full;
            e.system = -1;
            h->tune_log.push_back(e);
            if (ms_full < best) { best = ms_full; best_t = h->mix_threads; best_o = h->mix_order; }
        }
    // one launch per system, each with its fastest workgroup size (with a
    // single system this is the batched launch again)
    std::vector<int> sep_threads(h->sys.size(), kMixThreads);
    float sep_total = 0.f;
    if (!rc && h->mix_order.size() > 1) {
        h->mix_order = best_o;
        rc = upload_mix_tables(h);
        for (int k : best_o) {
            if (rc) break;
            float bk = 1e30f;
            for (int ti = 0; ti < 3 && !rc; ++ti) {
                float ms_full = 0.f;
                if ((rc = project(k, threads[ti], ms_full))) break;
                lrdmc_tune_entry e;
                e.threads = threads[ti];
                e.order_big_first = 0;
                e.ms = ms_full;
                e.system = k;
                h->tune_log.push_back(e);
                if (ms_full < bk) { bk = ms_full; sep_threads[k] = threads[ti]; }
            }
            sep_total += bk;
        }
        if (!rc) {
            lrdmc_tune_entry e;
            e.threads = 0;
            e.order_big_first = 0;
            e.ms = sep_total;
            e.system = -2;
            h->tune_log.push_back(e);
        }
    }
    const bool use_sep = !rc && h->mix_order.size() > 1 && sep_total < best;
    for (int k : keep_order) {
        SysRun& r = h->sys[k];
        if (hipMemcpyAsync(r.lw, r.cum, (size_t)r.nw * 8, hipMemcpyDeviceToDevice, h->stream) && !rc)
            rc = fail(LRDMC_ERR_HIP, "restoring the log-weights failed");
    }
    h->mix_order = rc ? keep_order : best_o;
    h->mix_threads = rc ? keep_threads : best_t;
    h->mix_separate = rc ? keep_sep : (use_sep ? 1 : 0);
    h->mix_sys_threads = rc ? keep_sys_threads : sep_threads;
    const int rc2 = upload_mix_tables(h);
    drop_graphs(h);
    (void)reset_counters(h, h->stream);
    if (log && n_log) {
        const int n = std::min(log_cap, (int)h->tune_log.size());
        for (int k = 0; k < n; ++k) log[k] = h->tune_log[k];
        *n_log = n;
    }
    return rc ? rc : rc2;
}

int lrdmc_set_launch(lrdmc_handle* h, int threads, int order_big_first)
{
    if (!h || (threads != 0 && threads != 64 && threads != 128 && threads != 256))
        return fail(LRDMC_ERR_INVALID_ARG, "threads must be 0, 64, 128 or 256");
    std::stable_sort(h->mix_order.begin(), h->mix_order.end(), [&](int x, int y) {
        return order_big_first ? h->sys[x].N > h->sys[y].N : h->sys[x].N < h->sys[y].N;
    });
    if (threads) h->mix_threads = threads;
    h->mix_separate = threads == 0 ? 1 : 0;
    drop_graphs(h);
    return upload_mix_tables(h);
}

int lrdmc_energy_forces(lrdmc_handle* h, lrdmc_energy* e, double* forces, double* jgrad)
{
    if (!h || !e) return fail(LRDMC_ERR_INVALID_ARG, "null argument");
    if (forces || jgrad) {
        // per-walker derivatives at the current population, then the weighted
        // population sums on the device
        SysRun& r = h->sys[0];
        int rc = run_derivs(h, 0, nullptr, nullptr, nullptr, nullptr, nullptr);
        if (rc) return rc;
        const int nth = r.L.nth, M = r.ad.M;
        hipLaunchKernelGGL(derivs_reduce, dim3(3 * nth + 2), dim3(256), 0, h->stream, r.nw, nth,
                           h->prm.scheme == LRDMC_SCHEME_LB ? 0 : 1, (const double*)r.lw,
                           (const double*)r.Wd[h->parity], (const double*)r.d_e0,
                           (const double*)r.a_eL, (const double*)r.a_deL, (const double*)r.a_dlp,
                           r.a_out);
        HIPCHK(hipGetLastError());
        std::vector<double> o(3 * (size_t)nth + 2);
        HIPCHK(hipMemcpyAsync(o.data(), r.a_out, o.size() * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        const double S = o[0], E = o[1] / S;
        if (!(S > 0)) return fail(LRDMC_ERR_ALL_DEAD, "every walker weight is zero");
        for (int q = 0; q < nth; ++q) {
            const double g = o[2 + q] / S + 2.0 * (o[2 + nth + q] / S - E * o[2 + 2 * nth + q] / S);
            if (q < 3 * M) { if (forces) forces[q] = -g; }
            else if (jgrad) jgrad[q - 3 * M] = g;
        }
    }
    const SysRun& r = h->sys[0];
    const int n = (int)r.hist_e.size(), p = std::max(0, h->prm.p_corr);
    const int start = std::max(p, h->prm.n_therm > 0 ? h->prm.n_therm : n / 10);
    e->energy = NAN; e->sigma = NAN; e->n_used = 0;
    if (start >= n) return LRDMC_OK;
    std::vector<double> lg(n - start), g(n - start);
    double mx = -INFINITY;
    for (int k = start; k < n; ++k) {
        double s = 0.0;
        for (int q = k - p; q < k; ++q) s += r.hist_lwb[q];
        lg[k - start] = s;
        mx = std::max(mx, s);
    }
    double num = 0.0, den = 0.0;
    for (int k = start; k < n; ++k) {
        g[k - start] = std::exp(lg[k - start] - mx);
        num += g[k - start] * r.hist_e[k];
        den += g[k - start];
    }
    e->energy = num / den;
    const int m = n - start, block = std::max(1, m / 10), nb = m / block;
    e->n_used = m;
    if (nb >= 2) {
        std::vector<double> eb(nb);
        double mean = 0.0;
        for (int b = 0; b < nb; ++b) {
            double a = 0.0, c = 0.0;
            for (int q = b * block; q < (b + 1) * block; ++q) { a += g[q] * r.hist_e[start + q]; c += g[q]; }
            eb[b] = a / c;
            mean += eb[b];
        }
        mean /= nb;
        double var = 0.0;
        for (double x : eb) var += (x - mean) * (x - mean);
        e->sigma = std::sqrt(var / (nb - 1) / nb);
    }
    return LRDMC_OK;
}

int lrdmc_n_theta(lrdmc_handle* h, int isys)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size()) return fail(LRDMC_ERR_INVALID_ARG, "bad handle/system");
    return h->sys[isys].L.nth;
}

// Adjoint pass over the walkers of system isys at their current positions,
// with the system's parameters replaced by theta (host, n_theta) when given.
static int run_derivs(lrdmc_handle* h, int isys, const double* theta, double* eL, double* lp,
                      double* deL, double* dlp)
{
    SysRun& r = h->sys[isys];
    const Layout& L = r.L;
    if (h->prm.rotate)
        return fail(LRDMC_ERR_UNSUPPORTED, "the adjoint pass evaluates the fixed lattice axes only");
    if (r.nl)
        return fail(LRDMC_ERR_UNSUPPORTED, "the adjoint pass has no non-local pseudopotential");
    const size_t lds = (size_t)L.a_doubles * 8;
    hipFuncAttributes fa;
    HIPCHK(hipFuncGetAttributes(&fa, (const void*)walker_derivs));
    if (lds + fa.sharedSizeBytes > (size_t)kMaxLdsBytes)
        return fail(LRDMC_ERR_UNSUPPORTED, "system too large for the LDS layout of the adjoint pass");
    HIPCHK(hipFuncSetAttribute((const void*)walker_derivs, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMaxLdsBytes - fa.sharedSizeBytes)));
    const int M = r.ad.M, Nb = r.ad.Nb, nj = 3 * (2 + r.ad.nspec);
    std::vector<double> R(r.h_R), jas(r.h_jas);
    if (theta) {
        for (int q = 0; q < 3 * M + nj; ++q)
            if (!std::isfinite(theta[q])) return fail(LRDMC_ERR_INVALID_ARG, "non-finite theta");
        for (int q = 0; q < 3 * M; ++q) R[q] = theta[q];
        for (int q = 0; q < nj; ++q) jas[q] = theta[3 * M + q];
    }
    std::vector<double> btab((size_t)Nb * 4);
    for (int mu = 0; mu < Nb; ++mu) {
        for (int c = 0; c < 3; ++c) btab[4 * mu + c] = R[3 * r.h_batom[mu] + c];
        btab[4 * mu + 3] = r.h_bexp[mu];
    }
    double vii = 0.0;
    for (int I = 0; I < M; ++I)
        for (int J = I + 1; J < M; ++J) {
            const double dx = R[3 * I] - R[3 * J], dy = R[3 * I + 1] - R[3 * J + 1],
                         dz = R[3 * I + 2] - R[3 * J + 2];
            vii += r.h_Z[I] * r.h_Z[J] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
    DevAdj ad = r.ad;
    ad.vii = vii;
    ad.pos = r.pos[h->parity];
    if (eL) ad.eL = eL;
    if (lp) ad.lp = lp;
    if (deL) ad.deL = deL;
    if (dlp) ad.dlp = dlp;
    int zero = 0, nbad = 0;
    HIPCHK(hipMemcpyAsync(r.R_t, R.data(), R.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(r.jas_t, jas.data(), jas.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(r.btab_t, btab.data(), btab.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(r.a_status, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(r.dadj, &ad, sizeof(DevAdj), hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(walker_derivs, dim3(r.nw), dim3(kAdjThreads), lds, h->stream,
                       (const DevAdj*)r.dadj);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&nbad, r.a_status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (nbad) return fail(LRDMC_ERR_SINGULAR, "singular Slater matrix in the adjoint pass");
    return LRDMC_OK;
}

int lrdmc_walker_derivs(lrdmc_handle* h, int isys, const double* theta, double* eL, double* logpsi,
                        double* deL, double* dlogpsi)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size()) return fail(LRDMC_ERR_INVALID_ARG, "bad handle/system");
    return run_derivs(h, isys, theta, eL, logpsi, deL, dlogpsi);
}

int lrdmc_get_walkers(lrdmc_handle* h, int isys, double* pos, double* lw, double* eL, double* W,
                      int32_t* iters, int32_t* sel, int32_t* trace)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size()) return fail(LRDMC_ERR_INVALID_ARG, "bad handle/system");
    const SysRun& r = h->sys[isys];
    const int p = h->parity;
    const size_t nw = r.nw;
    auto dn = [&](void* dst, const void* src, size_t b) {
        return dst ? hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, h->stream) : hipSuccess;
    };
    if (dn(pos, r.pos[p], nw * 3 * r.N * 8) || dn(lw, r.lw, nw * 8) || dn(eL, r.eL[p], nw * 8) ||
        dn(W, r.Wd[p], nw * 8) || dn(iters, r.iters, nw * 4) || dn(sel, r.sel, nw * 4))
        return fail(LRDMC_ERR_HIP, "device-to-host copy failed");
    if (trace) {
        if (!r.trace) return fail(LRDMC_ERR_INVALID_ARG, "tracing is off (trace_cap = 0)");
        HIPCHK(hipMemcpyAsync(trace, r.trace, nw * (size_t)h->prm.trace_cap * 4, hipMemcpyDeviceToHost,
                              h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return LRDMC_OK;
}

int lrdmc_get_precision_report(lrdmc_handle* h, int isys, double* out)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size() || !out)
        return fail(LRDMC_ERR_INVALID_ARG, "bad arguments");
    const SysRun& r = h->sys[isys];
    if (r.kind != kKindMixed)
        return fail(LRDMC_ERR_INVALID_ARG, "the FP64 walker layout has no precision report");
    HIPCHK(hipMemcpyAsync(out, r.hmix[0].diag, (size_t)r.nw * 4 * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LRDMC_OK;
}

int lrdmc_set_walkers(lrdmc_handle* h, int isys, const double* pos, const double* lw)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size() || !pos)
        return fail(LRDMC_ERR_INVALID_ARG, "bad arguments");
    SysRun& r = h->sys[isys];
    const size_t nw = r.nw;
    HIPCHK(hipMemcpyAsync(r.pos[h->parity], pos, nw * 3 * r.N * 8, hipMemcpyHostToDevice, h->stream));
    if (lw) HIPCHK(hipMemcpyAsync(r.lw, lw, nw * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    r.need_build = r.kind == kKindMixed;   // mixed layout: orbital data follow the positions
    return LRDMC_OK;
}

double lrdmc_get_e0(lrdmc_handle* h, int isys)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size()) { g_err = "bad handle/system"; return NAN; }
    return h->sys[isys].e0;
}

int lrdmc_set_e0(lrdmc_handle* h, int isys, double e0)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size()) return fail(LRDMC_ERR_INVALID_ARG, "bad handle/system");
    SysRun& r = h->sys[isys];
    r.e0 = e0;
    HIPCHK(hipMemcpyAsync(r.d_e0, &r.e0, 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LRDMC_OK;
}

int lrdmc_reconfigure_noalloc(int scheme, int nw, const double* lw, const double* eL,
                              const double* W, double e0, uint64_t seed, uint64_t sysid, int j,
                              int32_t* sel, double* out, void* stream)
{
    int rc = check_reconf_args(scheme, nw, lw, eL, W, sel, out);
    if (rc) return rc;
    if (nw > LRDMC_NOALLOC_MAX_WALKERS)
        return fail(LRDMC_ERR_INVALID_ARG, "nw = " + std::to_string(nw) +
                                               " exceeds LRDMC_NOALLOC_MAX_WALKERS = " +
                                               std::to_string(LRDMC_NOALLOC_MAX_WALKERS));
    double* scr = nullptr;
    if ((rc = noalloc_scratch(&scr))) return rc;
    return enqueue_reconfigure(scheme, nw, lw, eL, W, e0, seed, sysid, j, sel, out, scr,
                               (hipStream_t)stream);
}

int lrdmc_get_branch_index(lrdmc_handle* h) { return h ? h->j : -1; }

size_t lrdmc_reconfigure_workspace_bytes(int nw)
{
    if (nw < 1) { (void)fail(LRDMC_ERR_INVALID_ARG, "nw must be positive"); return 0; }
    return (size_t)reconf_scratch_doubles(nw) * 8;
}

int lrdmc_reconfigure(int scheme, int nw, const double* lw, const double* eL, const double* W,
                      double e0, uint64_t seed, uint64_t sysid, int j, int32_t* sel, double* out,
                      void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_reconf_args(scheme, nw, lw, eL, W, sel, out);
    if (rc) return rc;
    if (!ws) return fail(LRDMC_ERR_INVALID_ARG, "null workspace");
    if (ws_bytes < (size_t)reconf_scratch_doubles(nw) * 8)
        return fail(LRDMC_ERR_WORKSPACE, "workspace smaller than lrdmc_reconfigure_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(LRDMC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    return enqueue_reconfigure(scheme, nw, lw, eL, W, e0, seed, sysid, j, sel, out,
                               static_cast<double*>(ws), (hipStream_t)stream);
}


void lrdmc_destroy(lrdmc_handle* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    delete h;
}

}  // extern "C"
