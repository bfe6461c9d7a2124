// Host side of the C ABI declared in include/lrdmc.h: validation, workspace
// carving, kernel launches on the caller's stream, and the host-level pieces
// of the method (E_0 update after each branching, Algorithm 2; the
// correcting-factor energy estimate and its blocking error bar, Sec. II.A).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lrdmc.h"
#include "lrdmc_dev.hpp"

namespace lrdmc {
__global__ void phase_fp64(const DevSys* __restrict__ sys, PhaseArgs pa);
__global__ void branch_scan(DevSys s, int scheme, double E0, double* cum, double* out);
__global__ void branch_comb(DevSys s, uint64_t seed, int j, const double* cum, const double* out,
                            int32_t* sel);
__global__ void branch_count(const int32_t* sel, int nw, int* n_distinct);
__global__ void branch_gather(DevSys s, const int32_t* sel, const double* pos_old,
                              const double* eL_old, const double* W_old);
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

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Per-system sizes and layout, computed identically by workspace_bytes and init.
struct Layout {
    int N, P, ns;
    // LDS offsets (doubles)
    int o_pos, o_R, o_Rdet, o_dJ, o_Arow, o_AinvT, o_Jg, o_Jl, o_nue, o_nua, o_dje, o_scal, o_B,
        o_rows, o_tmp, o_C, lds_doubles;
    int s_Phi, s_dPhi;
    long spill_stride;
    // workspace bytes of each device array
    size_t b_sys, b_state;
};

Layout make_layout(const lrdmc_system& s, const lrdmc_params& p)
{
    Layout L{};
    L.N = s.n_up + s.n_dn;
    L.P = 6 * L.N;
    L.ns = std::max(1, std::max(s.n_up, s.n_dn));
    int o = 0;
    auto take = [&](int n) { int r = o; o += (n + 1) / 2 * 2; return r; };
    L.o_pos = take(3 * L.N);
    L.o_R = take(L.P);
    L.o_Rdet = take(L.P);
    L.o_dJ = take(L.P);
    L.o_Arow = take(L.N * L.ns);
    L.o_AinvT = take(2 * L.ns * L.ns);
    L.o_Jg = take(3 * L.N);
    L.o_Jl = take(L.N);
    L.o_nue = take(L.N);
    L.o_nua = take(L.N);
    L.o_dje = take(L.N);
    L.o_scal = take(kScLen);
    L.o_B = take(std::max(std::max(11 * s.n_basis, 2 * L.ns * L.ns), 7 * L.N));
    L.o_rows = take(11 * L.ns);
    L.o_tmp = take(3 * L.ns + 8);
    L.o_C = take(s.n_basis * L.ns);
    L.lds_doubles = o;
    L.s_Phi = 0;
    L.s_dPhi = L.P * L.ns;
    L.spill_stride = (long)(align_up((size_t)(L.P * L.ns + 4 * L.N * L.ns) * 8) / 8);
    const int M = s.n_atoms, Nb = s.n_basis;
    L.b_sys = align_up(M * 3 * 8) + 2 * align_up(M * 8) + 2 * align_up(M * 4) + 2 * align_up(Nb * 4) +
              align_up(Nb * 8) + align_up((size_t)Nb * s.n_orb * 8) +
              align_up((2 + s.n_species) * 3 * 8) + align_up((size_t)Nb * 4 * 8);
    const size_t nw = s.n_walkers;
    L.b_state = 2 * align_up(nw * 3 * L.N * 8)      // positions, double-buffered
                + align_up(nw * 8)                  // lw
                + 4 * align_up(nw * 8)              // eL, W double-buffered
                + align_up(nw * L.spill_stride * 8) // spill
                + 2 * align_up(nw * 4)              // iters, sel
                + align_up(nw * 8)                  // cumulative weights
                + align_up(8 * 8)                   // branch outputs
                + align_up(8)                       // distinct counter
                + 2 * align_up(sizeof(DevSys))      // device copies of the descriptor
                + (p.trace_cap > 0 ? align_up(nw * (size_t)p.trace_cap * 4) : 0);
    (void)p;
    return L;
}

std::string validate(const lrdmc_system* sys, int n_sys, const lrdmc_params* prm)
{
    if (!sys || n_sys < 1) return "no systems";
    if (!prm) return "null params";
    if (prm->scheme != LRDMC_SCHEME_LB && prm->scheme != LRDMC_SCHEME_CONV) return "bad scheme";
    if (prm->precision != LRDMC_FP64) return "only LRDMC_FP64 precision is available";
    if (!(prm->a > 0)) return "lattice space a must be > 0";
    if (prm->scheme == LRDMC_SCHEME_CONV && !(prm->tau > 0)) return "tau must be > 0";
    if (prm->scheme == LRDMC_SCHEME_LB && prm->n_proj < 1) return "n_proj must be >= 1";
    if (prm->refresh_every < 1) return "refresh_every must be >= 1";
    if (prm->nu_opt_mode < 0 || prm->nu_opt_mode > 2) return "bad nu_opt_mode";
    if (prm->trace_cap < 0) return "bad trace_cap";
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
        const Layout L = make_layout(s, *prm);
        if ((size_t)L.lds_doubles * 8 > (size_t)kMaxLdsBytes)
            return "system too large for the LDS-resident walker layout";
        if (s.n_walkers > (1 << 24)) return "too many walkers";
    }
    return "";
}

struct SysRun {
    DevSys d;             // current buffers
    DevSys* dsys[2];      // device copies of d for the two buffer parities
    DevSys hsys[2];       // their host sources
    int parity;
    double *pos_alt, *eL_alt, *W_alt;
    double *cum, *bout;
    int32_t* sel;
    int* ndist;
    Layout L;
    double e0;
    std::vector<double> hist_lwb, hist_e;
    std::vector<double> btab_host;
    size_t lds_bytes;
};

}  // namespace

struct lrdmc_handle {
    std::vector<SysRun> sys;
    lrdmc_params prm;
    hipStream_t stream;
    int j;
    unsigned long long* counters;   // [kCntLen] device
    unsigned long long cnt_init[kCntLen];   // host source of the counter reset
    hipEvent_t ev0, ev1;
    unsigned long long* timers = nullptr;   // instrumentation builds: [nw][8]
};

extern "C" {

const char* lrdmc_last_error(void) { return g_err.c_str(); }

size_t lrdmc_workspace_bytes(const lrdmc_system* sys, int n_sys, const lrdmc_params* prm)
{
    const std::string v = validate(sys, n_sys, prm);
    if (!v.empty()) { g_err = v; return 0; }
    size_t tot = align_up(kCntLen * 8);
    for (int k = 0; k < n_sys; ++k) {
        const Layout L = make_layout(sys[k], *prm);
        tot += L.b_sys + L.b_state;
    }
    return tot;
}

// Termination bound of the conventional loop: 1000 times the mean number of
// moves tau * 3N/a^2 (plus a floor).  Reaching it is counted and reported.
static int conv_cap(const lrdmc_params& p, int N)
{
    const double mean = p.tau * 3.0 * N / (p.a * p.a);
    const double cap = 1000.0 * mean + 10000.0;
    return cap > 2e9 ? 2000000000 : (int)cap;
}

static int launch_phase(lrdmc_handle* h, SysRun& r)
{
    PhaseArgs pa{};
    pa.scheme = h->prm.scheme;
    pa.nproj = h->prm.n_proj;
    pa.j = h->j;
    pa.refresh_every = h->prm.refresh_every;
    pa.nu_mode = h->prm.nu_opt_mode;
    pa.conv_cap = conv_cap(h->prm, r.d.N);
    pa.a = h->prm.a;
    pa.tau = h->prm.tau;
    pa.E0 = r.e0;
    pa.seed = h->prm.seed;
    pa.counters = h->counters;
    pa.timers = h->timers;
    hipLaunchKernelGGL(phase_fp64, dim3(r.d.nw), dim3(kWave), r.lds_bytes, h->stream,
                       (const DevSys*)r.dsys[r.parity], pa);
    HIPCHK(hipGetLastError());
    return LRDMC_OK;
}

static int reset_counters(lrdmc_handle* h)
{
    for (int k = 0; k < kCntLen; ++k) h->cnt_init[k] = (k == kCntMinIters) ? ~0ull : 0ull;
    HIPCHK(hipMemcpyAsync(h->counters, h->cnt_init, sizeof(h->cnt_init), hipMemcpyHostToDevice,
                          h->stream));
    return LRDMC_OK;
}

int lrdmc_init_system(const lrdmc_system* sys, int n_sys, const lrdmc_params* prm,
                      const double* init_pos, void* dev_workspace, size_t ws_bytes, void* stream,
                      lrdmc_handle** out)
{
    if (!out) return fail(LRDMC_ERR_INVALID_ARG, "null handle pointer");
    *out = nullptr;
    const std::string v = validate(sys, n_sys, prm);
    if (!v.empty()) return fail(v.find("too large") != std::string::npos ? LRDMC_ERR_UNSUPPORTED
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
    char* base = (char*)dev_workspace;
    size_t off = 0;
    auto carve = [&](size_t bytes) { void* p = base + off; off += align_up(bytes); return p; };
    h->counters = (unsigned long long*)carve(kCntLen * 8);
    hipError_t e1 = hipEventCreate(&h->ev0), e2 = hipEventCreate(&h->ev1);
    if (e1 != hipSuccess || e2 != hipSuccess) { delete h; return fail(LRDMC_ERR_HIP, "hipEventCreate"); }

    auto up = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream);
    };
    const double* ip = init_pos;
    int rc = LRDMC_OK;
    for (int k = 0; k < n_sys && rc == LRDMC_OK; ++k) {
        const lrdmc_system& s = sys[k];
        SysRun r{};
        r.L = make_layout(s, *prm);
        const Layout& L = r.L;
        DevSys& d = r.d;
        d.M = s.n_atoms; d.Nb = s.n_basis; d.Norb = s.n_orb; d.Nup = s.n_up; d.Ndn = s.n_dn;
        d.N = L.N; d.P = L.P; d.ns = L.ns; d.nspec = s.n_species; d.nw = s.n_walkers;
        d.sysid = s.system_id;
        d.has_en = 0;
        for (int q = 0; q < s.n_species; ++q)
            if (s.jastrow[3 * (2 + q)] != 0.0 || s.jastrow[3 * (2 + q) + 1] != 0.0) d.has_en = 1;
        double vii = 0.0;
        for (int I = 0; I < s.n_atoms; ++I)
            for (int J = I + 1; J < s.n_atoms; ++J) {
                const double* A = s.atom_pos + 3 * I;
                const double* B = s.atom_pos + 3 * J;
                const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
                vii += s.atom_charge[I] * s.atom_charge[J] / std::sqrt(dx * dx + dy * dy + dz * dz);
            }
        d.vii = vii;
        const int M = s.n_atoms, Nb = s.n_basis;
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
            up(btab, r.btab_host.data(), (size_t)Nb * 32)) {
            rc = fail(LRDMC_ERR_HIP, "upload of system arrays failed");
            break;
        }
        d.R = R; d.Z = Z; d.rc = rcs; d.core = core; d.spec = spec; d.batom = batom;
        d.btype = btype; d.bexp = bexp; d.C = C; d.jas = jas; d.btab = btab;
        const size_t nw = s.n_walkers;
        d.pos = (double*)carve(nw * 3 * L.N * 8);
        r.pos_alt = (double*)carve(nw * 3 * L.N * 8);
        d.lw = (double*)carve(nw * 8);
        d.eL = (double*)carve(nw * 8);
        r.eL_alt = (double*)carve(nw * 8);
        d.Wd = (double*)carve(nw * 8);
        r.W_alt = (double*)carve(nw * 8);
        d.spill = (double*)carve(nw * L.spill_stride * 8);
        d.spill_stride = L.spill_stride;
        d.iters = (int32_t*)carve(nw * 4);
        r.sel = (int32_t*)carve(nw * 4);
        r.cum = (double*)carve(nw * 8);
        r.bout = (double*)carve(8 * 8);
        r.ndist = (int*)carve(8);
        d.trace_cap = prm->trace_cap;
        d.trace = prm->trace_cap > 0 ? (int32_t*)carve(nw * (size_t)prm->trace_cap * 4) : nullptr;
        d.o_pos = L.o_pos; d.o_R = L.o_R; d.o_Rdet = L.o_Rdet; d.o_dJ = L.o_dJ;
        d.o_Arow = L.o_Arow; d.o_AinvT = L.o_AinvT; d.o_Jg = L.o_Jg; d.o_Jl = L.o_Jl;
        d.o_nue = L.o_nue; d.o_nua = L.o_nua; d.o_dje = L.o_dje; d.o_scal = L.o_scal;
        d.o_B = L.o_B; d.o_rows = L.o_rows; d.o_tmp = L.o_tmp; d.o_C = L.o_C;
        d.lds_doubles = L.lds_doubles;
        d.s_Phi = L.s_Phi; d.s_dPhi = L.s_dPhi;
        r.lds_bytes = (size_t)L.lds_doubles * 8;
        r.dsys[0] = (DevSys*)carve(sizeof(DevSys));
        r.dsys[1] = (DevSys*)carve(sizeof(DevSys));
        r.parity = 0;
        if (up(d.pos, ip, nw * 3 * L.N * 8) != hipSuccess ||
            hipMemsetAsync(d.lw, 0, nw * 8, h->stream) != hipSuccess) {
            rc = fail(LRDMC_ERR_HIP, "upload of walkers failed");
            break;
        }
        if (d.trace && hipMemsetAsync(d.trace, 0xfe, nw * (size_t)prm->trace_cap * 4, h->stream)) {
            rc = fail(LRDMC_ERR_HIP, "trace init failed");
            break;
        }
        ip += nw * 3 * L.N;
        h->sys.push_back(r);
        SysRun& rr = h->sys.back();
        rr.hsys[0] = rr.d;
        rr.hsys[1] = rr.d;
        rr.hsys[1].pos = rr.pos_alt; rr.hsys[1].eL = rr.eL_alt; rr.hsys[1].Wd = rr.W_alt;
    }
    if (rc == LRDMC_OK && off > ws_bytes) rc = fail(LRDMC_ERR_WORKSPACE, "workspace layout overflow");
    for (auto& r : h->sys) {
        if (rc) break;
        if (up(r.dsys[0], &r.hsys[0], sizeof(DevSys)) || up(r.dsys[1], &r.hsys[1], sizeof(DevSys)))
            rc = fail(LRDMC_ERR_HIP, "upload of system descriptors failed");
    }
    if (rc == LRDMC_OK) {
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void*)phase_fp64,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
            attr = true;
        }
        // initial local energies: a zero-step load-balanced phase
        rc = reset_counters(h);
        for (auto& r : h->sys) {
            if (rc) break;
            PhaseArgs pa{};
            pa.scheme = 0; pa.nproj = 0; pa.j = 0; pa.refresh_every = prm->refresh_every;
            pa.nu_mode = prm->nu_opt_mode; pa.a = prm->a; pa.tau = prm->tau; pa.E0 = 0.0;
            pa.conv_cap = 1;
            pa.seed = prm->seed; pa.counters = h->counters;
            hipLaunchKernelGGL(phase_fp64, dim3(r.d.nw), dim3(kWave), r.lds_bytes, h->stream,
                               (const DevSys*)r.dsys[r.parity], pa);
            if (hipGetLastError() != hipSuccess) { rc = fail(LRDMC_ERR_HIP, "init launch failed"); break; }
            std::vector<double> eL(r.d.nw);
            if (hipMemcpyAsync(eL.data(), r.d.eL, r.d.nw * 8, hipMemcpyDeviceToHost, h->stream) ||
                hipStreamSynchronize(h->stream)) {
                rc = fail(LRDMC_ERR_HIP, "init evaluation failed");
                break;
            }
            double acc = 0.0;
            for (double x : eL) acc += x;
            r.e0 = acc / r.d.nw;
            if (!std::isfinite(r.e0)) rc = fail(LRDMC_ERR_SINGULAR, "non-finite initial local energy");
        }
        unsigned long long cnt[kCntLen];
        if (!rc && (hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream) !=
                        hipSuccess ||
                    hipStreamSynchronize(h->stream) != hipSuccess))
            rc = fail(LRDMC_ERR_HIP, "counter readback failed");
        if (!rc && cnt[kCntSingular]) rc = fail(LRDMC_ERR_SINGULAR, "singular Slater matrix at init");
    }
    if (rc) {
        (void)hipEventDestroy(h->ev0); (void)hipEventDestroy(h->ev1);
        delete h;
        return rc;
    }
#ifdef LRDMC_SECTION_TIMERS
    if (hipMalloc((void**)&h->timers, (size_t)h->sys[0].d.nw * 8 * 8) != hipSuccess) h->timers = nullptr;
#endif
    *out = h;
    return LRDMC_OK;
}

#ifdef LRDMC_SECTION_TIMERS
// instrumentation builds only: per-walker section cycle counts of the last phase
int lrdmc_section_timers(lrdmc_handle* h, unsigned long long* out)
{
    if (!h || !h->timers) return fail(LRDMC_ERR_INVALID_ARG, "no timers");
    HIPCHK(hipMemcpy(out, h->timers, (size_t)h->sys[0].d.nw * 64, hipMemcpyDeviceToHost));
    return LRDMC_OK;
}
#endif

int lrdmc_step(lrdmc_handle* h, lrdmc_step_stats* st)
{
    if (!h) return fail(LRDMC_ERR_INVALID_ARG, "null handle");
    int rc = reset_counters(h);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    for (auto& r : h->sys)
        if ((rc = launch_phase(h, r))) return rc;
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    if (st) {
        unsigned long long cnt[kCntLen];
        HIPCHK(hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        st->walker_iters = (int64_t)cnt[kCntIters];
        st->max_iters = (int32_t)cnt[kCntMaxIters];
        st->min_iters = (int32_t)cnt[kCntMinIters];
        st->n_neg_weight = (int64_t)cnt[kCntNegW];
        st->n_no_move = (int64_t)cnt[kCntNoMove];
        st->n_refresh = (int64_t)cnt[kCntRefresh];
        st->n_small_ratio = (int64_t)cnt[kCntSmallR];
        st->n_capped = (int64_t)cnt[kCntCapped];
        st->elapsed_ms = ms;
        if (cnt[kCntSingular]) return fail(LRDMC_ERR_SINGULAR, "singular Slater matrix in a refresh");
    }
    return LRDMC_OK;
}

int lrdmc_branch(lrdmc_handle* h, lrdmc_branch_stats* st)
{
    if (!h) return fail(LRDMC_ERR_INVALID_ARG, "null handle");
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    std::vector<std::vector<double>> outs(h->sys.size(), std::vector<double>(5));
    std::vector<int> nd(h->sys.size());
    for (size_t k = 0; k < h->sys.size(); ++k) {
        SysRun& r = h->sys[k];
        const int nw = r.d.nw;
        const int nt = std::min(kMaxBranchBlock, std::max(64, 1 << (int)std::ceil(std::log2((double)nw))));
        hipLaunchKernelGGL(branch_scan, dim3(1), dim3(nt), 0, h->stream, r.d, h->prm.scheme, r.e0,
                           r.cum, r.bout);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(branch_comb, dim3((nw + 255) / 256), dim3(256), 0, h->stream, r.d,
                           h->prm.seed, h->j, r.cum, r.bout, r.sel);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemsetAsync(r.ndist, 0, sizeof(int), h->stream));
        hipLaunchKernelGGL(branch_count, dim3((nw + 255) / 256), dim3(256), 0, h->stream, r.sel, nw,
                           r.ndist);
        HIPCHK(hipGetLastError());
        // gather into the alternate buffers, then swap
        DevSys dn = r.d;
        dn.pos = r.pos_alt; dn.eL = r.eL_alt; dn.Wd = r.W_alt;
        const long tot = (long)nw * 3 * r.d.N;
        hipLaunchKernelGGL(branch_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                           h->stream, dn, r.sel, r.d.pos, r.d.eL, r.d.Wd);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(outs[k].data(), r.bout, 5 * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(&nd[k], r.ndist, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        r.pos_alt = r.d.pos; r.eL_alt = r.d.eL; r.W_alt = r.d.Wd;
        r.d.pos = dn.pos; r.d.eL = dn.eL; r.d.Wd = dn.Wd;
        r.parity ^= 1;
    }
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    int rc = LRDMC_OK;
    for (size_t k = 0; k < h->sys.size(); ++k) {
        SysRun& r = h->sys[k];
        const double mx = outs[k][0], tot = outs[k][1], se = outs[k][2], so = outs[k][3];
        if (!(mx > -INFINITY) || !(tot > 0)) { rc = fail(LRDMC_ERR_ALL_DEAD, "every walker weight is zero"); continue; }
        const double lwb = std::log(tot / r.d.nw) + mx;
        const double eb = se / so;
        r.hist_lwb.push_back(lwb);
        r.hist_e.push_back(eb);
        const int win = std::max(1, h->prm.e0_window);
        const size_t n = r.hist_e.size(), k0 = n > (size_t)win ? n - win : 0;
        double acc = 0.0;
        for (size_t q = k0; q < n; ++q) acc += r.hist_e[q];
        r.e0 = acc / (double)(n - k0);
        if (st && k == 0) {
            st->log_wbar = lwb; st->e_bar = eb; st->e0 = r.e0; st->max_lw = mx;
            st->n_distinct = nd[k]; st->elapsed_ms = ms;
        }
    }
    h->j++;
    return rc;
}

int lrdmc_energy_forces(lrdmc_handle* h, lrdmc_energy* e, double* forces, double* jgrad)
{
    if (!h || !e) return fail(LRDMC_ERR_INVALID_ARG, "null argument");
    if (forces || jgrad) return fail(LRDMC_ERR_UNSUPPORTED, "forces are not available in this build");
    const SysRun& r = h->sys[0];
    const int n = (int)r.hist_e.size(), p = std::max(0, h->prm.p_corr);
    const int start = std::max(p, n / 10);
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

int lrdmc_get_walkers(lrdmc_handle* h, int isys, double* pos, double* lw, double* eL, double* W,
                      int32_t* iters, int32_t* sel, int32_t* trace)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size()) return fail(LRDMC_ERR_INVALID_ARG, "bad handle/system");
    const SysRun& r = h->sys[isys];
    const size_t nw = r.d.nw;
    auto dn = [&](void* dst, const void* src, size_t b) {
        return dst ? hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, h->stream) : hipSuccess;
    };
    if (dn(pos, r.d.pos, nw * 3 * r.d.N * 8) || dn(lw, r.d.lw, nw * 8) || dn(eL, r.d.eL, nw * 8) ||
        dn(W, r.d.Wd, nw * 8) || dn(iters, r.d.iters, nw * 4) || dn(sel, r.sel, nw * 4))
        return fail(LRDMC_ERR_HIP, "device-to-host copy failed");
    if (trace) {
        if (!r.d.trace) return fail(LRDMC_ERR_INVALID_ARG, "tracing is off (trace_cap = 0)");
        HIPCHK(hipMemcpyAsync(trace, r.d.trace, nw * (size_t)r.d.trace_cap * 4, hipMemcpyDeviceToHost,
                              h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return LRDMC_OK;
}

int lrdmc_set_walkers(lrdmc_handle* h, int isys, const double* pos, const double* lw)
{
    if (!h || isys < 0 || isys >= (int)h->sys.size() || !pos)
        return fail(LRDMC_ERR_INVALID_ARG, "bad arguments");
    const SysRun& r = h->sys[isys];
    const size_t nw = r.d.nw;
    HIPCHK(hipMemcpyAsync(r.d.pos, pos, nw * 3 * r.d.N * 8, hipMemcpyHostToDevice, h->stream));
    if (lw) HIPCHK(hipMemcpyAsync(r.d.lw, lw, nw * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
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
    h->sys[isys].e0 = e0;
    return LRDMC_OK;
}

int lrdmc_get_branch_index(lrdmc_handle* h) { return h ? h->j : -1; }

void lrdmc_destroy(lrdmc_handle* h)
{
    if (!h) return;
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    delete h;
}

}  // extern "C"
