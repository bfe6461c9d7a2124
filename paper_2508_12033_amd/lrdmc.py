"""Thin ctypes binding of liblrdmc.so (C ABI in include/lrdmc.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies the device workspace and the HIP stream.
There is no CPU fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrdmc.so")

SCHEME_LB, SCHEME_CONV = 0, 1
FP64 = 0
MIXED_FP32 = 1
MIXED_BF16 = 2
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "bf16": MIXED_BF16}
NU_OPT_OWN, NU_OPT_ANY, NU_MAX = 0, 1, 2

ERRORS = {-1: "INVALID_ARG", -2: "HIP", -3: "WORKSPACE", -4: "SINGULAR", -5: "ALL_DEAD",
          -6: "UNSUPPORTED", -7: "NONFINITE", -8: "NEG_WEIGHT", -9: "NO_MOVE"}


class LrdmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lrdmc error %d (%s): %s" % (code, ERRORS.get(code, "?"), msg))
        self.code = code


class lrdmc_system(ct.Structure):
    _fields_ = [("n_atoms", ct.c_int32), ("atom_pos", ct.c_void_p), ("atom_charge", ct.c_void_p),
                ("atom_core", ct.c_void_p), ("core_rc", ct.c_void_p),
                ("atom_species", ct.c_void_p), ("n_basis", ct.c_int32),
                ("basis_atom", ct.c_void_p), ("basis_type", ct.c_void_p),
                ("basis_exp", ct.c_void_p), ("n_orb", ct.c_int32), ("mo_coeff", ct.c_void_p),
                ("n_up", ct.c_int32), ("n_dn", ct.c_int32), ("n_species", ct.c_int32),
                ("jastrow", ct.c_void_p), ("n_walkers", ct.c_int32), ("system_id", ct.c_uint64),
                ("n_ecp", ct.c_int32), ("ecp_atom", ct.c_void_p), ("ecp_l", ct.c_void_p),
                ("ecp_pow", ct.c_void_p), ("ecp_coef", ct.c_void_p), ("ecp_exp", ct.c_void_p),
                ("ecp_rcut", ct.c_void_p)]


class lrdmc_params(ct.Structure):
    _fields_ = [("scheme", ct.c_int32), ("precision", ct.c_int32), ("a", ct.c_double),
                ("tau", ct.c_double), ("n_proj", ct.c_int32), ("seed", ct.c_uint64),
                ("refresh_every", ct.c_int32), ("nu_opt_mode", ct.c_int32),
                ("p_corr", ct.c_int32), ("e0_window", ct.c_int32), ("trace_cap", ct.c_int32),
                ("strict", ct.c_int32), ("rotate", ct.c_int32), ("n_therm", ct.c_int32)]


class lrdmc_step_stats(ct.Structure):
    _fields_ = [("walker_iters", ct.c_int64), ("max_iters", ct.c_int32),
                ("min_iters", ct.c_int32), ("n_neg_weight", ct.c_int64),
                ("n_no_move", ct.c_int64), ("n_refresh", ct.c_int64),
                ("n_small_ratio", ct.c_int64), ("n_capped", ct.c_int64),
                ("n_nonfinite", ct.c_int64), ("elapsed_ms", ct.c_double)]


class lrdmc_branch_stats(ct.Structure):
    _fields_ = [("log_wbar", ct.c_double), ("e_bar", ct.c_double), ("e0", ct.c_double),
                ("max_lw", ct.c_double), ("n_distinct", ct.c_int32), ("elapsed_ms", ct.c_double)]


class lrdmc_tune_entry(ct.Structure):
    _fields_ = [("threads", ct.c_int32), ("order_big_first", ct.c_int32), ("ms", ct.c_float),
                ("system", ct.c_int32)]


class lrdmc_energy(ct.Structure):
    _fields_ = [("energy", ct.c_double), ("sigma", ct.c_double), ("n_used", ct.c_int32)]


EXPORTS = ["lrdmc_workspace_bytes", "lrdmc_init_system", "lrdmc_step", "lrdmc_branch",
           "lrdmc_energy_forces", "lrdmc_get_walkers", "lrdmc_set_walkers", "lrdmc_get_e0",
           "lrdmc_set_e0", "lrdmc_get_branch_index", "lrdmc_destroy", "lrdmc_last_error",
           "lrdmc_n_theta", "lrdmc_walker_derivs", "lrdmc_get_precision_report",
           "lrdmc_run", "lrdmc_autotune", "lrdmc_set_launch",
           "lrdmc_reconfigure_workspace_bytes", "lrdmc_reconfigure",
           "lrdmc_reconfigure_noalloc"]

_lib = None


def load(path=LIB_PATH):
    """Load the HIP library (torch first, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    if not os.path.exists(path):
        raise ImportError("liblrdmc.so is not built (run paper_2508_12033_amd.build)")
    L = ct.CDLL(path)
    vp, i32, sz, dbl = ct.c_void_p, ct.c_int32, ct.c_size_t, ct.c_double
    L.lrdmc_workspace_bytes.argtypes = [vp, ct.c_int, vp]
    L.lrdmc_workspace_bytes.restype = sz
    L.lrdmc_init_system.argtypes = [vp, ct.c_int, vp, vp, vp, sz, vp, ct.POINTER(vp)]
    L.lrdmc_step.argtypes = [vp, vp]
    L.lrdmc_branch.argtypes = [vp, vp]
    L.lrdmc_energy_forces.argtypes = [vp, vp, vp, vp]
    L.lrdmc_get_walkers.argtypes = [vp, ct.c_int, vp, vp, vp, vp, vp, vp, vp]
    L.lrdmc_set_walkers.argtypes = [vp, ct.c_int, vp, vp]
    L.lrdmc_get_e0.argtypes = [vp, ct.c_int]
    L.lrdmc_get_e0.restype = dbl
    L.lrdmc_set_e0.argtypes = [vp, ct.c_int, dbl]
    L.lrdmc_get_branch_index.argtypes = [vp]
    L.lrdmc_destroy.argtypes = [vp]
    L.lrdmc_destroy.restype = None
    L.lrdmc_last_error.restype = ct.c_char_p
    L.lrdmc_n_theta.argtypes = [vp, ct.c_int]
    L.lrdmc_get_precision_report.argtypes = [vp, ct.c_int, vp]
    L.lrdmc_run.argtypes = [vp, ct.c_int, vp, vp]
    L.lrdmc_autotune.argtypes = [vp, ct.c_int, vp, ct.c_int, vp]
    L.lrdmc_set_launch.argtypes = [vp, ct.c_int, ct.c_int]
    L.lrdmc_walker_derivs.argtypes = [vp, ct.c_int, vp, vp, vp, vp, vp]
    u64 = ct.c_uint64
    L.lrdmc_reconfigure_workspace_bytes.argtypes = [ct.c_int]
    L.lrdmc_reconfigure_workspace_bytes.restype = sz
    L.lrdmc_reconfigure.argtypes = [ct.c_int, ct.c_int, vp, vp, vp, dbl, u64, u64, ct.c_int, vp, vp,
                                    vp, sz, vp]
    L.lrdmc_reconfigure.restype = ct.c_int
    L.lrdmc_reconfigure_noalloc.argtypes = [ct.c_int, ct.c_int, vp, vp, vp, dbl, u64, u64,
                                            ct.c_int, vp, vp, vp]
    L.lrdmc_reconfigure_noalloc.restype = ct.c_int
    for k in ("lrdmc_init_system", "lrdmc_step", "lrdmc_branch", "lrdmc_energy_forces",
              "lrdmc_get_walkers", "lrdmc_set_walkers", "lrdmc_set_e0",
              "lrdmc_get_branch_index", "lrdmc_n_theta", "lrdmc_walker_derivs",
              "lrdmc_get_precision_report", "lrdmc_run", "lrdmc_autotune",
              "lrdmc_set_launch"):
        getattr(L, k).restype = ct.c_int
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise LrdmcError(rc, _lib.lrdmc_last_error().decode())
    return rc


def _sys_struct(d, keep):
    arrs = {}
    for k, dt in (("atom_pos", np.float64), ("atom_charge", np.float64), ("atom_core", np.int32),
                  ("core_rc", np.float64), ("atom_species", np.int32), ("basis_atom", np.int32),
                  ("basis_type", np.int32), ("basis_exp", np.float64), ("mo_coeff", np.float64),
                  ("jastrow", np.float64)):
        arrs[k] = np.ascontiguousarray(d[k], dtype=dt)
        keep.append(arrs[k])
    n_walkers = int(d.get("n_walkers_run", d["init_pos"].shape[0]))
    n_ecp = len(d.get("ecp_atom", ()))
    ecp = [None] * 6
    if n_ecp:
        for n, (k, dt) in enumerate((("ecp_atom", np.int32), ("ecp_l", np.int32), ("ecp_pow", np.int32),
                                     ("ecp_coef", np.float64), ("ecp_exp", np.float64),
                                     ("ecp_rcut", np.float64))):
            a = np.ascontiguousarray(d[k], dtype=dt)
            keep.append(a)
            ecp[n] = a.ctypes.data
    return lrdmc_system(
        int(arrs["atom_pos"].shape[0]), arrs["atom_pos"].ctypes.data,
        arrs["atom_charge"].ctypes.data, arrs["atom_core"].ctypes.data,
        arrs["core_rc"].ctypes.data, arrs["atom_species"].ctypes.data,
        int(arrs["basis_exp"].shape[0]), arrs["basis_atom"].ctypes.data,
        arrs["basis_type"].ctypes.data, arrs["basis_exp"].ctypes.data,
        int(arrs["mo_coeff"].shape[1]), arrs["mo_coeff"].ctypes.data, int(d["n_up"]),
        int(d["n_dn"]), int(arrs["jastrow"].shape[0] - 2), arrs["jastrow"].ctypes.data,
        n_walkers, int(d.get("system_id", 0)), n_ecp, *ecp)


def make_params(scheme="lb", a=0.2, tau=0.25, n_proj=300, seed=12033, refresh_every=None,
                nu_opt_mode=NU_OPT_OWN, p_corr=10, e0_window=50, trace_cap=0, precision="fp64",
                strict=False, rotate=False, n_therm=0):
    """precision: "fp64" (every step in FP64), "fp32" or "bf16" (mixed: the
    orbital product on FP32 or BF16 MFMA, FP32 rank-one updates, FP64
    accumulation and refreshes).

    refresh_every: moves between rebuilds of the inverses and Jastrow caches
    from scratch; by default 128 in FP64 (the rounding drift of 128 rank-one
    updates stays far below the FP64 error bar: local energies within 2e-12 Ha
    of the oracle's from-scratch values) and 16 in the mixed modes."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if refresh_every is None:
        refresh_every = 128 if prec == PRECISIONS["fp64"] else 16
    return lrdmc_params(SCHEME_LB if scheme == "lb" else SCHEME_CONV, prec, float(a), float(tau),
                        int(n_proj), int(seed), int(refresh_every), int(nu_opt_mode), int(p_corr),
                        int(e0_window), int(trace_cap), 1 if strict else 0, 1 if rotate else 0,
                        int(n_therm))


def params_for(d, scheme="lb", **kw):
    """Parameters from a generated system dict (a, tau, n_proj, seed, nu mode)."""
    base = dict(a=d["a"], tau=d["tau"], n_proj=d["n_proj"], seed=d["seed"],
                nu_opt_mode=int(d.get("nu_opt_mode", 0)))
    base.update(kw)
    return make_params(scheme, **base)


class Handle:
    """Owns the torch workspace tensor and the library handle of one run.

    systems: list of generator dicts; init_pos of each is used (or the
    n_walkers_run first walkers if that key is present)."""

    def __init__(self, systems, prm, device="cuda:0", stream=None):
        import torch
        L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the lattice-regularized DMC library runs only on gfx950")
        if isinstance(systems, dict):
            systems = [systems]
        self.systems = systems
        self.prm = prm
        self.keep = []
        arr = (lrdmc_system * len(systems))(*[_sys_struct(d, self.keep) for d in systems])
        self.sys_arr = arr
        self.nw = [int(s.n_walkers) for s in arr]
        self.N = [int(s.n_up + s.n_dn) for s in arr]
        init = np.concatenate([np.ascontiguousarray(d["init_pos"][:nw], np.float64).reshape(-1)
                               for d, nw in zip(systems, self.nw)])
        self.keep.append(init)
        nbytes = L.lrdmc_workspace_bytes(ct.byref(arr), len(systems), ct.byref(prm))
        if nbytes == 0:
            msg = L.lrdmc_last_error().decode()
            unsupported = "too large" in msg or "not supported" in msg
            raise LrdmcError(-6 if unsupported else -1, msg)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            self.stream = stream or torch.cuda.current_stream(self.device)
            h = ct.c_void_p()
            _check(L.lrdmc_init_system(ct.byref(arr), len(systems), ct.byref(prm), init.ctypes.data,
                                       base + off, nbytes, self.stream.cuda_stream, ct.byref(h)))
        self.h = h
        self.L = L

    def step(self, stats=True):
        st = lrdmc_step_stats()
        _check(self.L.lrdmc_step(self.h, ct.byref(st) if stats else None))
        return st if stats else None

    def branch(self):
        st = lrdmc_branch_stats()
        _check(self.L.lrdmc_branch(self.h, ct.byref(st)))
        return st

    def run(self, n_branchings):
        """n_branchings graph-replayed cycles of phase + reconfiguration;
        returns (summed step stats, last branch stats)."""
        st = lrdmc_step_stats()
        bs = lrdmc_branch_stats()
        _check(self.L.lrdmc_run(self.h, int(n_branchings), ct.byref(st), ct.byref(bs)))
        return st, bs

    def autotune(self, n_steps=8):
        """Time the launch candidates of the mixed-precision phase; returns the
        list of (threads, big_first, ms, system) -- system -1: all systems in
        one launch, k: system k alone, -2: one launch per system (sum) -- and
        keeps the fastest."""
        log = (lrdmc_tune_entry * 64)()
        n = ct.c_int(0)
        _check(self.L.lrdmc_autotune(self.h, int(n_steps), log, 64, ct.byref(n)))
        return [(log[k].threads, log[k].order_big_first, log[k].ms, log[k].system)
                for k in range(n.value)]

    def set_launch(self, threads, big_first=True):
        _check(self.L.lrdmc_set_launch(self.h, int(threads), 1 if big_first else 0))

    def energy(self):
        e = lrdmc_energy()
        _check(self.L.lrdmc_energy_forces(self.h, ct.byref(e), None, None))
        return e.energy, e.sigma, e.n_used

    def n_theta(self, isys=0):
        n = self.L.lrdmc_n_theta(self.h, isys)
        _check(n)
        return n

    def forces(self):
        """(forces [n_atoms][3], Jastrow-table energy gradient) of system 0 from
        the adjoint pass over the current population."""
        e = lrdmc_energy()
        nth = self.n_theta(0)
        M = self.systems[0]["atom_pos"].shape[0]
        f = np.zeros(3 * M); jg = np.zeros(nth - 3 * M)
        _check(self.L.lrdmc_energy_forces(self.h, ct.byref(e), f.ctypes.data, jg.ctypes.data))
        return f.reshape(M, 3), jg

    def walker_derivs(self, theta=None, isys=0):
        """Per-walker e_L, log|Psi| [nw] and d/dtheta of both [nw][n_theta]
        as float64 tensors on the handle's device (adjoint pass)."""
        import torch
        nw, nth = self.nw[isys], self.n_theta(isys)
        dev = self.device
        eL = torch.empty(nw, dtype=torch.float64, device=dev)
        lp = torch.empty(nw, dtype=torch.float64, device=dev)
        deL = torch.empty(nw, nth, dtype=torch.float64, device=dev)
        dlp = torch.empty(nw, nth, dtype=torch.float64, device=dev)
        th = None
        if theta is not None:
            th = np.ascontiguousarray(np.asarray(theta, np.float64).reshape(-1))
            if th.size != nth:
                raise ValueError("theta has %d entries, expected %d" % (th.size, nth))
        _check(self.L.lrdmc_walker_derivs(self.h, isys, None if th is None else th.ctypes.data,
                                          eL.data_ptr(), lp.data_ptr(), deL.data_ptr(),
                                          dlp.data_ptr()))
        return eL, lp, deL, dlp

    def walkers(self, isys=0, trace=False):
        nw, N = self.nw[isys], self.N[isys]
        pos = np.zeros((nw, N, 3)); lw = np.zeros(nw); eL = np.zeros(nw); W = np.zeros(nw)
        it = np.zeros(nw, np.int32); sel = np.zeros(nw, np.int32)
        tr = np.zeros((nw, max(1, self.prm.trace_cap)), np.int32) if trace else None
        _check(self.L.lrdmc_get_walkers(self.h, isys, pos.ctypes.data, lw.ctypes.data,
                                        eL.ctypes.data, W.ctypes.data, it.ctypes.data,
                                        sel.ctypes.data, None if tr is None else tr.ctypes.data))
        out = dict(pos=pos, lw=lw, eL=eL, W=W, iters=it, sel=sel)
        if trace:
            out["trace"] = tr
        return out

    def precision_report(self, isys=0):
        """Mixed precisions: [nw][4] = e_L, W, bbar of the mixed-precision step
        at the last phase's final configuration and its largest ratio error."""
        out = np.zeros((self.nw[isys], 4))
        _check(self.L.lrdmc_get_precision_report(self.h, isys, out.ctypes.data))
        return out

    def set_walkers(self, pos, lw=None, isys=0):
        pos = np.ascontiguousarray(pos, np.float64)
        lwa = None if lw is None else np.ascontiguousarray(lw, np.float64)
        _check(self.L.lrdmc_set_walkers(self.h, isys, pos.ctypes.data,
                                        None if lwa is None else lwa.ctypes.data))

    def e0(self, isys=0):
        return self.L.lrdmc_get_e0(self.h, isys)

    def set_e0(self, e0, isys=0):
        _check(self.L.lrdmc_set_e0(self.h, isys, float(e0)))

    def branch_index(self):
        return self.L.lrdmc_get_branch_index(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.lrdmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _walker_energy_fn():
    import torch

    class WalkerEnergy(torch.autograd.Function):
        """theta (float64 CPU tensor [n_theta]: nuclear coordinates, then the
        Jastrow table) -> per-walker (e_L, log|Psi|) of the handle's current
        walkers, with the adjoint pass supplying the vector-Jacobian product."""

        @staticmethod
        def forward(ctx, theta, handle, isys):
            eL, lp, deL, dlp = handle.walker_derivs(theta.detach().cpu().numpy(), isys)
            ctx.save_for_backward(deL, dlp)
            ctx.theta_device = theta.device
            return eL, lp

        @staticmethod
        def backward(ctx, g_eL, g_lp):
            deL, dlp = ctx.saved_tensors
            g = torch.zeros(deL.shape[1], dtype=torch.float64, device=deL.device)
            if g_eL is not None:
                g = g + g_eL.to(torch.float64) @ deL
            if g_lp is not None:
                g = g + g_lp.to(torch.float64) @ dlp
            return g.to(ctx.theta_device), None, None

    return WalkerEnergy


_WE = None


def walker_energy(theta, handle, isys=0):
    """Differentiable per-walker (e_L, log|Psi|) as functions of theta."""
    global _WE
    if _WE is None:
        _WE = _walker_energy_fn()
    return _WE.apply(theta, handle, isys)


def reconfigure(lw, eL, W=None, e0=0.0, scheme="lb", seed=12033, sysid=0, j=0, stream=None):
    """Reconfiguration of a caller-held population (lrdmc_reconfigure): lw, eL
    (and W for the load-balanced weighting) are float64 CUDA tensors of one
    length.  Returns (sel int32 tensor, out float64 tensor [8]) on the same
    device, enqueued on `stream` (default: torch's current stream)."""
    import torch
    L = load()
    nw = int(lw.shape[0])
    dev = lw.device
    for t in (lw, eL) + ((W,) if W is not None else ()):
        if t.dtype != torch.float64 or not t.is_cuda or t.shape != lw.shape or not t.is_contiguous():
            raise ValueError("lw, eL, W must be contiguous float64 CUDA tensors of one length")
    sel = torch.empty(nw, dtype=torch.int32, device=dev)
    out = torch.empty(8, dtype=torch.float64, device=dev)
    nb = L.lrdmc_reconfigure_workspace_bytes(nw)
    if nb == 0:
        raise LrdmcError(-1, L.lrdmc_last_error().decode())
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    st = stream or torch.cuda.current_stream(dev)
    _check(L.lrdmc_reconfigure(SCHEME_LB if scheme == "lb" else SCHEME_CONV, nw, lw.data_ptr(),
                               eL.data_ptr(), None if W is None else W.data_ptr(), float(e0),
                               int(seed), int(sysid), int(j), sel.data_ptr(), out.data_ptr(), base,
                               nb, st.cuda_stream))
    return sel, out

