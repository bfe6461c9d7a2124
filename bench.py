"""Benchmark of the lattice-regularized DMC hot path on one MI355X.

Headline workload (one step = one pass of the hot path): one load-balanced
projection phase of N_proj = 300 lattice moves for every walker (ratios of all
6N moves, local energy, weight update, heat-bath move, Sherman-Morrison
update, FP64 refreshes) followed by the reconfiguration, on the 16-electron /
8-atom synthetic molecule with 4096 walkers in FP64.  Inputs are resident in
HBM before the timed region; the timed cycles are graph replays of
(phase, reconfiguration) with E_0 and the history kept on the device.

Metric: electron-move proposals per second = walker-iterations that evaluated
all 6N move ratios x 6N / wall time.  Printed beside it:
  - conventional (continuous-time) scheme on the same system at matched mean
    iterations, its lane occupancy, and the load-balanced speedup, against the
    conventional kernel (each walker's wavefront ends when its time is used
    up) and against the lockstep-masked batch of the paper's definition
    (every walker pays the phase maximum of iterations);
  - the mixed-precision paths with their stated errors: the same 16-electron
    workload in FP32, the 128-electron / 2048-walker system with the BF16
    orbital product (and FP32) beside the same system in FP64, the
    32-electron system in all three precisions, the three uneven systems in
    one launch;
  - the 16-electron system with a non-local pseudopotential (6N lattice moves
    plus the quadrature points of the electrons inside a cutoff sphere);
  - the adjoint pass (per-walker parameter derivatives) on the 16-electron
    system with electron-nucleus Jastrow terms;
  - the roofline of the phase kernel and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-conv]
                       [--no-extra] [--copy-calibration]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("electron-move proposals/sec on 1 GPU, mixed vs FP64 at stated error; "
          "speedup vs conventional")
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector
KERNEL_SOURCES = ["paper_2508_12033_amd/csrc/lrdmc_phase.hip",
                  "paper_2508_12033_amd/csrc/lrdmc_dev.hpp",
                  "paper_2508_12033_amd/csrc/lrdmc_devfn.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phase_fp64_c1_traffic.json")
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
MIXED_SOURCES = ["paper_2508_12033_amd/csrc/lrdmc_mixed.hip",
                 "paper_2508_12033_amd/csrc/lrdmc_dev.hpp",
                 "paper_2508_12033_amd/csrc/lrdmc_devfn.hpp"]
MIXED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phase_mixed_c3_bf16_traffic.json")


def flops_per_walker_step(N, n, Nb, M, has_en, refresh_every):
    """Algorithmic floating-point operations of one incremental walker-step
    (exp, log, sqrt and division count as one operation each):
      basis functions of the moved electron at its position and 6 neighbours
      (+ gradient, Laplacian) ~ 85 Nb; orbital rows 2*11*Nb*n; Sherman-Morrison
      4 n^2; determinant ratios of the moved spin 12 n^2; ratios of all moves
      2P; Jastrow pair differences (N-1)*166 + (P-6)*35 (+ nuclei); local
      energy N(8n+20) + 2P; heat bath 2P; the refresh (Gauss-Jordan 8 n^3 over
      both spins and the full Jastrow N(N-1)*137) divided by its cadence."""
    P = 6 * N
    f = 85 * Nb + 2 * 11 * Nb * n + 4 * n * n + 12 * n * n + 2 * P
    f += (N - 1) * 166 + (P - 6) * 35 + M * (145 if has_en else 8)
    f += N * (8 * n + 20) + 2 * P + 2 * P
    refresh = 8 * n ** 3 + N * ((N - 1) * 137 + M * (137 if has_en else 8))
    return f + refresh / refresh_every


def kernel_hash(sources=None):
    """Hash of the kernel sources and the compiler flags they are built with
    (include paths left out), so that stored counters go stale when either
    changes."""
    from paper_2508_12033_amd.build import FLAGS
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    h.update(" ".join(f for f in FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def traffic_per_launch(path=TRAFFIC_FILE, sources=None):
    """HBM bytes per phase launch from the committed rocprofv3 counter runs,
    or None when the kernel sources changed since they were taken."""
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash(sources):
        return None
    return t.get("bytes_per_launch")


def mixed_bytes_per_walker_step(n, refresh_every):
    """Algorithmic HBM bytes of one mixed-precision walker-step (FP32 walker
    block in HBM, n orbitals of the moved electron's spin): the orbital rows
    of the spin's 6n moves and its 4n derivative rows read for the ratio and
    gradient products (10 n^2 floats), the spin's inverse read and written
    back (2 n^2), the moved electron's new rows written and the accepted row
    read (12 n), and the refresh, which reads the Slater rows and inverses of
    both spins and writes the inverses (6 n^2), once every refresh_every
    moves."""
    return 4.0 * (10 * n * n + 2 * n * n + 12 * n + 6.0 * n * n / refresh_every)


def mixed_roofline(systems, prm, launch_ms, traffic=None):
    """HBM roofline of one mixed-precision phase launch over all systems."""
    if isinstance(systems, dict):
        systems = [systems]
    byts = sum(mixed_bytes_per_walker_step(max(int(d["n_up"]), int(d["n_dn"])), prm.refresh_every) *
               int(d.get("n_walkers_run", d["init_pos"].shape[0])) * prm.n_proj for d in systems)
    gbs = byts / (launch_ms * 1e-3) / 1e9
    return dict(bound="hbm", kernel="phase_mixed", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=gbs / HBM_PEAK_GBS, traffic=traffic, bytes_per_launch=byts, launch_ms=launch_ms)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, n_walk=4096, n_steps=600, n_walk_1=256, n_steps_1=300):
    """The FP64 oracle as it stands, on a bounded sample of the same workload:
    all host threads on the first n_walk walkers for n_steps load-balanced
    steps, and one thread on the first n_walk_1 walkers for n_steps_1 steps."""
    import oracle as O
    S = O.System(d)
    e0 = -20.0

    def rate(nw, ns, nt):
        prm = S.params(nproj=ns)
        pos = np.array(d["init_pos"][:nw], copy=True)
        lw = np.zeros(nw)
        t0 = time.perf_counter()
        O.population_phase(S, prm, "lb", 0, e0, pos, lw, nthreads=nt, record=False)
        dt = time.perf_counter() - t0
        return nw * ns * S.P / dt, dt

    nt = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    v, dt = rate(n_walk, n_steps, nt)
    v1, dt1 = rate(n_walk_1, n_steps_1, 1)
    return dict(value=v, unit="proposals/s", cores=nt, kind="oracle",
                sample="%d walkers x %d load-balanced steps of the 16-electron system "
                       "(%.1f s wall, %d threads)" % (n_walk, n_steps, dt, nt),
                value_1core=v1,
                sample_1core="%d walkers x %d steps on one thread (%.1f s)" % (n_walk_1, n_steps_1,
                                                                               dt1),
                cpu_model=_cpu_model())


def proposals_of(systems, prm, st, scheme):
    """Proposals evaluated: load-balanced N_proj x walkers x 6N per system per
    cycle; conventional: the active walker-iterations (one system) x 6N."""
    if scheme == "conv":
        return st.walker_iters * 6 * int(systems[0]["n_elec"])
    return sum(int(d["n_elec"]) * 6 * int(d.get("n_walkers_run", d["init_pos"].shape[0]))
               for d in systems) * prm.n_proj


def run_cycles(B, systems, scheme, steps, warmup, precision="fp64", tune=False, threads=None, **kw):
    """Init, warm up, then time `steps` graph-replayed (phase, reconfiguration)
    cycles with one synchronisation at each end."""
    import torch
    if isinstance(systems, dict):
        systems = [systems]
    prm = B.params_for(systems[0], scheme, precision=precision, **kw)
    h = B.Handle(systems, prm)
    h.step(stats=False)
    h.branch()
    log = None
    if threads:
        h.set_launch(threads)
    if tune:
        log = h.autotune(n_steps=8)
    if warmup > 0:
        h.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, bs = h.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nw = sum(int(d.get("n_walkers_run", d["init_pos"].shape[0])) for d in systems)
    props = proposals_of(systems, prm, st, scheme) * (steps if scheme == "lb" else 1)
    out = dict(proposals=props, seconds=dt, walker_iters=st.walker_iters,
               ms_per_cycle=1e3 * dt / steps, max_iters=st.max_iters,
               mean_iters=st.walker_iters / (steps * nw),
               occupancy=st.walker_iters / (steps * nw * max(1, st.max_iters)) if scheme == "conv"
               else 1.0, e0=h.e0(), tune=log)
    return h, prm, out


def phase_kernel_ms(h, n=3):
    """Average duration of the phase launch(es) of one step, HIP events on the
    handle's stream."""
    ms = []
    for _ in range(n):
        st = h.step(stats=True)
        ms.append(st.elapsed_ms)
        h.branch()
    return float(np.mean(ms))


def precision_summary(h, isys=0):
    """Stated error of a mixed-precision run at its last phase: the mixed
    step's own e_L and W against the FP64 estimator values at the same
    configurations, and the largest ratio error against FP64.  (Read after a
    phase and before the next reconfiguration, which reorders the walkers.)"""
    rep = h.precision_report(isys)
    g = h.walkers(isys)
    e = np.abs(rep[:, 0] - g["eL"]) / np.abs(g["eL"])
    w = np.abs(rep[:, 1] - g["W"]) / np.abs(g["W"])
    return dict(step_eL_rel_err_max=float(e.max()), step_eL_rel_err_median=float(np.median(e)),
                step_eL_rel_err_p99=float(np.quantile(e, 0.99)),
                step_W_rel_err_max=float(w.max()), ratio_err_max=float(rep[:, 3].max()),
                ratio_err_median=float(np.median(rep[:, 3])),
                ratio_err_p99=float(np.quantile(rep[:, 3], 0.99)), walkers=int(len(e)),
                reported_eL="FP64 evaluation at the phase's final configuration")


def copy_calibration():
    """A plain 256 MiB device-to-device copy, for scaling the FETCH_SIZE and
    WRITE_SIZE counters to bytes."""
    import torch
    a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=256 << 20, copies=3)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-conv", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only (no mixed, batched or adjoint lines)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--profile-workload",
                    choices=["c3_bf16", "c3_fp32", "c3_fp64", "c1_fp32", "c2_fp32", "ce_fp64"],
                    help="run only this workload (ce: the 16-electron system with the non-local "
                         "pseudopotential) for --steps cycles (for profilers) and print its line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; --gpus %d is not supported "
              "(the walker population of one GPU is the unit of work)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_2508_12033_amd import inputs as I
    from paper_2508_12033_amd import lrdmc as B

    if args.profile_workload:
        wl = args.profile_workload
        sysd = {"c3": lambda: I.c3_system(n_walkers=2048), "c1": lambda: I.c1_system(n_walkers=4096),
                "c2": I.c2_systems, "ce": lambda: I.c1_ecp_system(n_walkers=4096)}[wl[:2]]()
        hx, _, r = run_cycles(B, sysd, "lb", args.steps, args.warmup, precision=wl[3:],
                              threads=128 if wl == "c2_fp32" else None)
        hx.close()
        print(json.dumps(dict(workload=wl, proposals_per_s=r["proposals"] / r["seconds"],
                              ms_per_branching=r["ms_per_cycle"])), flush=True)
        return

    d = I.c1_system(n_walkers=4096)
    nw, N, n_proj = 4096, d["n_elec"], d["n_proj"]

    h, prm, lb = run_cycles(B, d, "lb", args.steps, args.warmup)
    value = lb["proposals"] / lb["seconds"]
    kms = phase_kernel_ms(h)
    h.close()

    fl = flops_per_walker_step(N, d["n_up"], d["n_basis"], d["n_atoms"], 0, prm.refresh_every)
    achieved = fl * nw * n_proj / (kms * 1e-3) / 1e12
    tr = traffic_per_launch()
    roof = dict(bound="alu", kernel="phase_fp64", achieved=achieved, peak=FP64_PEAK_TFLOPS,
                unit="TFLOP/s", frac=achieved / FP64_PEAK_TFLOPS, traffic=tr,
                flops_per_walker_step=fl, walker_steps_per_launch=nw * n_proj, launch_ms=kms)

    res = dict(metric=METRIC, value=value, unit="proposals/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=lb["ms_per_cycle"], higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="16-electron 8-atom synthetic molecule (1 C-like and 1 "
                                    "O-like soft core, 6 protons, 80 s/p Gaussians), 4096 "
                                    "walkers, a=0.2 bohr, load-balanced N_proj=300, FP64, "
                                    "refresh every %d moves" % prm.refresh_every,
                           walkers=nw, electrons=N, n_proj=n_proj, precision="fp64",
                           refresh_every=prm.refresh_every,
                           scheme="load-balanced", step="one projection phase + reconfiguration"),
               roofline=roof)

    if not args.no_conv:
        hc, _, cv = run_cycles(B, d, "conv", args.steps, args.warmup)
        # per-phase maxima: the lockstep batch of a phase lasts as long as its
        # slowest walker
        pmax, piters = [], []
        for _ in range(5):
            st = hc.step(stats=True)
            hc.branch()
            pmax.append(st.max_iters)
            piters.append(st.walker_iters)
        hc.close()
        nbar = cv["mean_iters"]
        mbar = float(np.mean(pmax))
        hm, _, lbm = run_cycles(B, d, "lb", args.steps, 1, n_proj=int(round(nbar)))
        hm.close()
        # the conventional scheme run lockstep-masked (walkers that have reached
        # tau wait, masked, for the slowest one): every walker pays the phase
        # maximum of iterations, the cost of a load-balanced phase of that length
        hl, _, lbl = run_cycles(B, d, "lb", args.steps, 1, n_proj=int(round(mbar)))
        hl.close()
        from scipy.stats import poisson
        mu = nbar - 1.0
        k = np.arange(0, int(mu + 40 * np.sqrt(mu) + 100))
        emax = float(np.sum(1.0 - poisson.cdf(k, mu) ** nw)) + 1.0
        res["conventional"] = dict(
            tau=d["tau"], mean_iters=nbar, max_iters=cv["max_iters"], lane_occupancy=cv["occupancy"],
            proposals_per_s=cv["proposals"] / cv["seconds"], ms_per_branching=cv["ms_per_cycle"],
            poisson_model_max_iters=emax, poisson_model_time_ratio=emax / nbar)
        res["conventional"].update(
            phase_max_iters=pmax, lockstep_lane_occupancy=float(np.sum(piters)) / (nw * float(np.sum(pmax))))
        res["lb_matched"] = dict(n_proj=int(round(nbar)), ms_per_branching=lbm["ms_per_cycle"])
        res["conventional_lockstep"] = dict(
            n_proj=int(round(mbar)), ms_per_branching=lbl["ms_per_cycle"],
            note="conventional scheme with finished walkers masked until the slowest of the phase "
                 "finishes (the batched definition): every walker pays the phase maximum of iterations")
        res["speedup_vs_conventional"] = cv["ms_per_cycle"] / lbm["ms_per_cycle"]
        res["speedup_vs_lockstep_conventional"] = lbl["ms_per_cycle"] / lbm["ms_per_cycle"]

        # the idle-lane model of App. C: emulated iteration counts at the
        # measured mean (b held at its mean), beside the measured phase maxima
        from paper_2508_12033_amd import emulation as EM
        emu = EM.emulate_counts(nw, tau=1.0, b_mean=nbar - 1.0, b_std=0.0, seed=5)
        res["conventional"]["app_c_emulation"] = dict(
            mean=float(emu.mean()), max=int(emu.max()), min=int(emu.min()),
            model=EM.poisson_extremes(nw, nbar - 1.0), measured_phase_max_mean=mbar)

    if not args.no_conv:
        # Sec. II.C / Sec. III: both schemes sample the same fixed-node state;
        # energies with blocking error bars and their z-score after an
        # equilibration left out of the estimate, on the H2 system (256
        # walkers) and the 16-electron system (4096 walkers)
        agree = {}
        for name, dd, nw_, nb in (("h2_256w", I.h2_system(n_walkers=256), 100, 300),
                                  ("c1_4096w", d, 100, 300),
                                  ("c1_ecp_4096w", I.c1_ecp_system(n_walkers=4096), 200, 600)):
            row = dict(equilibration_branchings=nw_, measured_branchings=nb)
            for sch in ("lb", "conv"):
                hs = B.Handle(dd, B.params_for(dd, sch, n_therm=nw_))
                hs.run(nw_ + nb)
                E, sig, n = hs.energy()
                hs.close()
                row[sch] = dict(E=E, sigma=sig, n_used=n)
            row["z"] = (row["lb"]["E"] - row["conv"]["E"]) / float(np.hypot(row["lb"]["sigma"],
                                                                              row["conv"]["sigma"]))
            agree[name] = row
        res["scheme_agreement"] = agree

    if not args.no_extra:
        extra = {}
        steps_x = max(2, args.steps // 3)
        # the same 16-electron workload on the mixed-precision path
        hx, px, r = run_cycles(B, d, "lb", steps_x, 1, precision="fp32", tune=True)
        stx = hx.step(stats=True)
        extra["c1_mixed_fp32"] = dict(proposals_per_s=r["proposals"] / r["seconds"],
                                      ms_per_branching=r["ms_per_cycle"], tune=r["tune"],
                                      vs_fp64=(r["proposals"] / r["seconds"]) / value,
                                      error=precision_summary(hx),
                                      roofline=mixed_roofline(d, px, stx.elapsed_ms))
        hx.close()
        # 128 electrons, 640 basis functions, 2048 walkers
        c3 = I.c3_system(n_walkers=2048)
        for prec in ("bf16", "fp32"):
            hx, px, r = run_cycles(B, c3, "lb", 2, 0, precision=prec)
            stx = hx.step(stats=True)
            tr = traffic_per_launch(MIXED_TRAFFIC_FILE, MIXED_SOURCES) if prec == "bf16" else None
            extra["c3_mixed_" + prec] = dict(
                workload="128 electrons (64+64), 32 atoms, 640 basis functions, 2048 walkers, "
                         "a=0.15, N_proj=300, refresh every 16",
                proposals_per_s=r["proposals"] / r["seconds"], ms_per_branching=r["ms_per_cycle"],
                error=precision_summary(hx), roofline=mixed_roofline(c3, px, stx.elapsed_ms, tr))
            hx.close()
        # the same system in FP64 (the large-system layout of the FP64 kernel:
        # two 64-lane walkers per CU, coefficient block, Slater rows and the
        # inverse of the spin not moving in global memory), one timed branching
        hx, px, r = run_cycles(B, c3, "lb", 1, 0, precision="fp64")
        fp64_rate = r["proposals"] / r["seconds"]
        extra["c3_fp64"] = dict(
            workload="128 electrons (64+64), 32 atoms, 640 basis functions, 2048 walkers, "
                     "a=0.15, N_proj=300, FP64 (large-system layout: two walkers per CU)",
            proposals_per_s=fp64_rate, ms_per_branching=r["ms_per_cycle"])
        hx.close()
        for prec in ("bf16", "fp32"):
            extra["c3_mixed_" + prec]["vs_fp64"] = extra["c3_mixed_" + prec]["proposals_per_s"] / fp64_rate
        # three uneven systems in one launch, graph-replayed cycles, tuned launch
        c2 = I.c2_systems()
        hx, px, r = run_cycles(B, c2, "lb", 2, 0, precision="fp32", tune=True)
        stx = hx.step(stats=True)
        extra["c2_batched_fp32"] = dict(
            workload="16e/8 atoms x 8192, 32e/16 atoms x 4096, 64e/32 atoms x 2048 walkers "
                     "in one launch, N_proj=300",
            proposals_per_s=r["proposals"] / r["seconds"], ms_per_branching=r["ms_per_cycle"],
            tune=r["tune"], error=[precision_summary(hx, k) for k in range(3)],
            roofline=mixed_roofline(c2, px, stx.elapsed_ms))
        hx.close()
        # the launch modes the tuner chooses between: all three systems in one
        # launch (128 threads per walker, the best single-launch size), and
        # the three systems as three handles, one launch each (each tuned)
        h1, _, r1 = run_cycles(B, c2, "lb", steps_x, 1, precision="fp32", threads=128)
        h1.close()
        sep = []
        for dk in c2:
            hk, _, rk = run_cycles(B, dk, "lb", steps_x, 1, precision="fp32", tune=True)
            sep.append(rk["ms_per_cycle"])
            hk.close()
        extra["c2_batched_fp32"]["one_launch_128_threads_ms"] = r1["ms_per_cycle"]
        extra["c2_batched_fp32"]["separate_handles_ms"] = sep
        extra["c2_batched_fp32"]["tuned_vs_one_launch"] = r1["ms_per_cycle"] / r["ms_per_cycle"]
        # mixed vs FP64 on the 32-electron molecule of the uneven set (16
        # orbitals per spin, 160 basis functions), 4096 walkers, N_proj = 300;
        # the FP64 kernel holds eight such walkers per CU
        d32 = dict(I.c2_systems()[1])
        row = dict(workload="32 electrons (16+16), 16 atoms, 160 basis functions, 4096 walkers, "
                            "a=0.2, N_proj=300")
        for prec in ("fp64", "fp32", "bf16"):
            hx, px, r = run_cycles(B, d32, "lb", 2, 1, precision=prec, tune=prec != "fp64")
            stx = hx.step(stats=True)
            row[prec] = dict(proposals_per_s=r["proposals"] / r["seconds"],
                             ms_per_branching=r["ms_per_cycle"])
            if prec != "fp64":
                row[prec]["error"] = precision_summary(hx)
                row[prec]["roofline"] = mixed_roofline(d32, px, stx.elapsed_ms)
            hx.close()
        row["fp32_vs_fp64"] = row["fp32"]["proposals_per_s"] / row["fp64"]["proposals_per_s"]
        row["bf16_vs_fp64"] = row["bf16"]["proposals_per_s"] / row["fp64"]["proposals_per_s"]
        extra["e32_mixed_vs_fp64"] = row
        # the 16-electron system with a non-local pseudopotential (synthetic s
        # and p channels on its two cores, cutoff 1.3 bohr): per step the 6N
        # lattice moves plus six quadrature points per electron inside a sphere
        de = I.c1_ecp_system(n_walkers=4096)
        hx, px, r = run_cycles(B, de, "lb", steps_x, 1)
        wk = hx.walkers()
        Ra, rc = np.asarray(de["atom_pos"]), np.asarray(de["ecp_rcut"])
        dist = np.linalg.norm(wk["pos"].reshape(4096, -1, 1, 3) - Ra[None, None], axis=3)
        inside = float(((dist < rc[None, None]) & (rc[None, None] > 0)).any(axis=2).mean())
        extra["c1_ecp_fp64"] = dict(
            workload="16 electrons, 8 atoms, non-local s and p channels on the two cores, 4096 walkers, "
                     "a=0.2, N_proj=300, FP64",
            lattice_proposals_per_s=r["proposals"] / r["seconds"],
            proposals_per_s=r["proposals"] / r["seconds"] * (1.0 + inside),
            ms_per_branching=r["ms_per_cycle"], electrons_inside_spheres=inside,
            time_vs_local_only=r["ms_per_cycle"] / lb["ms_per_cycle"])
        hx.close()
        # adjoint pass: 4096 walkers, 24 nuclear coordinates + 15 Jastrow parameters
        c4 = I.c4_system(n_walkers=4096)
        ha = B.Handle(c4, B.params_for(c4, "lb", n_proj=10))
        ha.walker_derivs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ha.walker_derivs()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / 5
        extra["c4_adjoint"] = dict(walkers=4096, n_theta=ha.n_theta(), ms_per_call=ms,
                                   walker_gradients_per_s=4096 / (ms * 1e-3), precision="fp64")
        ha.close()
        res["extra"] = extra

    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
