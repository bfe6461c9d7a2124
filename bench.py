"""Benchmark of the lattice-regularized DMC hot path on one MI355X.

Workload (one step = one pass of the hot path): one load-balanced projection
phase of N_proj = 300 lattice moves for every walker (ratios of all 6N moves,
local energy, weight update, heat-bath move, Sherman-Morrison update, FP64
refreshes) followed by the reconfiguration, on the 16-electron / 8-atom
synthetic molecule with 4096 walkers in FP64.  Inputs are resident in HBM
before the timed region.

Metric: electron-move proposals per second = walker-iterations that evaluated
all 6N move ratios x 6N / wall time.  Printed beside it: the conventional
(continuous-time) scheme on the same system at matched mean iterations, the
load-balanced-over-conventional speedup, the roofline of the phase kernel and
the CPU oracle's throughput on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-conv]
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
KERNEL_SOURCES = ["paper_2508_12033_amd/csrc/lrdmc_phase.hip",
                  "paper_2508_12033_amd/csrc/lrdmc_dev.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phase_fp64_c1_traffic.json")


def flops_per_walker_step(N, n, Nb, M, has_en, refresh_every):
    """Algorithmic FP64 operations of one incremental walker-step (exp, log,
    sqrt and division count as one operation each):
      basis functions of the moved electron at its position and 6 neighbours
      (+ gradient, Laplacian) ~ 85 Nb; orbital rows 2*11*Nb*n; Sherman-Morrison
      4 n^2; determinant ratios of the moved spin 12 n^2; ratios of all moves
      2P; Jastrow pair differences (N-1)*166 + (P-6)*35 (+ nuclei); local
      energy N(8n+20) + 2P; heat bath 2P; the FP64 refresh (Gauss-Jordan 8 n^3
      over both spins and the full Jastrow N(N-1)*137) divided by its cadence."""
    P = 6 * N
    f = 85 * Nb + 2 * 11 * Nb * n + 4 * n * n + 12 * n * n + 2 * P
    f += (N - 1) * 166 + (P - 6) * 35 + M * (145 if has_en else 8)
    f += N * (8 * n + 20) + 2 * P + 2 * P
    refresh = 8 * n ** 3 + N * ((N - 1) * 137 + M * (137 if has_en else 8))
    return f + refresh / refresh_every


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per phase launch from the committed rocprofv3 counter runs,
    or None when the kernel sources changed since they were taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(d, n_walk=2048, n_steps=100):
    """The FP64 oracle as it stands, all host cores, on a bounded sample: the
    first n_walk walkers of the same system for n_steps load-balanced steps."""
    import oracle as O
    S = O.System(d)
    prm = S.params(nproj=n_steps)
    pos = np.array(d["init_pos"][:n_walk], copy=True)
    lw = np.zeros(n_walk)
    nt = os.cpu_count() or 1
    e0 = -20.0
    t0 = time.perf_counter()
    O.population_phase(S, prm, "lb", 0, e0, pos, lw, nthreads=nt, record=False)
    dt = time.perf_counter() - t0
    return dict(value=n_walk * n_steps * S.P / dt, unit="proposals/s", cores=nt, kind="oracle",
                sample="%d walkers x %d load-balanced steps of the 16-electron system "
                       "(%.1f s wall)" % (n_walk, n_steps, dt))


def run_scheme(B, d, scheme, steps, warmup, **kw):
    import torch
    prm = B.params_for(d, scheme, **kw)
    h = B.Handle(d, prm)
    N = d["n_elec"]
    for _ in range(warmup):
        h.step(stats=False)
        h.branch()
    torch.cuda.synchronize()
    iters, kms, maxit, bms = 0, [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = h.step(stats=True)
        bs = h.branch()
        iters += st.walker_iters
        kms.append(st.elapsed_ms)
        maxit.append(st.max_iters)
        bms.append(bs.elapsed_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nw = d["init_pos"].shape[0]
    out = dict(proposals=iters * 6 * N, seconds=dt, walker_iters=iters,
               kernel_ms=float(np.mean(kms)), branch_ms=float(np.mean(bms)),
               max_iters=float(np.mean(maxit)), mean_iters=iters / (steps * nw),
               occupancy=iters / (steps * nw * float(np.mean(maxit))), e0=h.e0())
    h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-conv", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the walker population of one GPU is the unit of work)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2508_12033_amd import inputs as I
    from paper_2508_12033_amd import lrdmc as B
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    d = I.c1_system(n_walkers=4096)
    nw, N, n_proj = 4096, d["n_elec"], d["n_proj"]

    lb = run_scheme(B, d, "lb", args.steps, args.warmup)
    value = lb["proposals"] / lb["seconds"]
    ms_per_step = 1e3 * lb["seconds"] / args.steps

    fl = flops_per_walker_step(N, d["n_up"], d["n_basis"], d["n_atoms"], 0, 16)
    achieved = fl * nw * n_proj / (lb["kernel_ms"] * 1e-3) / 1e12
    tr = traffic_per_launch()
    roof = dict(bound="alu", kernel="phase_fp64", achieved=achieved, peak=FP64_PEAK_TFLOPS,
                unit="TFLOP/s", frac=achieved / FP64_PEAK_TFLOPS, traffic=tr,
                flops_per_walker_step=fl, launch_ms=lb["kernel_ms"])

    res = dict(metric=METRIC, value=value, unit="proposals/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="16-electron 8-atom synthetic molecule (1 C-like and 1 "
                                    "O-like soft core, 6 protons, 80 s/p Gaussians), 4096 "
                                    "walkers, a=0.2 bohr, load-balanced N_proj=300, FP64",
                           walkers=nw, electrons=N, n_proj=n_proj, precision="fp64",
                           scheme="load-balanced"),
               roofline=roof,
               branch_ms=lb["branch_ms"])

    if not args.no_conv:
        cv = run_scheme(B, d, "conv", args.steps, args.warmup)
        nbar = cv["mean_iters"]
        lbm = run_scheme(B, d, "lb", args.steps, 1, n_proj=int(round(nbar)))
        t_conv = cv["seconds"] / args.steps
        t_lbm = lbm["seconds"] / args.steps
        # Poisson model of the lockstep maximum (iterations ~ 1 + Poisson(nbar - 1))
        from scipy.stats import poisson
        mu = nbar - 1.0
        k = np.arange(0, int(mu + 40 * np.sqrt(mu) + 100))
        emax = float(np.sum(1.0 - poisson.cdf(k, mu) ** nw)) + 1.0
        res["conventional"] = dict(
            tau=d["tau"], mean_iters=nbar, max_iters=cv["max_iters"], lane_occupancy=cv["occupancy"],
            proposals_per_s=cv["proposals"] / cv["seconds"], ms_per_branching=1e3 * t_conv,
            kernel_ms=cv["kernel_ms"], poisson_model_max_iters=emax,
            poisson_model_time_ratio=emax / nbar)
        res["lb_matched"] = dict(n_proj=int(round(nbar)), ms_per_branching=1e3 * t_lbm,
                                 kernel_ms=lbm["kernel_ms"])
        res["speedup_vs_conventional"] = t_conv / t_lbm

    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
