"""Emulation of the conventional scheme's load imbalance (App. C).

A toy model of the conventional continuous-time projection (Algorithm 1):
every walker draws persistence times tau_xi = -log(1 - xi) / b (Sec. II.B,
continuous-time limit of the diagonal moves) with b sampled from a normal
distribution at every iteration, subtracts them from its projection time tau
until tau_left reaches zero, and counts its iterations.  The branching has to
wait for the slowest walker, so the cost of a branching cycle of the batched
conventional scheme is the maximum iteration count over the N_w walkers, which
grows like log N_w while the mean stays fixed.  The paper's emulation uses
tau = 5 and b ~ Normal(1000, 0.5).

Also here: the Poisson model of the same counts (b held constant, the
number of persistence intervals that fit in tau is Poisson(b tau), plus the
final iteration that uses up tau_left), with the expected minimum and maximum
over N_w independent walkers, E[max] = sum_k (1 - F(k)^N_w).

Host-side analysis code (numpy); nothing here runs on the GPU.
"""
from __future__ import annotations

import numpy as np


def emulate_counts(n_walkers, tau=5.0, b_mean=1000.0, b_std=0.5, rng=None, seed=0):
    """Iterations per walker of one conventional projection phase of length
    tau (Algorithm 1 loop: draw xi, tau_xi = min(-log(1 - xi)/b, tau_left),
    tau_left -= tau_xi, stop when tau_left = 0).  Returns an int array
    [n_walkers]."""
    rng = np.random.default_rng(seed) if rng is None else rng
    tau_left = np.full(n_walkers, float(tau))
    iters = np.zeros(n_walkers, np.int64)
    active = np.arange(n_walkers)
    while active.size:
        xi = rng.random(active.size)
        b = rng.normal(b_mean, b_std, active.size) if b_std > 0 else np.full(active.size, b_mean)
        t = -np.log1p(-xi) / b
        left = tau_left[active]
        stop = ~(t < left)
        tau_left[active] = np.where(stop, 0.0, left - t)
        iters[active] += 1
        active = active[~stop]
    return iters


def emulate(n_walkers_list=(10, 100, 1000, 10000, 100000), tau=5.0, b_mean=1000.0, b_std=0.5,
            seed=12033):
    """Minimum, mean and maximum iteration counts per N_w (the figure of
    App. C).  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    out = []
    for nw in n_walkers_list:
        c = emulate_counts(int(nw), tau, b_mean, b_std, rng=rng)
        out.append(dict(n_walkers=int(nw), min=int(c.min()), mean=float(c.mean()),
                        max=int(c.max())))
    return out


def _poisson_cdf(k, mu):
    from scipy.stats import poisson
    return poisson.cdf(k, mu)


def poisson_extremes(n_walkers, mu):
    """Expected minimum, mean and maximum over n_walkers of (X + 1),
    X ~ Poisson(mu): the iteration counts of walkers with a constant rate
    b = mu / tau; also the standard deviations of the minimum and maximum
    (E[M] = sum_k P(M > k), E[M^2] = sum_k (2k + 1) P(M > k))."""
    k = np.arange(0, int(mu + 40.0 * np.sqrt(mu + 1.0) + 100))
    F = _poisson_cdf(k, mu)
    pmax = 1.0 - F ** n_walkers          # P(max > k)
    pmin = (1.0 - F) ** n_walkers        # P(min > k)
    emax, emin = float(np.sum(pmax)), float(np.sum(pmin))
    smax = float(np.sqrt(max(0.0, np.sum((2 * k + 1) * pmax) - emax ** 2)))
    smin = float(np.sqrt(max(0.0, np.sum((2 * k + 1) * pmin) - emin ** 2)))
    return dict(min=emin + 1.0, mean=mu + 1.0, max=emax + 1.0, std_min=smin, std_max=smax)


def lockstep_time_ratio(n_walkers, mu):
    """Predicted cost of the lockstep-masked conventional phase over a
    load-balanced phase of the same mean length: E[max]/E[mean]."""
    p = poisson_extremes(n_walkers, mu)
    return p["max"] / p["mean"]
