"""Lattice-space extrapolation of LRDMC energies.

The lattice regularization biases the fixed-node energy by O(a^2) (Sec. II.A,
App. D), so energies are computed at several lattice spaces and extrapolated
to a -> 0 (the pattern of Table I).  fit_a2 is a weighted least-squares fit of
E(a) = E_0 + c a^2 (+ d a^4) with the statistical error bars as weights;
run_series drives the GPU library over a list of lattice spaces for both
schemes and returns the energies, their error bars, the scheme z-scores and
the fit.

Host-side analysis code: the energies come from the GPU library
(lrdmc_run + lrdmc_energy_forces); only the least-squares fit runs here.
"""
from __future__ import annotations

import numpy as np


def fit_a2(a, E, sigma, quartic=False):
    """Weighted least squares of E(a) = E_0 + c a^2 (+ d a^4).

    Returns dict(E0, sigma_E0, coef, cov, chi2, dof).  coef = [E0, c(, d)];
    cov from the inverse normal matrix (statistical error bars only)."""
    a = np.asarray(a, np.float64)
    E = np.asarray(E, np.float64)
    s = np.asarray(sigma, np.float64)
    cols = [np.ones_like(a), a ** 2] + ([a ** 4] if quartic else [])
    X = np.stack(cols, axis=1)
    if len(a) < X.shape[1]:
        raise ValueError("need at least %d lattice spaces" % X.shape[1])
    w = 1.0 / s ** 2
    A = X.T @ (w[:, None] * X)
    bvec = X.T @ (w * E)
    cov = np.linalg.inv(A)
    coef = cov @ bvec
    r = E - X @ coef
    chi2 = float(np.sum(w * r * r))
    return dict(E0=float(coef[0]), sigma_E0=float(np.sqrt(cov[0, 0])), coef=coef.tolist(),
                cov=cov.tolist(), chi2=chi2, dof=int(len(a) - X.shape[1]))


def run_series(make_system, a_values, schemes=("lb", "conv"), n_branchings=200, n_warm=20,
               precision="fp64", quartic=False, **param_kw):
    """Energies E(a) +- sigma for each lattice space and scheme on the GPU.

    make_system(a) -> generator dict for lattice space a (its tau = N_proj a^2
    / (3N) keeps about N_proj moves per branching in both schemes).  Each run:
    n_warm graph-replayed cycles, then n_branchings more, energy from the
    correcting-factor estimator over the whole history (first 10 % dropped).
    Returns dict(rows=[...], fits={scheme: fit_a2 result})."""
    from . import lrdmc as B
    rows = []
    for a in a_values:
        d = make_system(float(a))
        row = dict(a=float(a))
        for sch in schemes:
            prm = B.params_for(d, sch, precision=precision, **param_kw)
            h = B.Handle(d, prm)
            h.run(n_warm + n_branchings)
            E, sig, n = h.energy()
            h.close()
            row[sch] = (E, sig, n)
        if "lb" in row and "conv" in row:
            (e1, s1, _), (e2, s2, _) = row["lb"], row["conv"]
            row["z"] = float((e1 - e2) / np.hypot(s1, s2))
        rows.append(row)
    fits = {}
    for sch in schemes:
        fits[sch] = fit_a2([r["a"] for r in rows], [r[sch][0] for r in rows],
                           [r[sch][1] for r in rows], quartic=quartic)
    return dict(rows=rows, fits=fits)
