"""Statistical pins of the oracle's full LRDMC dynamics.

1. One electron on one lattice: both schemes must reproduce the lowest
   eigenvalue of the finite-a fixed-node lattice Hamiltonian, obtained here by
   sparse exact diagonalisation (stationarity results of App. A and App. B).
   The Hamiltonian is assembled by tests/lattice_exact.py from its definition
   in App. D (discrete Laplacian hops of -1/(2a^2), sign-violating hops moved
   to the spin-flip diagonal, regularized potential nu_opt), using only numpy
   values of the trial function -- the continuum Laplacian comes from a
   fourth-order finite-difference stencil, not from the oracle's analytic
   derivatives.
2. Conventional and load-balanced energies agree within error bars for a
   two-electron molecule (Sec. II.C, Sec. III).
"""
import numpy as np
import pytest

import oracle as O
from lattice_exact import lattice_lambda_min
from paper_2508_12033_amd import inputs as I


def _run(d, scheme, n_branch):
    return O.run(d, scheme, n_branch, nthreads=8)


@pytest.mark.slow
def test_one_electron_nodeless_lambda_min():
    d = I.one_electron_system("gauss", n_walkers=1000)
    lam = lattice_lambda_min(d, 9.0)
    for scheme in ("lb", "conv"):
        r = _run(d, scheme, 300)
        z = (r["E"] - lam) / r["sigma"]
        assert abs(z) < 3.5, (scheme, r["E"], r["sigma"], lam)
        assert r["sigma"] < 3e-3


@pytest.mark.slow
def test_one_electron_nodal_lambda_min():
    """p_z trial: the walkers stay in the z > 0 pocket; the fixed-node lattice
    energy includes V_sf and nu_opt (App. D)."""
    d = I.one_electron_system("nodal", n_walkers=2000, a=0.5)
    lam = lattice_lambda_min(d, 18.0)
    for scheme in ("lb", "conv"):
        r = _run(d, scheme, 600)
        assert np.all(r["pos"][:, 0, 2] > 0)
        z = (r["E"] - lam) / r["sigma"]
        assert abs(z) < 3.5, (scheme, r["E"], r["sigma"], lam)


@pytest.mark.slow
def test_conventional_equals_load_balanced_h2():
    """Sec. II.C / Sec. III: both schemes sample the same fixed-node state at
    fixed a when the mean number of moves per branching is matched."""
    d = I.h2_system(n_walkers=256)
    d["init_pos"] = d["init_pos"][:256]
    rc = O.run(d, "conv", 100, nthreads=8, tau=0.5)
    nbar = float(np.mean(rc["iters"]))
    rl = O.run(d, "lb", 100, nthreads=8, nproj=int(round(nbar)))
    z = (rc["E"] - rl["E"]) / np.hypot(rc["sigma"], rl["sigma"])
    assert abs(z) < 3.5, (rc["E"], rc["sigma"], rl["E"], rl["sigma"])
