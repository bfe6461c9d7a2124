"""Lattice-space series on the GPU (the pattern of Table I, Sec. II.A O(a^2)
bias) for one electron around a softened core -2/sqrt(r^2 + 0.25) with a
nodeless Gaussian trial function.

At every lattice space both schemes must reproduce the lowest eigenvalue of
the finite-a lattice Hamiltonian (brute-force sparse diagonalization, App. A /
App. B stationarity) and agree with each other (Sec. II.C, Sec. III); the
a -> 0 extrapolation of the GPU energies must reach the continuum
ground-state energy of the potential (independent radial solve)."""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

from lattice_exact import lattice_lambda_min
from paper_2508_12033_amd import inputs as I
from paper_2508_12033_amd.extrapolation import run_series
from parity_util import say

pytestmark = pytest.mark.gpu


def _continuum():
    out = []
    for n in (20000, 40000):
        h = 30.0 / (n + 1)
        r = h * np.arange(1, n + 1)
        d = 1.0 / h ** 2 - 2.0 / np.sqrt(r * r + 0.25)
        out.append(eigh_tridiagonal(d, np.full(n - 1, -0.5 / h ** 2), select="i",
                                    select_range=(0, 0))[0][0])
    return (4 * out[1] - out[0]) / 3


def test_soft_core_series_both_schemes():
    a_vals = (0.5, 0.4, 0.3)

    def make(a):
        return I.one_electron_system("soft", n_walkers=4096, a=a)

    say("case lattice-space series, one electron, soft core, a =", a_vals)
    res = run_series(make, a_vals, n_branchings=300, n_warm=30)
    e_cont = _continuum()
    for row in res["rows"]:
        lam = lattice_lambda_min(make(row["a"]), 6.0)
        for sch in ("lb", "conv"):
            E, s, n = row[sch]
            say("a %.2f %s E %.6f +- %.6f  lambda_min %.6f  z %.2f" % (row["a"], sch, E, s, lam,
                                                                     (E - lam) / s))
            assert abs(E - lam) < 3.5 * s
        say("a %.2f z(lb - conv) %.2f" % (row["a"], row["z"]))
        assert abs(row["z"]) < 3.5
    for sch in ("lb", "conv"):
        f = res["fits"][sch]
        say(sch, "E(a->0) = %.6f +- %.6f (continuum %.6f), c = %.5f, chi2 %.2f / %d"
            % (f["E0"], f["sigma_E0"], e_cont, f["coef"][1], f["chi2"], f["dof"]))
        assert abs(f["E0"] - e_cont) < 3.5 * f["sigma_E0"] + 1e-4
