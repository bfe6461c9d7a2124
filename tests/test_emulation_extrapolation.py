"""Host-side analysis pieces of the method, pinned without the GPU.

1. App. C emulation of the conventional scheme's load imbalance: with b held
   constant the iteration counts are 1 + Poisson(b tau), so their mean, the
   expected minimum and maximum over N_w walkers follow closed forms; the
   paper's own setting (tau = 5, b ~ Normal(1000, 0.5)) shows a constant mean
   and a maximum that grows like log N_w.
2. The a -> 0 extrapolation (Sec. II.A: O(a^2) lattice bias; Table I
   pattern): the weighted least-squares fit recovers exact coefficients, its
   error bar matches the scatter of fits to noisy data, and -- the physics
   pin -- the exact lowest eigenvalues of the one-electron lattice
   Hamiltonian of a smooth (softened-core) potential, extrapolated from
   a = 0.5 ... 0.2, reach the continuum ground-state energy obtained by an
   independent radial finite-difference solve."""
import numpy as np
from scipy.linalg import eigh_tridiagonal

from lattice_exact import lattice_lambda_min
from paper_2508_12033_amd import emulation as EM
from paper_2508_12033_amd import inputs as I
from paper_2508_12033_amd.extrapolation import fit_a2


def test_emulation_constant_rate_is_poisson():
    mu, nw, rep = 50.0, 400, 60
    rng = np.random.default_rng(7)
    maxima, minima, means, var = [], [], [], []
    m1 = EM.poisson_extremes(1, mu)
    assert abs(m1["max"] - (mu + 1)) < 1e-9 and abs(m1["std_max"] - np.sqrt(mu)) < 1e-6
    for _ in range(rep):
        c = EM.emulate_counts(nw, tau=mu / 1000.0, b_mean=1000.0, b_std=0.0, rng=rng)
        maxima.append(c.max()); minima.append(c.min()); means.append(c.mean()); var.append(c.var())
    model = EM.poisson_extremes(nw, mu)
    # mean of 1 + Poisson(mu), its variance mu
    assert abs(np.mean(means) - (mu + 1)) < 4 * np.sqrt(mu / (nw * rep))
    assert abs(np.mean(var) / mu - 1) < 0.05
    # expected extremes over nw walkers (their scatter is a few counts)
    assert abs(np.mean(maxima) - model["max"]) < 4 * np.std(maxima) / np.sqrt(rep)
    assert abs(np.mean(minima) - model["min"]) < 4 * np.std(minima) / np.sqrt(rep)


def test_emulation_paper_setting_log_growth():
    """tau = 5, b ~ Normal(1000, 0.5): the mean stays at b tau + 1 while the
    maximum grows with N_w as the Poisson-maximum model predicts."""
    rows = EM.emulate((10, 100, 1000, 10000), tau=5.0, b_mean=1000.0, b_std=0.5, seed=3)
    for r in rows:
        assert abs(r["mean"] - 5001.0) < 5 * np.sqrt(5000.0 / r["n_walkers"]) + 1
        m = EM.poisson_extremes(r["n_walkers"], 5000.0)
        assert abs(r["max"] - m["max"]) < 4 * m["std_max"] + 1
        assert abs(r["min"] - m["min"]) < 4 * m["std_min"] + 1
    assert rows[-1]["max"] > rows[0]["max"] and rows[-1]["min"] < rows[0]["min"]
    # the model's excess of the maximum approaches sqrt(2 mu ln N_w) from below
    for n in (100, 10000, 1000000):
        ex = EM.poisson_extremes(n, 5000.0)["max"] - 5001
        assert 0.75 < ex / np.sqrt(2 * 5000.0 * np.log(n)) < 1.0


def test_fit_recovers_exact_coefficients():
    a = np.array([0.1, 0.15, 0.2, 0.25, 0.3])
    E = -17.2345 - 0.0312 * a ** 2
    f = fit_a2(a, E, np.full(5, 1e-5))
    assert abs(f["E0"] + 17.2345) < 1e-12 and abs(f["coef"][1] + 0.0312) < 1e-10
    assert f["chi2"] < 1e-12 and f["dof"] == 3
    E4 = E + 0.4 * a ** 4
    f4 = fit_a2(a, E4, np.full(5, 1e-5), quartic=True)
    assert abs(f4["E0"] + 17.2345) < 1e-11 and abs(f4["coef"][2] - 0.4) < 1e-7


def test_fit_error_bar_matches_scatter():
    rng = np.random.default_rng(11)
    a = np.array([0.1, 0.2, 0.3])
    s = np.array([2e-5, 3e-5, 5e-5])
    est, errs = [], []
    for _ in range(4000):
        f = fit_a2(a, -1.0 + 0.02 * a ** 2 + s * rng.standard_normal(3), s)
        est.append(f["E0"]); errs.append(f["sigma_E0"])
    assert abs(np.mean(est) + 1.0) < 4 * np.std(est) / np.sqrt(4000)
    assert abs(np.std(est) / errs[0] - 1) < 0.05


def _radial_ground_state(Z, rc, n, R):
    h = R / (n + 1)
    r = h * np.arange(1, n + 1)
    d = 1.0 / h ** 2 - Z / np.sqrt(r * r + rc * rc)
    return eigh_tridiagonal(d, np.full(n - 1, -0.5 / h ** 2), select="i",
                            select_range=(0, 0))[0][0]


def test_lattice_energies_extrapolate_to_continuum():
    e1 = _radial_ground_state(2.0, 0.5, 20000, 30.0)
    e2 = _radial_ground_state(2.0, 0.5, 40000, 30.0)
    e_cont = (4 * e2 - e1) / 3            # Richardson: O(h^2) removed
    a = np.array([0.5, 0.45, 0.4, 0.35, 0.3, 0.25, 0.2])
    lam = np.array([lattice_lambda_min(I.one_electron_system("soft", n_walkers=4, a=x), 6.0)
                    for x in a])
    bias = lam - e_cont
    assert np.all(np.abs(bias) > 2e-4)            # the lattice bias is visible ...
    f = fit_a2(a, lam, np.full(len(a), 1e-6))
    assert abs(f["E0"] - e_cont) < 1e-4           # ... and extrapolates away as a^2
    assert abs(f["E0"] - e_cont) < 0.2 * np.abs(bias).min()
    resid = lam - (f["coef"][0] + f["coef"][1] * a ** 2)
    assert np.max(np.abs(resid)) < 0.1 * np.abs(bias).max()
