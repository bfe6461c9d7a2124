"""GPU (HIP, gfx950) projection phase and reconfiguration against the FP64 CPU
oracle on identical seeded inputs, element by element.

Bar: move choices, conventional stopping decisions, comb selections and
positions bit-exact (decisions inside the 1e-12 ambiguity band are adopted
and counted, and must be rare); e_L within 1e-9 Ha; W and the log-weights
within 1e-12 relative (log-weights: 1e-11, one rounding per step)."""
import numpy as np
import pytest

import oracle as O
from paper_2508_12033_amd import inputs as I
from parity_util import assert_phase_ok, compare_phase, make_handle, say

pytestmark = pytest.mark.gpu


def _initial_e0(d, nw, nu_mode):
    S = O.System(d)
    prm = S.params(nu_opt_mode=nu_mode)
    return np.mean([O.evaluate(S, prm, d["init_pos"][w])["eL"] for w in range(nw)])


@pytest.mark.parametrize("scheme", ["lb", "conv"])
def test_h2_phase_all_walkers(scheme):
    d = I.h2_system(n_walkers=256)
    say("case h2 phase", scheme, "256 walkers")
    h, d2, prm = make_handle(d, scheme, 256)
    e0 = h.e0()
    e0_orc = _initial_e0(d2, 256, prm.nu_opt_mode)
    assert abs(e0 - e0_orc) < 1e-11 * max(1.0, abs(e0_orc))
    pos0 = d2["init_pos"][:256].copy()
    st = h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, scheme, 0, e0, pos0, np.zeros(256), g, np.arange(256))
    say(scheme, {k: v for k, v in res.items() if k != "oracle"})
    assert_phase_ok(res)
    assert st.walker_iters == int(g["iters"].sum())
    assert st.max_iters == int(g["iters"].max())
    h.close()


@pytest.mark.parametrize("scheme", ["lb", "conv"])
@pytest.mark.parametrize("nw", [1, 70])
def test_c1_phase_small(scheme, nw):
    """16 electrons, 80 basis functions: several LDS tiles per walker, a walker
    count that is not a multiple of anything, and the single-walker edge."""
    d = I.c1_system(n_walkers=max(nw, 2))
    say("case c1 phase", scheme, nw, "walkers")
    h, d2, prm = make_handle(d, scheme, nw, n_proj=60, tau=0.05)
    e0 = h.e0()
    pos0 = d2["init_pos"][:nw].copy()
    h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, scheme, 0, e0, pos0, np.zeros(nw), g, np.arange(nw))
    say(scheme, nw, {k: v for k, v in res.items() if k != "oracle"})
    assert_phase_ok(res)
    h.close()


@pytest.mark.parametrize("nu_mode", [0, 1, 2])
def test_nu_modes_and_en_jastrow(nu_mode):
    """The three regularized-potential modes (App. D) and the
    electron-nucleus Jastrow terms."""
    d = I.c4_system(n_walkers=48)
    say("case c4 nu_mode", nu_mode)
    h, d2, prm = make_handle(d, "lb", 48, n_proj=40, nu_opt_mode=nu_mode)
    e0 = h.e0()
    pos0 = d2["init_pos"][:48].copy()
    h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, "lb", 0, e0, pos0, np.zeros(48), g, np.arange(48))
    say(nu_mode, {k: v for k, v in res.items() if k != "oracle"})
    assert_phase_ok(res)
    h.close()


def test_c1_full_population_sampled():
    """The benchmark's workload and launch: 4096 walkers, N_proj = 300, one
    phase; sampled walkers recomputed one by one by the oracle."""
    d = I.c1_system(n_walkers=4096)
    say("case c1 full population 4096 walkers, 300 steps")
    h, d2, prm = make_handle(d, "lb", 4096)
    e0 = h.e0()
    pos0 = d2["init_pos"].copy()
    st = h.step()
    g = h.walkers(trace=True)
    idx = np.array([0, 1, 63, 64, 1000, 2047, 3001, 4095])
    res = compare_phase(d2, prm, "lb", 0, e0, pos0, np.zeros(4096), g, idx)
    say({k: v for k, v in res.items() if k != "oracle"}, "elapsed ms", st.elapsed_ms)
    assert_phase_ok(res)
    assert st.walker_iters == 4096 * 300
    # properties at any size: every walker moved on its own lattice
    k = (g["pos"] - pos0) / d2["a"]
    assert np.allclose(k, np.round(k), atol=1e-9)
    assert np.all(np.isfinite(g["eL"])) and np.all(g["W"] - e0 > 0)
    h.close()


def test_exact_eigenstate_on_gpu():
    """Hydrogen 1s trial: e_L = -1/2 at every step; conventional weights are
    exp(tau/2) exactly; a one-electron system with no spin-down electrons."""
    d = I.hydrogenic_system(Z=1.0, zeta=1.0, n_walkers=64)
    say("case hydrogenic exact state")
    h, d2, prm = make_handle(d, "conv", 64)
    assert abs(h.e0() + 0.5) < 1e-12
    h.step()
    g = h.walkers()
    assert np.all(np.abs(g["eL"] + 0.5) < 1e-12)
    assert np.allclose(g["lw"], 0.5 * prm.tau, rtol=1e-12)
    h.close()


@pytest.mark.parametrize("scheme", ["lb", "conv"])
def test_h2_run_with_branching(scheme):
    """Co-simulation over 8 branchings: phases, comb selections (bit-exact),
    walker-averaged energies, E_0 updates and the gathered populations."""
    d = I.h2_system(n_walkers=256)
    say("case h2 run with branching", scheme)
    nproj, tau = 100, 0.7
    h, d2, prm = make_handle(d, scheme, 256, n_proj=nproj, tau=tau, p_corr=2)
    S = O.System(d2)
    op = S.params(a=prm.a, tau=prm.tau, nproj=prm.n_proj, nu_opt_mode=prm.nu_opt_mode,
                  seed=prm.seed)
    pos = d2["init_pos"][:256].copy()
    lw = np.zeros(256)
    e0 = h.e0()
    hist, lwb_hist = [], []
    for j in range(8):
        h.step()
        g = h.walkers(trace=True)
        res = compare_phase(d2, prm, scheme, j, e0, pos, lw, g, np.arange(256))
        assert_phase_ok(res)
        o = res["oracle"]
        ebar = O.walker_average(scheme, o["lw"], o["eL"], o["W"], e0)
        xi = O.uniform(prm.seed, 0, 0, j, 0, O.RNG_COMB)
        bs = h.branch()
        gsel = h.walkers()["sel"]
        sel, lwb, cnt = O.comb(g["lw"], xi, follow=gsel)
        assert cnt["hard_mismatch"] == 0
        assert np.array_equal(sel, gsel)
        assert abs(bs.e_bar - ebar) < 1e-10 * max(1.0, abs(ebar))
        assert abs(bs.log_wbar - lwb) < 1e-11 * max(1.0, abs(lwb))
        hist.append(ebar)
        lwb_hist.append(lwb)
        e0_orc = O.e0_update(hist)
        assert abs(bs.e0 - e0_orc) < 1e-10 * max(1.0, abs(e0_orc))
        pos = o["pos"][sel].copy()
        lw = np.zeros(256)
        e0 = bs.e0
        g2 = h.walkers()
        assert np.array_equal(g2["pos"], pos)
        assert np.all(g2["lw"] == 0.0)
        say(j, "ebar", bs.e_bar, "E0", bs.e0, "distinct", bs.n_distinct)
    E, sig, n = h.energy()
    # oracle estimator on the same history (first 10 % dropped, p = 2)
    Eo, so, no = O.energy_estimate(lwb_hist, hist, p=2)
    assert n == no == 6
    assert abs(E - Eo) < 1e-10 * max(1.0, abs(Eo))
    assert abs(sig - so) < 1e-8 * max(1e-3, abs(so))
    h.close()
