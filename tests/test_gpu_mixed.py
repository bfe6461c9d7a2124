"""Mixed-precision projection phase (orbital product on FP32 MFMA, or on BF16
MFMA with split operands; FP32 ratios, Jastrow sums and rank-one inverse
updates; FP64 positions, potentials, weights, the sums that form W, bbar and
e_L, the periodic Gauss-Jordan refresh, and an FP64 evaluation of e_L and W
at the end of every phase) against the FP64 oracle following the GPU's moves
on identical seeded inputs.

Errors stated per result:
  - move choices and conventional stopping decisions: identical, except
    decisions whose draw falls inside the relative band by which the mixed
    ratios can move a cumulative boundary (adopted and counted); positions
    therefore bit-exact;
  - e_L and W handed to the reconfiguration: FP64 evaluation, the FP64 bar
    (1e-9 Ha, 1e-12 relative);
  - log-weights: accumulate the per-step error of bbar and W of the mixed
    step; bound per step below;
  - per-step values of the mixed step at the final configuration (e_L, W,
    largest ratio error) from the library's precision report: printed, with
    the bounds below."""
import numpy as np
import pytest

import oracle as O
from paper_2508_12033_amd import inputs as I
from parity_util import TOL_EL, TOL_W_REL, compare_phase, make_handle, say

pytestmark = pytest.mark.gpu

BAND = dict(fp32=1e-4, bf16=1e-3)
LW_PER_STEP = dict(fp32=5e-6, bf16=5e-5)
RATIO_ERR = dict(fp32=1e-4, bf16=1e-3)
FP32_BAND = BAND["fp32"]


def _check(res, prec, nproj, report=None):
    c = res["cnt"]
    say(prec, {k: v for k, v in res.items() if k != "oracle"})
    assert c["singular"] == 0, res
    assert c["hard_mismatch"] == 0, res
    assert res["pos_equal"], res
    assert res["iters_equal"], res
    assert res["lw_dead_equal"], res
    assert res["eL_err"] < TOL_EL, res
    assert res["W_err"] < TOL_W_REL, res
    assert res["lw_err"] < LW_PER_STEP[prec] * nproj, res
    if report is not None:
        o = res["oracle"]
        e_step = np.abs(report[:, 0] - o["eL"]) / np.abs(o["eL"])
        w_step = np.abs(report[:, 1] - o["W"]) / np.abs(o["W"])
        say(prec, "mixed step at the final configuration: e_L rel err max %.2e median %.2e; "
            "W rel err max %.2e; ratio err max %.2e" % (e_step.max(), np.median(e_step),
                                                      w_step.max(), report[:, 3].max()))
        assert report[:, 3].max() < RATIO_ERR[prec]


def _run(d, scheme, nw, prec, band, **kw):
    h, d2, prm = make_handle(d, scheme, nw, precision=prec, **kw)
    e0 = h.e0()
    pos0 = d2["init_pos"][:nw].copy()
    st = h.step()
    g = h.walkers(trace=True)
    rep = h.precision_report()
    res = compare_phase(d2, prm, scheme, 0, e0, pos0, np.zeros(nw), g, np.arange(nw), band=band)
    res["report"] = rep
    h.close()
    return res, st


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_c1_lb(prec):
    d = I.c1_system(n_walkers=64)
    say("case mixed c1 lb", prec, "64 walkers x 60 steps")
    res, st = _run(d, "lb", 64, prec, BAND[prec], n_proj=60)
    _check(res, prec, 60, res["report"])
    assert st.n_refresh >= 64 * (60 // 16)


def test_mixed_c1_conv():
    d = I.c1_system(n_walkers=40)
    say("case mixed c1 conv fp32 40 walkers")
    res, st = _run(d, "conv", 40, "fp32", FP32_BAND, tau=0.05)
    _check(res, "fp32", int(res["oracle"]["iters"].max()), res["report"])


@pytest.mark.parametrize("nu_mode", [0, 1])
def test_mixed_en_jastrow_nu_modes(nu_mode):
    d = I.c4_system(n_walkers=32)
    say("case mixed c4 nu_mode", nu_mode)
    res, _ = _run(d, "lb", 32, "fp32", FP32_BAND, n_proj=40, nu_opt_mode=nu_mode)
    _check(res, "fp32", 40, res["report"])


def test_mixed_exact_eigenstate():
    """Hydrogen 1s trial: e_L = -1/2 at every step (reported: FP64; the mixed
    step itself: to FP32 accuracy)."""
    d = I.hydrogenic_system(Z=1.0, zeta=1.0, n_walkers=32)
    say("case mixed hydrogenic exact state")
    h, d2, prm = make_handle(d, "lb", 32, precision="fp32", n_proj=50)
    assert abs(h.e0() + 0.5) < 1e-12
    h.step()
    g = h.walkers()
    assert np.all(np.abs(g["eL"] + 0.5) < 1e-12), g["eL"]
    rep = h.precision_report()
    assert np.all(np.abs(rep[:, 0] + 0.5) < 1e-5), rep[:, 0]
    h.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_c3_sample(prec):
    """128 electrons, 640 basis functions, 64 orbitals per spin: four MFMA
    column tiles, several refreshes per phase."""
    d = I.c3_system(n_walkers=16)
    say("case mixed c3", prec, "16 walkers x 40 steps")
    res, st = _run(d, "lb", 16, prec, BAND[prec], n_proj=40)
    _check(res, prec, 40, res["report"])


def test_mixed_unequal_spins_256_threads():
    """64 up and 60 down electrons (the 128-electron system without its last
    four down electrons): the down block is narrower than the padded spin
    block, so the float4 pieces of its inverse carry padding columns, and its
    ratio products split 60 electrons over groups of adjacent lanes."""
    d = dict(I.c3_system(n_walkers=8))
    d["n_dn"] = 60
    d["n_elec"] = 124
    d["init_pos"] = np.ascontiguousarray(d["init_pos"][:, :124, :])
    say("case mixed unequal spins 64+60, 256 threads, 8 walkers x 30 steps")
    h, d2, prm = make_handle(d, "lb", 8, precision="fp32", n_proj=30)
    h.set_launch(256, big_first=True)
    e0 = h.e0()
    pos0 = d2["init_pos"][:8].copy()
    h.step()
    g = h.walkers(trace=True)
    rep = h.precision_report()
    res = compare_phase(d2, prm, "lb", 0, e0, pos0, np.zeros(8), g, np.arange(8), band=FP32_BAND)
    _check(res, "fp32", 30, rep)
    h.close()


def test_mixed_branching_gathers_state():
    """Three phases with reconfiguration between them: the gathered walker
    blocks (orbital data and inverses in HBM) must continue the trajectories
    of the selected parents exactly as the oracle does from their positions."""
    d = I.c1_system(n_walkers=64)
    say("case mixed c1 branching")
    nw, nproj = 64, 30
    h, d2, prm = make_handle(d, "lb", nw, precision="fp32", n_proj=nproj, p_corr=1)
    pos = d2["init_pos"][:nw].copy()
    lw = np.zeros(nw)
    e0 = h.e0()
    for j in range(3):
        h.step()
        g = h.walkers(trace=True)
        res = compare_phase(d2, prm, "lb", j, e0, pos, lw, g, np.arange(nw), band=FP32_BAND)
        _check(res, "fp32", nproj)
        bs = h.branch()
        gsel = h.walkers()["sel"]
        xi = O.uniform(prm.seed, 0, 0, j, 0, O.RNG_COMB)
        sel, _, cnt = O.comb(g["lw"], xi, follow=gsel)
        assert cnt["hard_mismatch"] == 0
        assert np.array_equal(sel, gsel)
        pos = res["oracle"]["pos"][sel].copy()
        lw = np.zeros(nw)
        e0 = bs.e0
        assert np.array_equal(h.walkers()["pos"], pos)


def test_mixed_set_walkers_rebuilds():
    """New positions from the host: the orbital data of every walker are
    rebuilt from them before the next phase."""
    d = I.c1_system(n_walkers=32)
    say("case mixed set_walkers")
    nw = 32
    h, d2, prm = make_handle(d, "lb", nw, precision="fp32", n_proj=20)
    e0 = h.e0()
    pos = d2["init_pos"][:nw][::-1].copy()
    h.set_walkers(pos)
    h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, "lb", 0, e0, pos, np.zeros(nw), g, np.arange(nw),
                        band=FP32_BAND)
    _check(res, "fp32", 20)
    h.close()
