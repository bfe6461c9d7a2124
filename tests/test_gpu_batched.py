"""Several molecules with different electron counts advanced by one launch of
the mixed-precision phase kernel, graph-replayed cycles of phase and
reconfiguration, and the launch autotuner.

Bar: every system's trajectories match the FP64 oracle under the mixed
precision's stated errors (decisions identical up to band adoptions, FP64
estimator values 1e-9 Ha); a graph-replayed run is bit-identical to the same
cycles issued eagerly; tuning leaves walkers, weights, E_0 and the random
streams untouched."""
import numpy as np
import pytest

import oracle as O
from paper_2508_12033_amd import inputs as I
from paper_2508_12033_amd import lrdmc as B
from parity_util import TOL_EL, compare_phase, say

pytestmark = pytest.mark.gpu

BAND = 1e-4


def _systems(nws=(48, 24, 12)):
    out = []
    for d, nw in zip(I.c2_systems(), nws):
        d = dict(d)
        d["n_walkers_run"] = nw
        out.append(d)
    return out


def _handle(ds, nproj=24, **kw):
    prm = B.params_for(ds[0], "lb", precision=kw.pop("precision", "fp32"), n_proj=nproj,
                       trace_cap=nproj, **kw)
    return B.Handle(ds, prm), prm


def _check_system(d, prm, j, e0, pos0, lw0, g, idx):
    res = compare_phase(d, prm, "lb", j, e0, pos0, lw0, g, idx, band=BAND)
    c = res["cnt"]
    say(d["name"], {k: v for k, v in res.items() if k != "oracle"})
    assert c["hard_mismatch"] == 0 and c["singular"] == 0, res
    assert res["pos_equal"] and res["lw_dead_equal"], res
    assert res["eL_err"] < TOL_EL, res
    assert res["lw_err"] < 5e-6 * prm.n_proj, res
    return res


def test_one_launch_three_systems():
    """16, 32 and 64 electrons in one launch; each system keeps its own
    Philox key (system_id), E_0 and history."""
    ds = _systems()
    say("case batched 3 systems one launch")
    h, prm = _handle(ds)
    e0s = [h.e0(k) for k in range(3)]
    pos0 = [d["init_pos"][:d["n_walkers_run"]].copy() for d in ds]
    st = h.step()
    assert st.walker_iters == sum(d["n_walkers_run"] for d in ds) * prm.n_proj
    for k, d in enumerate(ds):
        g = h.walkers(k, trace=True)
        nw = d["n_walkers_run"]
        idx = np.array(sorted({0, nw // 2, nw - 1}))
        _check_system(d, prm, 0, e0s[k], pos0[k], np.zeros(nw), g, idx)
    h.close()


@pytest.mark.parametrize("separate", [False, True])
def test_graph_replay_matches_eager(separate):
    """lrdmc_run (one graph replay per cycle, device-side E_0 and history)
    against lrdmc_step + lrdmc_branch on an identical second handle, with all
    systems in one launch or one launch per system."""
    ds = _systems((32, 16, 8))
    say("case batched graph replay vs eager, separate launches" if separate else
        "case batched graph replay vs eager")
    ha, prm = _handle(ds, nproj=16)
    hb, _ = _handle(ds, nproj=16)
    if separate:
        ha.set_launch(0)
        hb.set_launch(0)
    eager = []
    for _ in range(4):
        ha.step()
        eager.append(ha.branch())
    st, bs = hb.run(4)
    assert st.walker_iters == 4 * sum(d["n_walkers_run"] for d in ds) * 16
    assert hb.branch_index() == ha.branch_index() == 4
    for k in range(3):
        ga, gb = ha.walkers(k), hb.walkers(k)
        assert np.array_equal(ga["pos"], gb["pos"])
        assert np.array_equal(ga["lw"], gb["lw"])
        assert np.array_equal(ga["eL"], gb["eL"])
        assert ha.e0(k) == hb.e0(k)
    assert bs.e_bar == eager[-1].e_bar and bs.e0 == eager[-1].e0
    assert bs.log_wbar == eager[-1].log_wbar and bs.n_distinct == eager[-1].n_distinct
    # further replays continue the same chain as further eager cycles
    ha.step(); ha.branch()
    hb.run(1)
    assert np.array_equal(ha.walkers(2)["pos"], hb.walkers(2)["pos"])
    ha.close(); hb.close()


def test_autotune_keeps_state_and_parity():
    ds = _systems((32, 16, 8))
    say("case batched autotune")
    h, prm = _handle(ds, nproj=16)
    h.step(); h.branch()
    before = [h.walkers(k) for k in range(3)]
    e0s = [h.e0(k) for k in range(3)]
    log = h.autotune(n_steps=4)
    say("tuning log", log)
    batched = [e for e in log if e[3] == -1]
    single = [e for e in log if e[3] >= 0]
    total = [e for e in log if e[3] == -2]
    assert len(batched) == 6 and len(single) == 9 and len(total) == 1
    assert {e[0] for e in batched} == {64, 128, 256}
    assert {e[3] for e in single} == {0, 1, 2}
    best_single = [min(e[2] for e in single if e[3] == k) for k in range(3)]
    assert abs(total[0][2] - sum(best_single)) <= 1e-3 * sum(best_single)
    after = [h.walkers(k) for k in range(3)]
    for a, b in zip(before, after):
        assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["lw"], b["lw"])
    assert [h.e0(k) for k in range(3)] == e0s
    # the next phase with the chosen launch still follows the oracle
    pos0 = [b["pos"].copy() for b in before]
    h.step()
    for k, d in enumerate(ds):
        g = h.walkers(k, trace=True)
        nw = d["n_walkers_run"]
        _check_system(d, prm, 1, e0s[k], pos0[k], before[k]["lw"], g, np.array([0, nw - 1]))
    h.close()


def test_separate_launches_match_oracle():
    """One launch per system (each with its own LDS block), larger systems
    first: the same walkers, decisions and estimator values as the oracle."""
    ds = _systems((24, 12, 6))
    say("case separate launches")
    h, prm = _handle(ds, nproj=20)
    h.set_launch(0, big_first=True)
    e0s = [h.e0(k) for k in range(3)]
    pos0 = [d["init_pos"][:d["n_walkers_run"]].copy() for d in ds]
    h.step()
    for k, d in enumerate(ds):
        g = h.walkers(k, trace=True)
        nw = d["n_walkers_run"]
        _check_system(d, prm, 0, e0s[k], pos0[k], np.zeros(nw), g, np.arange(nw))
    h.close()


@pytest.mark.parametrize("threads", [64, 128])
def test_small_blocks_match_oracle(threads):
    """The 64- and 128-thread workgroup variants of the mixed kernel, smallest
    system first in the launch."""
    ds = _systems((24, 12, 6))
    say("case batched", threads, "threads")
    h, prm = _handle(ds, nproj=20)
    h.set_launch(threads, big_first=False)
    e0s = [h.e0(k) for k in range(3)]
    pos0 = [d["init_pos"][:d["n_walkers_run"]].copy() for d in ds]
    h.step()
    for k, d in enumerate(ds):
        g = h.walkers(k, trace=True)
        nw = d["n_walkers_run"]
        _check_system(d, prm, 0, e0s[k], pos0[k], np.zeros(nw), g, np.array([0, nw - 1]))
    h.close()
