"""Pins of the oracle's weight guards in the load-balanced scheme (Sec. II.C:
b_x = bbar / (W - E_0) is a weight only while W - E_0 > 0; reading: a walker
whose W - E_0 <= 0 at any step, or at the final configuration whose e_L and
W enter the walker average w / (W - E_0), gets weight zero and dies at the
reconfiguration).

The oracle's population phase is replayed here configuration by
configuration: the recorded moves are applied to the starting positions and
every configuration is evaluated on its own, and the log-weight is rebuilt as
the plain sum of log bbar - log(W - E_0) with the guard applied by hand."""
import numpy as np

import oracle as O
from paper_2508_12033_amd import inputs as I


def _replay(S, prm, d, pos0, moves, E0):
    a = prm.a
    lw = np.zeros(len(pos0))
    dead = np.zeros(len(pos0), bool)
    for w in range(len(pos0)):
        x = pos0[w].copy()
        acc = 0.0
        for k in range(prm.nproj + 1):
            ev = O.evaluate(S, prm, x)
            if not ev["W"] - E0 > 0:
                dead[w] = True
            elif k < prm.nproj:
                acc += np.log(ev["bbar"]) - np.log(ev["W"] - E0)
            if k < prm.nproj:
                p = int(moves[w, k])
                i, dd, s = p // 6, (p // 2) % 3, p % 2
                x[i, dd] += -a if s else a
        lw[w] = -np.inf if dead[w] else acc
    return lw, dead


def test_forced_e0_kills_exactly_the_violating_walkers():
    d = I.h2_system(n_walkers=48)
    S = O.System(d)
    prm = S.params(nproj=12)
    pos0 = np.array(d["init_pos"][:48], copy=True)
    W0 = np.array([O.evaluate(S, prm, pos0[w])["W"] for w in range(48)])
    # E_0 between the smallest and largest initial diagonal: part of the
    # population violates W - E_0 > 0 at some step, part never does
    E0 = float(np.quantile(W0, 0.4))
    pos = pos0.copy()
    lw = np.zeros(48)
    eL, W, moves, iters, cnt = O.population_phase(S, prm, "lb", 0, E0, pos, lw, nthreads=4)
    lw_ref, dead = _replay(S, prm, d, pos0, moves, E0)
    assert 5 < dead.sum() < 43, dead.sum()
    assert np.array_equal(~np.isfinite(lw), dead)
    assert cnt["neg_weight"] >= dead.sum()
    fin = ~dead
    assert np.max(np.abs(lw[fin] - lw_ref[fin])) < 1e-12 * max(1.0, np.abs(lw_ref[fin]).max())
    # the comb never selects a dead walker and keeps the population size
    sel, lwb, c = O.comb(lw, 0.37)
    assert len(sel) == 48 and np.all(np.isfinite(lw[sel]))
    # the walker average ignores the dead (zero-weight) walkers
    e = O.walker_average("lb", lw, eL, W, E0)
    w = np.exp(lw[fin] - lw[fin].max())
    om = w / (W[fin] - E0)
    assert abs(e - np.sum(om * eL[fin]) / np.sum(om)) < 1e-12 * abs(e)


def test_final_configuration_guard():
    """A walker that reaches a configuration with W - E_0 <= 0 only after its
    last move dies too (the estimator weight needs W - E_0 > 0 there)."""
    d = I.h2_system(n_walkers=64)
    S = O.System(d)
    prm = S.params(nproj=6)
    pos0 = np.array(d["init_pos"][:64], copy=True)
    # trajectories do not depend on E_0 (the heat bath uses the ratios only)
    pos = pos0.copy()
    lw = np.zeros(64)
    eL, W, moves, _, _ = O.population_phase(S, prm, "lb", 0, -1e9, pos, lw, nthreads=4)
    Wpath = np.zeros((64, prm.nproj + 1))
    for w in range(64):
        x = pos0[w].copy()
        for k in range(prm.nproj + 1):
            Wpath[w, k] = O.evaluate(S, prm, x)["W"]
            if k < prm.nproj:
                p = int(moves[w, k])
                x[p // 6, (p // 2) % 3] += -prm.a if p % 2 else prm.a
    # walkers whose final W is the lowest of their path: E_0 between
    cand = np.where(Wpath[:, -1] < Wpath[:, :-1].min(axis=1))[0]
    assert len(cand) > 0
    w0 = cand[0]
    E0 = 0.5 * (Wpath[w0, -1] + Wpath[w0, :-1].min())
    pos = pos0.copy()
    lw = np.zeros(64)
    O.population_phase(S, prm, "lb", 0, E0, pos, lw, nthreads=4)
    expect_dead = Wpath.min(axis=1) - E0 <= 0
    assert expect_dead[w0] and not np.isfinite(lw[w0])
    assert np.array_equal(~np.isfinite(lw), expect_dead)
