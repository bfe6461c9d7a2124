"""FP64 phase kernel beyond 16 electrons, against the FP64 oracle (Alg. 1 and
2; App. D): the 32-electron molecule of the uneven set (16 atoms, 160 basis
functions, 16 orbitals per spin; it runs in the large-system layout, which
puts eight walkers on a CU against three for the LDS-resident one: orbital
product in chunks of 64 basis functions, one spin's inverse in LDS), the
64-electron molecule and the 128-electron system (the same layout, four and
two walkers per CU); with unequal spins the 32-electron system takes the
chunked layout with both inverses in LDS.

At this size the kernel takes its general paths, which the 16-electron tests
do not reach: two column tiles of the orbital product, the Sherman-Morrison
products as loops over 16-element rows, ratio and derivative products past
the first eight fetched values, two 16-lane rows per lattice point in the
7-point Jastrow pass (32 partners) and, with the electron-nucleus Jastrow
(48 partners), one point per pass with a wavefront reduction; the
reconfiguration in between gathers 32-electron walkers.  Unequal spin counts
give ragged per-spin widths at both sizes.  Bar as for the other
FP64 tests: moves, stopping decisions, comb selections and positions
bit-exact, e_L within 1e-9 Ha, W to 1e-12, log-weights to 1e-11."""
import numpy as np
import pytest

import oracle as O
from paper_2508_12033_amd import inputs as I
from parity_util import assert_phase_ok, compare_phase, make_handle, say

pytestmark = pytest.mark.gpu


def e32(nw, en=False):
    """The 32-electron system of the uneven set; en: with electron-nucleus
    Pade rows (A = -1/4, B = 0, b = 1) for every species."""
    if not en:
        d = dict(I.c2_systems(n_walkers=(2, nw, 2))[1])
        return d
    return I.molecule_system(2, 2, 12, 4, 2, nw, 0.2, 10.0 * 2.0 ** (1.0 / 3.0),
                             I.BASE_SEED + 40, system_id=1, name="e32_en",
                             en_jastrow=(-0.25, 0.0, 1.0))


def _two_phases(d, scheme, nw, **kw):
    h, d2, prm = make_handle(d, scheme, nw, **kw)
    assert int(d2["n_elec"]) == 32 and int(d2["n_basis"]) == 160
    e0 = h.e0()
    pos = d2["init_pos"][:nw].copy()
    lw = np.zeros(nw)
    for j in range(2):
        h.step()
        g = h.walkers(trace=True)
        res = compare_phase(d2, prm, scheme, j, e0, pos, lw, g, np.arange(nw))
        say(scheme, "phase", j, {k: v for k, v in res.items() if k != "oracle"})
        assert_phase_ok(res)
        bs = h.branch()
        after = h.walkers()
        xi = O.uniform(prm.seed, int(d2["system_id"]), 0, j, 0, O.RNG_COMB)
        sel, _, cnt = O.comb(g["lw"], xi, follow=after["sel"])
        assert cnt["hard_mismatch"] == 0 and np.array_equal(sel, after["sel"])
        assert np.array_equal(after["pos"], g["pos"][after["sel"]])
        pos = after["pos"].copy()
        lw = np.zeros(nw)
        e0 = bs.e0
    h.close()


@pytest.mark.parametrize("scheme,rotate", [("lb", False), ("conv", False), ("lb", True)])
def test_32e_two_phases(scheme, rotate):
    """Two phases with the reconfiguration between them; the conventional
    phase at tau = 0.04 (about 100 moves per walker) and the load-balanced one
    at N_proj = 140, past the 128-move refresh; fixed and randomly rotated
    lattice versors."""
    nw = 40
    say("case 32 electrons FP64", scheme, "rotated" if rotate else "fixed axes", nw, "walkers")
    kw = dict(tau=0.04) if scheme == "conv" else dict(n_proj=140)
    _two_phases(e32(nw), scheme, nw, rotate=rotate, **kw)


@pytest.mark.parametrize("nu_mode", [0, 2])
def test_32e_en_jastrow(nu_mode):
    """48 Jastrow partners per electron (32 electrons, 16 nuclei): the 7-point
    pass takes one point per pass with a wavefront reduction."""
    nw = 32
    say("case 32 electrons FP64 with e-n Jastrow, nu_mode", nu_mode)
    _two_phases(e32(nw, en=True), "lb", nw, n_proj=100, nu_opt_mode=nu_mode)


def test_32e_full_population_sampled():
    """The launch the benchmark times for the FP64 side of its mixed-versus-
    FP64 comparison: 4096 walkers, N_proj = 300; sampled walkers recomputed
    one by one by the oracle."""
    nw = 4096
    d = e32(nw)
    say("case 32 electrons FP64 full population", nw)
    h, d2, prm = make_handle(d, "lb", nw)
    e0 = h.e0()
    pos0 = d2["init_pos"].copy()
    st = h.step()
    g = h.walkers(trace=True)
    idx = np.array([0, 1, 63, 64, 1000, 2047, 3001, 4095])
    res = compare_phase(d2, prm, "lb", 0, e0, pos0, np.zeros(nw), g, idx)
    say({k: v for k, v in res.items() if k != "oracle"}, "elapsed ms", st.elapsed_ms)
    assert_phase_ok(res)
    assert st.walker_iters == nw * int(prm.n_proj)
    k = (g["pos"] - pos0) / d2["a"]
    assert np.allclose(k, np.round(k), atol=1e-9)
    assert np.all(np.isfinite(g["eL"])) and np.all(g["W"] - e0 > 0)
    h.close()


@pytest.mark.parametrize("which,n_dn,scheme", [("c1", 5, "lb"), ("e32", 13, "lb"), ("e32", 13, "conv")])
def test_unequal_spins(which, n_dn, scheme):
    """Fewer down than up electrons (the last down electrons removed): the
    down block is narrower than the padded spin block (5 of 8 and 13 of 16
    columns), so every per-spin loop and product runs with a ragged width."""
    nw = 24
    d = dict(I.c1_system(n_walkers=nw) if which == "c1" else e32(nw))
    n = int(d["n_up"]) + n_dn
    d["n_dn"] = n_dn
    d["n_elec"] = n
    d["init_pos"] = np.ascontiguousarray(d["init_pos"][:, :n, :])
    say("case unequal spins", which, d["n_up"], "+", n_dn, scheme)
    kw = dict(tau=0.04) if scheme == "conv" else dict(n_proj=140)
    h, d2, prm = make_handle(d, scheme, nw, **kw)
    e0 = h.e0()
    pos0 = d2["init_pos"][:nw].copy()
    h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, scheme, 0, e0, pos0, np.zeros(nw), g, np.arange(nw))
    say({k: v for k, v in res.items() if k != "oracle"})
    assert_phase_ok(res)
    h.close()


@pytest.mark.parametrize("scheme", ["lb", "conv"])
def test_128e_large_system_layout(scheme):
    """The 128-electron, 640-function system in FP64: its walker does not fit
    the LDS-resident layout, so the kernel reads the coefficient block and the
    Slater rows from global memory, keeps one spin's inverse in LDS and the
    refresh's left half in global memory (two walkers per CU).  Past the
    128-move refresh in the load-balanced phase; the conventional phase at
    tau = 0.01 (about 170 moves)."""
    nw = 6
    d = I.c3_system(n_walkers=nw)
    say("case 128 electrons FP64 (large-system layout)", scheme, nw, "walkers")
    kw = dict(tau=0.01) if scheme == "conv" else dict(n_proj=140)
    h, d2, prm = make_handle(d, scheme, nw, **kw)
    e0 = h.e0()
    pos0 = d2["init_pos"][:nw].copy()
    st = h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, scheme, 0, e0, pos0, np.zeros(nw), g, np.arange(nw))
    say({k: v for k, v in res.items() if k != "oracle"}, "elapsed ms", st.elapsed_ms)
    assert_phase_ok(res)
    bs = h.branch()
    after = h.walkers()
    assert np.array_equal(after["pos"], g["pos"][after["sel"]])
    h.close()


def test_64e_chunked_layout():
    """The 64-electron molecule of the uneven set (32 atoms, 320 basis
    functions, 32 orbitals per spin) in FP64: the large-system layout with the
    orbital product in five chunks of 64 functions and one spin's inverse in
    LDS, four walkers per CU; past the 128-move refresh."""
    nw = 6
    d = dict(I.c2_systems(n_walkers=(2, 2, nw))[2])
    say("case 64 electrons FP64 (large-system layout in chunks)", nw, "walkers")
    h, d2, prm = make_handle(d, "lb", nw, n_proj=140)
    assert int(d2["n_elec"]) == 64 and int(d2["n_basis"]) == 320
    e0 = h.e0()
    pos0 = d2["init_pos"][:nw].copy()
    h.step()
    g = h.walkers(trace=True)
    res = compare_phase(d2, prm, "lb", 0, e0, pos0, np.zeros(nw), g, np.arange(nw))
    say({k: v for k, v in res.items() if k != "oracle"})
    assert_phase_ok(res)
    h.close()
