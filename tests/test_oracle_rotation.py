"""Pins of the oracle's randomized lattice (App. D: the three versors of the
discretized Laplacian rotate with random angles along the simulation;
reading: one random rotation per walker and projection phase).

1. The rotations are proper and orthonormal, and Haar-distributed: every
   entry has mean 0 and mean square 1/3, the trace (the character of the
   three-dimensional representation) has mean 0 and mean square 1.
2. Move ratios along rotated versors equal the quotients of two trial-function
   values computed independently in numpy (slogdet, pairwise Jastrow).
3. The exact hydrogenic eigenstate keeps e_L = -Z^2/2 under any orientation.
4. Fixed axes are the identity rotation: bit-identical results.
5. Within a phase every electron stays on its rotated lattice
   r_i(0) + a R Z^3, and a new phase draws a new rotation."""
import numpy as np

import oracle as O
from paper_2508_12033_amd import inputs as I
from test_oracle_local_energy import log_psi_np, ratio_np


def test_rotations_orthonormal_and_haar():
    Rs = np.array([O.rotation(12033, 1, slot, j) for slot in range(400) for j in range(5)])
    eye = np.einsum("nxd,nxe->nde", Rs, Rs)
    assert np.max(np.abs(eye - np.eye(3))) < 4e-16 * 8
    assert np.max(np.abs(np.linalg.det(Rs) - 1.0)) < 1e-14
    n = len(Rs)
    assert np.max(np.abs(Rs.mean(axis=0))) < 5.0 / np.sqrt(3 * n)
    assert np.max(np.abs((Rs ** 2).mean(axis=0) - 1 / 3)) < 5.0 * np.sqrt(0.08 / n)
    tr = np.trace(Rs, axis1=1, axis2=2)
    assert abs(tr.mean()) < 5.0 / np.sqrt(n)
    assert abs((tr ** 2).mean() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    # different walkers, branchings and seeds give different rotations
    assert not np.allclose(O.rotation(1, 0, 0, 0), O.rotation(1, 0, 1, 0))
    assert not np.allclose(O.rotation(1, 0, 0, 0), O.rotation(1, 0, 0, 1))
    assert not np.allclose(O.rotation(1, 0, 0, 0), O.rotation(2, 0, 0, 0))


def test_rotated_ratios_bruteforce():
    for d in (I.c4_system(n_walkers=4), I.h2_system(n_walkers=4)):
        S = O.System(d)
        prm = S.params(rotate=True)
        a = prm.a
        N = d["n_elec"]
        for w in range(3):
            pos = d["init_pos"][w].copy()
            R = O.rotation(prm.seed, prm.sysid, w, 3)
            ev = O.evaluate(S, prm, pos, rot=R)
            ref = log_psi_np(d, pos)
            for i in range(N):
                for dd in range(3):
                    for s in range(2):
                        st = a * R[:, dd]
                        r = pos[i] + (-st if s else st)
                        want = ratio_np(d, pos, ref, i, r)
                        got = ev["R"][(3 * i + dd) * 2 + s]
                        assert abs(got - want) < 1e-10 * max(1.0, abs(want)), (i, dd, s)


def test_fixed_axes_are_the_identity_rotation():
    d = I.c1_system(n_walkers=4)
    S = O.System(d)
    prm = S.params()
    for w in range(4):
        e1 = O.evaluate(S, prm, d["init_pos"][w])
        e2 = O.evaluate(S, prm, d["init_pos"][w], rot=np.eye(3))
        assert np.array_equal(e1["R"], e2["R"]) and e1["eL"] == e2["eL"] and e1["W"] == e2["W"]


def test_exact_eigenstate_any_orientation():
    for Z in (1.0, 2.0):
        d = I.hydrogenic_system(Z=Z, zeta=Z, n_walkers=16)
        S = O.System(d)
        prm = S.params(rotate=True)
        for w in range(16):
            R = O.rotation(7, 0, w, 0)
            ev = O.evaluate(S, prm, d["init_pos"][w], rot=R)
            assert abs(ev["eL"] + 0.5 * Z * Z) < 1e-12 * ev["W"]
        pos = d["init_pos"].copy()
        lw = np.zeros(16)
        eL, W, mv, it, cnt = O.population_phase(S, prm, "lb", 0, -0.5 * Z * Z, pos, lw, nthreads=2)
        assert np.all(np.abs(lw) < 1e-11) and np.all(np.abs(eL + 0.5 * Z * Z) < 1e-12 * W)


def test_moves_stay_on_the_rotated_lattice():
    d = I.c1_system(n_walkers=6)
    S = O.System(d)
    prm = S.params(rotate=True, nproj=40)
    pos0 = d["init_pos"][:6].copy()
    for j in (0, 1):
        pos = pos0.copy()
        lw = np.zeros(6)
        O.population_phase(S, prm, "lb", j, -30.0, pos, lw, nthreads=2)
        moved = False
        for w in range(6):
            R = O.rotation(prm.seed, prm.sysid, w, j)
            k = (pos[w] - pos0[w]) @ R / prm.a          # coordinates in the rotated frame
            assert np.allclose(k, np.round(k), atol=1e-9)
            moved |= np.any(np.abs(np.round(k)) > 0)
            # the same walker is not on the fixed-axis lattice
            kf = (pos[w] - pos0[w]) / prm.a
            if np.any(np.abs(np.round(k)) > 0):
                assert not np.allclose(kf, np.round(kf), atol=1e-6)
        assert moved
