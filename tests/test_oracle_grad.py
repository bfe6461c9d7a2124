"""Pins of the oracle's parameter derivatives (fourth-order central differences
of its FP64 e_L and log|Psi_G|) against what the mathematics fixes: closed
forms of the Slater-orbital and Pade-Jastrow derivatives, the exact-eigenstate
property, and the invariance of a molecule under a rigid translation of all
nuclei and electrons."""
import numpy as np

import oracle as O
from paper_2508_12033_amd import inputs as I


def _pade_dp(A, B, b, r):
    """d u / d(A, B, b) of u(r) = (A r + B r^2) / (1 + b r)."""
    den = 1.0 + b * r
    return np.array([r / den, r * r / den, -r * (A * r + B * r * r) / den ** 2])


def test_hydrogenic_nuclear_and_en_jastrow_derivatives():
    """One electron, Slater 1s exp(-zeta |r - R|) times exp(u_en(|r - R|)):
    d log|Psi| / dR = (zeta - u'(r)) (r - R)/r, d log|Psi| / d(A, B, b) = du/dp;
    with u_en = 0 the trial state is exact, so d e_L / dR = 0."""
    d = I.hydrogenic_system(Z=1.0, zeta=1.0, n_walkers=6)
    for w in range(3):
        pos = d["init_pos"][w]
        deL, dlp, ok = O.gradient_fd(d, pos)
        assert ok.all()
        rv = pos[0] - d["atom_pos"][0]
        r = np.linalg.norm(rv)
        assert np.allclose(dlp[:3], rv / r, atol=1e-9)
        assert np.all(np.abs(deL[:3]) < 1e-8)
        assert np.allclose(dlp[9:12], _pade_dp(0.0, 0.0, 0.0, r), atol=1e-9)
    # a non-trivial electron-nucleus factor
    A, Bq, b = 0.3, 0.1, 0.8
    d2 = dict(d)
    jas = np.array(d["jastrow"], np.float64)
    jas[2] = (A, Bq, b)
    d2["jastrow"] = jas
    pos = d["init_pos"][1]
    deL, dlp, ok = O.gradient_fd(d2, pos)
    rv = pos[0] - d["atom_pos"][0]
    r = np.linalg.norm(rv)
    du = (A + 2 * Bq * r + Bq * b * r * r) / (1 + b * r) ** 2
    assert np.allclose(dlp[:3], (1.0 - du) * rv / r, atol=1e-9)
    assert np.allclose(dlp[9:12], _pade_dp(A, Bq, b, r), atol=1e-9)
    # e_L of exp(-r + u(r)) in closed form: -1/2 (f'' + 2 f'/r) - 1/r with
    # f = -r + u; its A-derivative by the chain rule through u
    def eL_of(Av):
        den = 1 + b * r
        up = (Av + 2 * Bq * r + Bq * b * r * r) / den ** 2
        upp = 2 * (Bq - Av * b) / den ** 3
        fp, fpp = -1.0 + up, upp
        return -0.5 * (fpp + 2 * fp / r + fp * fp) - 1.0 / r
    e_cf = (eL_of(A + 1e-6) - eL_of(A - 1e-6)) / 2e-6
    # the lattice e_L differs from the continuum one by O(a^2): compare the
    # lattice derivative with the continuum closed form at that order
    assert abs(deL[9] - e_cf) < 0.05 * max(1.0, abs(e_cf))


def test_two_electron_ee_jastrow_derivatives():
    """H2 (one up, one down electron): the antiparallel Pade row enters
    log|Psi| only through u(r_12), the parallel row not at all."""
    d = I.h2_system(n_walkers=4)
    M = d["atom_pos"].shape[0]
    for w in range(3):
        pos = d["init_pos"][w]
        deL, dlp, ok = O.gradient_fd(d, pos)
        A, Bq, b = d["jastrow"][1]
        r12 = np.linalg.norm(pos[0] - pos[1])
        assert np.allclose(dlp[3 * M + 3:3 * M + 6], _pade_dp(A, Bq, b, r12), atol=1e-9)
        assert np.all(np.abs(dlp[3 * M:3 * M + 3]) < 1e-9)
        assert np.all(np.abs(deL[3 * M:3 * M + 3]) < 1e-8)


def test_rigid_translation_invariance():
    """Moving every nucleus and every electron by the same vector changes
    neither log|Psi| nor the lattice e_L (the lattice moves are translated
    with them), so sum_I d/dR_I = -sum_i d/dr_i.  The electron side of
    log|Psi| is the oracle's analytic gradient; of e_L a difference in the
    electron coordinates.  A basis function that did not move with its
    nucleus, or a dropped electron-nucleus term, breaks this."""
    d = I.c4_system(n_walkers=4)
    M = d["atom_pos"].shape[0]
    S = O.System(d)
    prm = S.params()
    h = 1e-3
    for w in range(2):
        pos = d["init_pos"][w].copy()
        deL, dlp, ok = O.gradient_fd(d, pos, which=np.arange(3 * M))
        assert ok.all()
        out = O.evaluate(S, prm, pos)
        nuc_lp = dlp.reshape(M, 3).sum(0)
        assert np.allclose(nuc_lp, -out["grad"].sum(0), atol=1e-8)
        # electron side of e_L: difference of a common electron translation,
        # with a step whose stencil stays on one smooth piece of e_L
        _, _, pat0 = O.local_values(d, pos)
        el = np.zeros(3)
        for c in range(3):
            for hh in (h, h / 4, h / 16):
                v, same = [], True
                for s in (2, 1, -1, -2):
                    p2 = pos.copy()
                    p2[:, c] += s * hh
                    e, _, pat = O.local_values(d, p2)
                    same &= bool(np.array_equal(pat, pat0))
                    v.append(e)
                if same:
                    break
            assert same
            el[c] = (-v[0] + 8 * v[1] - 8 * v[2] + v[3]) / (12 * hh)
        assert np.allclose(deL.reshape(M, 3).sum(0), -el, atol=1e-6)


def test_difference_order():
    """Halving the step changes the fourth-order difference by little (its
    truncation error scales as h^4, so at h = 1e-3 it is about 1/15 of the
    change seen here): h = 1e-3 gives derivatives to ~1e-8."""
    d = I.c4_system(n_walkers=2)
    pos = d["init_pos"][0]
    which = np.array([0, 5, 13, 24, 27, 30, 33])
    a1, b1, ok1 = O.gradient_fd(d, pos, h=2e-3, which=which)
    a2, b2, ok2 = O.gradient_fd(d, pos, h=1e-3, which=which)
    assert ok1.all() and ok2.all()
    assert np.max(np.abs(a1 - a2)) < 2e-7
    assert np.max(np.abs(b1 - b2)) < 2e-7
