"""Pins of the oracle's non-local pseudopotential (App. D: the non-local
elements V^nl_{x',x} of the fixed-node Hamiltonian under the determinant
locality approximation, i.e. with D_G(x')/D_G(x) in place of the
guiding-function ratio).

Reading: the semi-local channels v_l(r) of an atom act on an electron inside
the atom's cutoff sphere; the angular integral of the projector onto channel l
is the 6-point octahedral quadrature of the sphere through the electron, along
the walker's lattice versors, so that each quadrature point is one proposal
with element V_q = sum_l (2l + 1)/6 v_l(r) P_l(cos theta_q).

1. Closed forms on one electron (no Jastrow factor, so the determinant ratio
   is the full ratio): a trial function of pure angular momentum L about the
   atom (Slater 1s or s Gaussian: L = 0; p_z Gaussian: L = 1) is projected
   exactly by the quadrature (degree <= 3), so the local energy changes by
   exactly v_L(r), and by 0 for a channel l != L, in every lattice orientation.
   With the hydrogen 1s state the lattice local energy is -1/2 + v_0(r).  The
   sign of V_q D(x')/D(x) decides where the element goes: into the spin-flip
   term of W (positive) or into the move rates bbar (negative).
2. A second evaluation at configurations of the 16-electron molecule with
   channels on its two cores: quadrature points, Legendre weights, the
   determinant ratios by numpy.linalg.slogdet, the element signs split
   between W and bbar, and the node indicators of the non-local proposals.
3. A non-local move puts the electron on the sphere at the chosen point.
4. Each of a set of deliberate mistakes planted in the oracle source fails at
   least one of the checks above.
"""
import numpy as np
import pytest

import oracle as O
from paper_2508_12033_amd import inputs as I

TOL = 1e-9


def random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def vl(terms, l, r):
    """v_l(r) of a list of (l, power, coefficient, exponent) terms."""
    return sum(c * r ** k * np.exp(-b * r * r) for (ll, k, c, b) in terms if ll == l)


# --------------------------------------------------------------------------
# 1. closed forms on one electron
# --------------------------------------------------------------------------
def one_electron(kind):
    if kind == "slater":
        d = I.hydrogenic_system(Z=1.0, zeta=1.0, n_walkers=16)
    elif kind == "sgauss":
        d = I.one_electron_system("gauss", n_walkers=16)
    else:
        d = I.one_electron_system("nodal", n_walkers=16)
    return d


ANGULAR = {"slater": 0, "sgauss": 0, "pz": 1}


def closed_form_checks():
    """List of failure messages (empty when every closed form holds)."""
    bad = []
    rng = np.random.default_rng(5)
    for kind, L in ANGULAR.items():
        d0 = one_electron(kind)
        for l in (0, 1, 2):
            for terms in ([(l, 0, 2.5, 0.7)], [(l, 2, -1.5, 0.4)], [(l, 1, 0.8, 0.3), (l, 0, -3.0, 1.1)]):
                d = I.with_ecp(d0, [0], terms=terms, rcut=30.0)
                S0, S = O.System(d0), O.System(d)
                p0, p = S0.params(nu_opt_mode=2), S.params(nu_opt_mode=2)
                for t in range(4):
                    pos = np.array([[0.3, -0.5, 0.8]]) + 0.6 * rng.standard_normal((1, 3))
                    rot = None if t == 0 else random_rotation(rng)
                    e0 = O.evaluate(S0, p0, pos, rot=rot)
                    e = O.evaluate(S, p, pos, rot=rot)
                    r = float(np.linalg.norm(pos[0] - d["atom_pos"][0]))
                    want = vl(terms, l, r) if l == L else 0.0
                    got = e["eL"] - e0["eL"]
                    if abs(got - want) > TOL * max(1.0, abs(e0["eL"])):
                        bad.append("%s l=%d: dE_L %.3e want %.3e" % (kind, l, got, want))
                    if abs(e["vnl"] - want) > TOL:
                        bad.append("%s l=%d: V_nl %.3e want %.3e" % (kind, l, e["vnl"], want))
                    if abs(e["eL_cont"] - e0["eL_cont"] - want) > TOL * max(1.0, abs(e0["eL"])):
                        bad.append("%s l=%d: continuum e_L misses the non-local energy" % (kind, l))
                    if kind == "slater" and l == 0:
                        # hydrogen 1s: exact eigenstate of the local part; no
                        # proposal crosses a node, so nu_opt = nu_zv
                        e1 = O.evaluate(S, S.params(nu_opt_mode=0), pos, rot=rot)
                        if abs(e1["eL"] - (-0.5 + want)) > 1e-10:
                            bad.append("1s: e_L %.12f want %.12f" % (e1["eL"], -0.5 + want))
                        # spherically symmetric: every ratio is 1, every element
                        # has the sign of v_0 (W when positive, bbar when negative)
                        v0 = vl(terms, 0, r)
                        dW, db = e["W"] - e0["W"], e["bbar"] - e0["bbar"]
                        wW, wb = (v0, 0.0) if v0 > 0 else (0.0, -v0)
                        if abs(dW - wW) > TOL * max(1.0, abs(e0["W"])) or \
                                abs(db - wb) > TOL * max(1.0, abs(e0["bbar"])):
                            bad.append("1s sign split: dW %.3e dbbar %.3e want %.3e %.3e" % (dW, db, wW, wb))
                    if kind == "pz" and l == 1 and t > 0:
                        # points on both sides of the nodal plane: node flag set
                        pm = S.params(nu_opt_mode=0)
                        if O.evaluate(S, pm, pos, rot=rot)["node"][0] != 1:
                            bad.append("pz: non-local proposal across the node not flagged")
        # outside the cutoff sphere nothing changes
        d = I.with_ecp(d0, [0], terms=[(L, 0, 2.5, 0.7)], rcut=0.4)
        S0, S = O.System(d0), O.System(d)
        p0, p = S0.params(nu_opt_mode=2), S.params(nu_opt_mode=2)
        pos = np.array([[0.5, 0.45, -0.3]])
        e0, e = O.evaluate(S0, p0, pos), O.evaluate(S, p, pos)
        if e["eL"] != e0["eL"] or np.any(e["R"][6:] != 0.0):
            bad.append("%s: channels act outside the cutoff sphere" % kind)
    return bad


def test_closed_forms():
    bad = closed_form_checks()
    assert bad == [], bad[:5]


# --------------------------------------------------------------------------
# 2. independent evaluation on a molecule
# --------------------------------------------------------------------------
def basis_np(d, r):
    R = d["atom_pos"][d["basis_atom"]]
    x = np.asarray(r, np.float64)[None, :] - R
    r2 = np.einsum("ij,ij->i", x, x)
    t, al = d["basis_type"], d["basis_exp"]
    g = np.exp(-al * r2)
    out = np.where(t == I.S, g, 0.0)
    for ax, tt in enumerate((I.PX, I.PY, I.PZ)):
        out = np.where(t == tt, x[:, ax] * g, out)
    return np.where(t == I.STO1S, np.exp(-al * np.sqrt(r2)), out)


def det_ratio(d, pos, i, r):
    """D(x with electron i at r) / D(x) from two numpy determinants."""
    nup = int(d["n_up"])
    off, n = (0, nup) if i < nup else (nup, int(d["n_dn"]))
    C = d["mo_coeff"][:, :n]
    A = np.array([basis_np(d, pos[off + c]) @ C for c in range(n)])
    B = A.copy()
    B[i - off] = basis_np(d, r) @ C
    s0, l0 = np.linalg.slogdet(A)
    s1, l1 = np.linalg.slogdet(B)
    return s0 * s1 * np.exp(l1 - l0)


def nonlocal_reference(d, pos, rot, a):
    """(X[6N], V_nl, node flags) with X_q = -2 a^2 V_q D(x')/D(x)."""
    N = pos.shape[0]
    R = d["atom_pos"]
    rc = d["ecp_rcut"]
    terms = list(zip(d["ecp_atom"], d["ecp_l"], d["ecp_pow"], d["ecp_coef"], d["ecp_exp"]))
    U = np.eye(3) if rot is None else np.asarray(rot)
    X = np.zeros(6 * N)
    vnl, node = 0.0, np.zeros(N, bool)
    for i in range(N):
        dist = np.linalg.norm(pos[i][None, :] - R, axis=1)
        inside = np.where((rc > 0) & (dist < rc))[0]
        assert len(inside) <= 1
        if not len(inside):
            continue
        Ia = inside[0]
        r = dist[Ia]
        v = [sum(c * r ** k * np.exp(-b * r * r) for (at, ll, k, c, b) in terms
                 if at == Ia and ll == l) for l in range(3)]
        for q in range(6):
            u = U[:, q // 2] * (1.0 if q % 2 == 0 else -1.0)
            xq = R[Ia] + r * u
            cth = float(np.dot(pos[i] - R[Ia], u) / r)
            V = (v[0] + 3 * v[1] * cth + 5 * v[2] * 0.5 * (3 * cth * cth - 1)) / 6.0
            D = det_ratio(d, pos, i, xq)
            X[6 * i + q] = -2.0 * a * a * V * D
            vnl += V * D
            node[i] |= D < 0
    return X, vnl, node


def molecule_cases():
    rng = np.random.default_rng(11)
    out = []
    for terms in (I.ECP_TERMS, I.ECP_TERMS + ((2, 0, 4.0, 3.0), (2, 1, -2.0, 2.0))):
        d0 = I.c1_system(n_walkers=24)
        d = I.with_ecp(d0, np.where(d0["atom_core"] == I.SOFTCORE)[0], terms=terms)
        R = d["atom_pos"]
        for w in range(8):
            pos = d["init_pos"][w].copy()
            # put a few electrons inside the spheres at random directions
            for k, Ia in enumerate(np.where(d["ecp_rcut"] > 0)[0]):
                e = (3 * w + k) % pos.shape[0]
                u = rng.standard_normal(3)
                pos[e] = R[Ia] + rng.uniform(0.2, 1.2) * u / np.linalg.norm(u)
            rot = None if w % 2 == 0 else random_rotation(rng)
            out.append((d0, d, pos, rot))
    return out


def molecule_checks():
    bad = []
    for d0, d, pos, rot in molecule_cases():
        S0, S = O.System(d0), O.System(d)
        N = S.N
        for mode in (0, 2):
            p0, p = S0.params(nu_opt_mode=mode), S.params(nu_opt_mode=mode)
            e0 = O.evaluate(S0, p0, pos, rot=rot)
            e = O.evaluate(S, p, pos, rot=rot)
            X, vnl, nl_node = nonlocal_reference(d, pos, rot, p.a)
            scale = np.max(np.abs(X)) + 1e-300
            if np.max(np.abs(e["R"][6 * N:] - X)) > 1e-9 * scale:
                bad.append("non-local entries differ by %.3e" % np.max(np.abs(e["R"][6 * N:] - X)))
            if np.any(e["R"][:6 * N] != e0["R"]):
                bad.append("lattice ratios changed by the pseudopotential")
            if abs(e["vnl"] - vnl) > TOL * max(1.0, abs(vnl)):
                bad.append("V_nl %.10f want %.10f" % (e["vnl"], vnl))
            inv = 1.0 / (2.0 * p.a * p.a)
            wb = X[X > 0].sum() * inv
            wW = -X[X < 0].sum() * inv
            kin_node = (e0["R"].reshape(N, 6) < 0).any(axis=1)
            want_node = kin_node | nl_node
            if mode == 0 and np.any(e["node"].astype(bool) != want_node):
                bad.append("node indicators differ")
            if mode == 2:
                if abs((e["bbar"] - e0["bbar"]) - wb) > TOL * e0["bbar"]:
                    bad.append("bbar gain %.6e want %.6e" % (e["bbar"] - e0["bbar"], wb))
                if abs((e["W"] - e0["W"]) - wW) > TOL * abs(e0["W"]):
                    bad.append("W gain %.6e want %.6e" % (e["W"] - e0["W"], wW))
                if abs((e["eL"] - e0["eL"]) - vnl) > TOL * max(1.0, abs(e0["eL"])):
                    bad.append("e_L gain %.6e want %.6e" % (e["eL"] - e0["eL"], vnl))
    return bad


def test_molecule_independent():
    cases = molecule_cases()
    # the cases hold elements of both signs and electrons in both spheres
    d = cases[0][1]
    X = np.concatenate([nonlocal_reference(c[1], c[2], c[3], d["a"])[0] for c in cases])
    assert (X > 0).sum() > 20 and (X < 0).sum() > 20
    bad = molecule_checks()
    assert bad == [], bad[:5]


# --------------------------------------------------------------------------
# 3. a non-local move lands on the sphere
# --------------------------------------------------------------------------
def move_checks():
    bad = []
    for rotate in (False, True):
        d0 = I.c1_system(n_walkers=4)
        d = I.with_ecp(d0, np.where(d0["atom_core"] == I.SOFTCORE)[0])
        S = O.System(d)
        prm = S.params(nproj=1, rotate=rotate)
        Ia = int(np.where(d["ecp_rcut"] > 0)[0][0])
        for q in range(6):
            pos = d["init_pos"][:1].copy()
            i = 3
            pos[0, i] = d["atom_pos"][Ia] + np.array([0.31, -0.52, 0.44])
            before = pos[0].copy()
            lw = np.zeros(1)
            follow = np.array([[6 * S.N + 6 * i + q]], np.int32)
            O.population_phase(S, prm, "lb", 0, 0.0, pos, lw, follow=follow, nthreads=1)
            U = O.rotation(prm.seed, prm.sysid, 0, 0) if rotate else np.eye(3)
            dv = before[i] - d["atom_pos"][Ia]
            r = np.sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2])
            u = U[:, q // 2]
            want = d["atom_pos"][Ia] + (-(r * u) if q % 2 else r * u)
            if not np.array_equal(pos[0, i], want):
                bad.append("move %d rotate=%s: %s want %s" % (q, rotate, pos[0, i], want))
            others = np.delete(np.arange(S.N), i)
            if not np.array_equal(pos[0, others], before[others]):
                bad.append("a non-local move moved another electron")
    return bad


def test_nonlocal_move():
    bad = move_checks()
    assert bad == [], bad


# --------------------------------------------------------------------------
# 4. the pins reject altered arithmetic
# --------------------------------------------------------------------------
MUTATIONS = [
    ("no 2l+1 weights", "(v[0] + 3.0 * v[1] * P1 + 5.0 * v[2] * P2) / 6.0",
     "(v[0] + v[1] * P1 + v[2] * P2) / 6.0"),
    ("quadrature weight 1/4", "(v[0] + 3.0 * v[1] * P1 + 5.0 * v[2] * P2) / 6.0",
     "(v[0] + 3.0 * v[1] * P1 + 5.0 * v[2] * P2) / 4.0"),
    ("point direction sign dropped in cos theta", "double cth = (q % 2 ? -ud : ud) / r;",
     "double cth = ud / r;"),
    ("P_2 = 3c^2 - 1", "P2 = 0.5 * (3.0 * cth * cth - 1.0)", "P2 = (3.0 * cth * cth - 1.0)"),
    ("element sign flipped", "Rl[P + 6 * i + q] = -2.0 * a * a * V * rd;",
     "Rl[P + 6 * i + q] = 2.0 * a * a * V * rd;"),
    ("Jastrow factor in the non-local ratio (no DLA)", "Rl[P + 6 * i + q] = -2.0 * a * a * V * rd;",
     "Rl[P + 6 * i + q] = -2.0 * a * a * V * rd * exp(jastrow_of(s, pos, i, xq) - J0nl);"),
    ("non-local node test ignored", "        if (nlneg[i]) nd = 1;\n", "\n"),
    ("continuum e_L without the non-local energy", "elc += vee + vii + vnl;", "elc += vee + vii;"),
    ("quadrature radius a", "        double t = r * u;", "        double t = a_unused * u;"),
    ("power ignored", "double rp = s->ecp_pow[t] == 0 ? 1.0 : (s->ecp_pow[t] == 1 ? r : r * r);",
     "double rp = 1.0;"),
    ("move to the wrong point", "nl_point(s, I, rr, rot, (p - 6 * N) % 6, r);",
     "nl_point(s, I, rr, rot, ((p - 6 * N) % 6) ^ 1, r);"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_reject_altered_oracle(tmp_path, name, old, new):
    src = open(O.SRC).read()
    assert src.count(old) >= 1, "mutation target not found: " + old
    src = src.replace(old, new)
    if "J0nl" in new:
        # the Jastrow value at the electron's own position, for the planted ratio
        src = src.replace("        double r = atom_distance(s, I, pos + 3 * i, dv);\n",
                          "        double r = atom_distance(s, I, pos + 3 * i, dv);\n"
                          "        double J0nl = jastrow_of(s, pos, i, pos + 3 * i);\n", 1)
    if "a_unused" in new:
        src = src.replace("static void nl_point(const orc_system *s, int I, double r, const double *rot, int q,\n"
                          "                     double out[3])\n{",
                          "static void nl_point(const orc_system *s, int I, double r, const double *rot, int q,\n"
                          "                     double out[3])\n{\n    const double a_unused = 0.2;", 1)
    path = O.build_variant(src, str(tmp_path / "liboracle_variant.so"))
    with O.use_library(path):
        failures = closed_form_checks() + molecule_checks() + move_checks()
    assert failures, "the pins did not notice: " + name
