"""Statistical pins of the oracle's full LRDMC dynamics.

1. One electron on one lattice: both schemes must reproduce the lowest
   eigenvalue of the finite-a fixed-node lattice Hamiltonian, obtained here by
   sparse exact diagonalisation (stationarity results of App. A and App. B).
   The Hamiltonian is assembled in this file from its definition in App. D
   (discrete Laplacian hops of -1/(2a^2), sign-violating hops moved to the
   spin-flip diagonal, regularized potential nu_opt), using only numpy values
   of the trial function -- the continuum Laplacian comes from a fourth-order
   finite-difference stencil, not from the oracle's analytic derivatives.
2. Conventional and load-balanced energies agree within error bars for a
   two-electron molecule (Sec. II.C, Sec. III).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle as O
from paper_2508_12033_amd import inputs as I


def _psi_numpy(d, pts):
    """Trial function of a one-electron system at points [n,3] (s and p_z
    Gaussians only), straight from its definition."""
    out = np.zeros(len(pts))
    for mu in range(d["n_basis"]):
        R = d["atom_pos"][d["basis_atom"][mu]]
        x = pts - R
        g = np.exp(-d["basis_exp"][mu] * np.sum(x * x, axis=1))
        t = d["basis_type"][mu]
        if t == I.S:
            out += d["mo_coeff"][mu, 0] * g
        elif t == I.PZ:
            out += d["mo_coeff"][mu, 0] * x[:, 2] * g
        else:
            raise NotImplementedError
    return out


def lattice_lambda_min(d, L, nu_opt_mode=0):
    a = d["a"]
    o = d["lattice_origin"]
    k = np.arange(int(np.floor((-L - o[0]) / a)), int(np.ceil((L - o[0]) / a)) + 1)
    n = len(k)
    grid = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1).reshape(-1, 3)
    pts = o + a * grid
    psi = _psi_numpy(d, pts)
    h = 1e-3
    lap = np.zeros(len(pts))
    for c in range(3):
        e = np.zeros(3); e[c] = h
        lap += (-_psi_numpy(d, pts - 2 * e) + 16 * _psi_numpy(d, pts - e) - 30 * psi
                + 16 * _psi_numpy(d, pts + e) - _psi_numpy(d, pts + 2 * e)) / (12 * h * h)
    lap /= psi
    r = np.linalg.norm(pts - d["atom_pos"][0], axis=1)
    nu = -1.0 / r
    nua = -1.0 / np.maximum(r, a)
    idx = np.arange(len(pts)).reshape(n, n, n)
    rows, cols, vals = [], [], []
    lapA = np.zeros(len(pts)); vsf = np.zeros(len(pts)); node = np.zeros(len(pts), bool)
    for c in range(3):
        for s in (1, -1):
            e = np.zeros(3); e[c] = s * a
            ratio = _psi_numpy(d, pts + e) / psi
            lapA += (ratio - 1.0) / a ** 2
            neg = ratio < 0
            vsf += np.where(neg, -ratio, 0.0) / (2 * a * a)
            node |= neg
            nb = np.roll(idx, -s, axis=c).reshape(-1)
            inside = np.ones((n, n, n), bool)
            if s == 1:
                sl = [slice(None)] * 3; sl[c] = -1; inside[tuple(sl)] = False
            else:
                sl = [slice(None)] * 3; sl[c] = 0; inside[tuple(sl)] = False
            inside = inside.reshape(-1) & ~neg
            rows.append(np.arange(len(pts))[inside]); cols.append(nb[inside])
            vals.append(np.full(inside.sum(), -1.0 / (2 * a * a)))
    nuzv = nu + 0.5 * (lapA - lap)
    numax = np.maximum(nuzv, nua)
    nuop = np.where(node, numax, nuzv) if nu_opt_mode != 2 else numax
    diag = 3.0 / a ** 2 + nuop + vsf
    rows.append(np.arange(len(pts))); cols.append(np.arange(len(pts))); vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(pts), len(pts)))
    # fixed-node: restrict to the pocket of the walkers (psi > 0)
    keep = np.where(psi > 0)[0]
    H = H[keep][:, keep]
    w = spl.eigsh(H, k=1, which="SA", tol=1e-10, return_eigenvectors=False)
    return float(w[0])


def _run(d, scheme, n_branch):
    return O.run(d, scheme, n_branch, nthreads=8)


@pytest.mark.slow
def test_one_electron_nodeless_lambda_min():
    d = I.one_electron_system("gauss", n_walkers=1000)
    lam = lattice_lambda_min(d, 9.0)
    for scheme in ("lb", "conv"):
        r = _run(d, scheme, 300)
        z = (r["E"] - lam) / r["sigma"]
        assert abs(z) < 3.5, (scheme, r["E"], r["sigma"], lam)
        assert r["sigma"] < 3e-3


@pytest.mark.slow
def test_one_electron_nodal_lambda_min():
    """p_z trial: the walkers stay in the z > 0 pocket; the fixed-node lattice
    energy includes V_sf and nu_opt (App. D)."""
    d = I.one_electron_system("nodal", n_walkers=2000, a=0.5)
    lam = lattice_lambda_min(d, 18.0)
    for scheme in ("lb", "conv"):
        r = _run(d, scheme, 600)
        assert np.all(r["pos"][:, 0, 2] > 0)
        z = (r["E"] - lam) / r["sigma"]
        assert abs(z) < 3.5, (scheme, r["E"], r["sigma"], lam)


@pytest.mark.slow
def test_conventional_equals_load_balanced_h2():
    """Sec. II.C / Sec. III: both schemes sample the same fixed-node state at
    fixed a when the mean number of moves per branching is matched."""
    d = I.h2_system(n_walkers=256)
    d["init_pos"] = d["init_pos"][:256]
    rc = O.run(d, "conv", 100, nthreads=8, tau=0.5)
    nbar = float(np.mean(rc["iters"]))
    rl = O.run(d, "lb", 100, nthreads=8, nproj=int(round(nbar)))
    z = (rc["E"] - rl["E"]) / np.hypot(rc["sigma"], rl["sigma"])
    assert abs(z) < 3.5, (rc["E"], rc["sigma"], rl["E"], rl["sigma"])
