"""Brute-force lowest eigenvalue of the one-electron fixed-node lattice
Hamiltonian (App. D), assembled from its definition: discrete Laplacian hops
of -1/(2a^2), sign-violating hops moved to the spin-flip diagonal, the
regularized potential nu_opt with the continuum Laplacian from a fourth-order
finite-difference stencil of a numpy trial function (never the oracle's
analytic derivatives), restricted to the walkers' nodal pocket and
diagonalized by scipy's sparse eigensolver.  One nucleus at the origin, bare
(-Z/r, lattice bound -Z/max(r, a)) or softened (-Z/sqrt(r^2 + r_c^2)); s and
p_z Gaussian trial functions."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

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
    Z = float(d["atom_charge"][0])
    if int(d["atom_core"][0]) == I.BARE:
        nu = -Z / r
        nua = -Z / np.maximum(r, a)
    else:   # softened core: no lattice bound is needed (App. D, smooth potentials)
        rc = float(d["core_rc"][0])
        nu = -Z / np.sqrt(r * r + rc * rc)
        nua = nu
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
