"""Seeded synthetic molecular systems for lattice-regularized DMC.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no wavefunction, Hamiltonian, Green's function or
branching).  It is the single source of inputs for both the FP64 CPU oracle
and the GPU library, so that both see bit-identical systems and starting
configurations.

The paper's own benchmark systems (water, methane, the water-methane dimer and
benzene with ccECP pseudopotentials, cc-pVTZ/aug-cc-pVTZ basis sets and
SR-optimized Jastrow factors, Sec. III and Sec. IV) need parameter sets that are
not available here.  These synthetic stand-ins match the regime of the paper's
weak-scaling benchmark (Sec. IV): tens of electrons, ~300 projection steps per
branching, thousands of walkers.

System layout (all arrays numpy, C-contiguous):
  atom_pos     [M,3] f64   nuclear positions (bohr)
  atom_charge  [M]   f64   charge seen by electrons (Z for bare nuclei,
                           the valence charge Z_v for local-potential cores)
  atom_core    [M]   i32   0 = bare Coulomb nucleus, 1 = smooth local core
                           -Z_v/sqrt(r^2 + rc^2)
  core_rc      [M]   f64   core radius of the smooth core (bohr)
  atom_species [M]   i32   species index for electron-nucleus Jastrow terms
  basis_atom   [Nb]  i32   centre of each basis function
  basis_type   [Nb]  i32   0 = s, 1/2/3 = p_x/p_y/p_z, 4 = Slater 1s
  basis_exp    [Nb]  f64   Gaussian exponent alpha (or Slater zeta)
  mo_coeff     [Nb,Norb] f64  orbital coefficients, row-major
  n_up, n_dn   electrons per spin; electrons 0..n_up-1 are spin up
  jastrow      [2+n_species,3] f64  Pade parameters (A, B, b) of
                           u(r) = (A r + B r^2)/(1 + b r); row 0 = parallel
                           e-e pairs, row 1 = antiparallel e-e pairs,
                           row 2+s = electron-nucleus pairs of species s
  init_pos     [Nw,N,3] f64  initial electron positions of every walker
  a, tau, n_proj, n_walkers, seed, system_id
Optional non-local pseudopotential (semi-local channels, App. D non-local
elements; synthetic parameters, since ccECP tables are not available):
  ecp_atom, ecp_l, ecp_pow [T] i32, ecp_coef, ecp_exp [T] f64: term t adds
                           coef r^pow exp(-exp r^2) to channel l of its atom
  ecp_rcut     [M]   f64   radius inside which an atom's channels act (0: none;
                           the spheres of different atoms do not overlap)
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 12033

S, PX, PY, PZ, STO1S = 0, 1, 2, 3, 4
BARE, SOFTCORE = 0, 1

# Regularized electron-nucleus potential (App. D).  NU_OPT_OWN: nu_max only
# for electrons whose own 6 lattice moves cross the node (the paper's
# nu_opt); NU_OPT_ANY: when any move crosses; NU_MAX_ALWAYS: nu_max for every
# electron.  The synthetic molecules use Gaussian trial functions without the
# electron-nucleus cusp around bare protons, where nu_zv keeps the -Z/r
# divergence; they therefore use the bound of the single-electron
# regularization everywhere.
NU_OPT_OWN, NU_OPT_ANY, NU_MAX_ALWAYS = 0, 1, 2


def _place_atoms(rng, n_atoms, box, min_sep):
    """Uniform positions in a cube of side `box`, rejection on min separation."""
    pos = np.zeros((n_atoms, 3))
    k = 0
    tries = 0
    while k < n_atoms:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("atom placement failed")
        p = rng.uniform(0.0, box, size=3)
        if k and np.min(np.linalg.norm(pos[:k] - p, axis=1)) < min_sep:
            continue
        pos[k] = p
        k += 1
    return pos


def _gaussian_basis(rng, n_atoms, n_s, n_p, lo=0.1, hi=5.0):
    """n_s s-shells and n_p p-shells per atom, exponents log-uniform in [lo, hi]."""
    batom, btype, bexp = [], [], []
    for a in range(n_atoms):
        es = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_s))
        ep = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_p))
        for e in es:
            batom.append(a); btype.append(S); bexp.append(e)
        for e in ep:
            for t in (PX, PY, PZ):
                batom.append(a); btype.append(t); bexp.append(e)
    return (np.array(batom, np.int32), np.array(btype, np.int32),
            np.array(bexp, np.float64))


def _initial_positions(rng, atom_pos, valence, n_up, n_dn, n_walkers):
    """Electrons assigned round-robin over atoms weighted by valence; up and
    down alternate along that list; r = R_I + N(0,1)^3."""
    slots = np.concatenate([np.full(int(v), i) for i, v in enumerate(valence)])
    n = n_up + n_dn
    if len(slots) < n:
        slots = np.resize(slots, n)
    up, dn = [], []
    for e in range(n):
        if (e % 2 == 0 and len(up) < n_up) or len(dn) >= n_dn:
            up.append(slots[e])
        else:
            dn.append(slots[e])
    centres = atom_pos[np.array(up + dn, dtype=np.int64)]
    return centres[None, :, :] + rng.standard_normal((n_walkers, n, 3))


def _jastrow(n_species, en=None):
    """Default Pade parameters: e-e cusps 1/4 (parallel) and 1/2 (anti), b=1."""
    jas = np.zeros((2 + n_species, 3))
    jas[0] = (0.25, 0.0, 1.0)
    jas[1] = (0.5, 0.0, 1.0)
    for s in range(n_species):
        jas[2 + s] = en if en is not None else (0.0, 0.0, 1.0)
    return jas


def _finish(d):
    for k in ("atom_pos", "atom_charge", "core_rc", "basis_exp", "mo_coeff",
              "jastrow", "init_pos"):
        d[k] = np.ascontiguousarray(d[k], dtype=np.float64)
    for k in ("atom_core", "atom_species", "basis_atom", "basis_type"):
        d[k] = np.ascontiguousarray(d[k], dtype=np.int32)
    d["n_atoms"] = int(d["atom_pos"].shape[0])
    d["n_basis"] = int(d["basis_exp"].shape[0])
    d["n_orb"] = int(d["mo_coeff"].shape[1])
    d["n_elec"] = int(d["n_up"] + d["n_dn"])
    d["n_species"] = int(d["jastrow"].shape[0] - 2)
    return d


def h2_system(n_walkers=256, a=0.2, seed=BASE_SEED + 0, system_id=0):
    """H2-like: protons at (0,0,+-0.7), 1 up + 1 down electron, 4 s Gaussians
    per atom (exponents log-uniform in [0.1,5]), MO coefficients N(0,1)."""
    rng = np.random.default_rng(seed)
    atom_pos = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
    batom, btype, bexp = _gaussian_basis(rng, 2, 4, 0)
    C = rng.standard_normal((len(bexp), 1))
    init = _initial_positions(rng, atom_pos, [1, 1], 1, 1, n_walkers)
    n = 2
    return _finish(dict(
        name="h2", atom_pos=atom_pos, atom_charge=np.array([1.0, 1.0]),
        atom_core=np.array([BARE, BARE]), core_rc=np.array([0.0, 0.0]),
        atom_species=np.array([0, 0]), basis_atom=batom, basis_type=btype,
        basis_exp=bexp, mo_coeff=C, n_up=1, n_dn=1, jastrow=_jastrow(1),
        init_pos=init, a=a, tau=300.0 * a * a / (3.0 * n), n_proj=300,
        n_walkers=n_walkers, seed=seed, system_id=system_id,
        nu_opt_mode=NU_MAX_ALWAYS))


def molecule_system(n_c, n_o, n_h, n_s, n_p, n_walkers, a, box, seed,
                    system_id=0, name="mol", en_jastrow=None, rc=0.5):
    """Atoms: n_c C-like cores (Z_v=4), n_o O-like cores (Z_v=6), both smooth
    local cores -Z_v/sqrt(r^2 + rc^2), plus n_h bare protons, placed uniformly in a
    cube with 1.8 bohr minimum separation.  Neutral, equal up/down counts."""
    rng = np.random.default_rng(seed)
    m = n_c + n_o + n_h
    atom_pos = _place_atoms(rng, m, box, 1.8)
    charge = np.array([4.0] * n_c + [6.0] * n_o + [1.0] * n_h)
    core = np.array([SOFTCORE] * (n_c + n_o) + [BARE] * n_h)
    rcs = np.array([rc] * (n_c + n_o) + [0.0] * n_h)
    species = np.array([1] * n_c + [2] * n_o + [0] * n_h)   # 0=H, 1=C, 2=O
    batom, btype, bexp = _gaussian_basis(rng, m, n_s, n_p)
    n = int(charge.sum())
    n_up = n_dn = n // 2
    C = rng.standard_normal((len(bexp), max(n_up, n_dn)))
    init = _initial_positions(rng, atom_pos, charge, n_up, n_dn, n_walkers)
    return _finish(dict(
        name=name, atom_pos=atom_pos, atom_charge=charge, atom_core=core,
        core_rc=rcs, atom_species=species, basis_atom=batom, basis_type=btype,
        basis_exp=bexp, mo_coeff=C, n_up=n_up, n_dn=n_dn,
        jastrow=_jastrow(3, en_jastrow), init_pos=init, a=a,
        tau=300.0 * a * a / (3.0 * n), n_proj=300, n_walkers=n_walkers,
        seed=seed, system_id=system_id, nu_opt_mode=NU_MAX_ALWAYS))


def c1_system(n_walkers=4096, seed=BASE_SEED + 1):
    """8 atoms (one C-like core Z_v=4, one O-like core Z_v=6, six protons) in a
    10 bohr box; 16 electrons (8 up, 8 down); 4 s + 2 p shells = 10 Gaussians
    per atom (80 basis functions, 8 orbitals); a = 0.2 bohr."""
    return molecule_system(1, 1, 6, 4, 2, n_walkers, 0.2, 10.0, seed, name="c1")


def c2_systems(n_walkers=(8192, 4096, 2048), seed=BASE_SEED + 2):
    """Three uneven systems (16e/8 atoms, 32e/16 atoms, 64e/32 atoms), each
    10 Gaussians per atom, box 10*(M/8)^(1/3) bohr, a = 0.2 bohr."""
    out = []
    for k, (mult, nw) in enumerate(zip((1, 2, 4), n_walkers)):
        m = 8 * mult
        out.append(molecule_system(mult, mult, 6 * mult, 4, 2, nw, 0.2,
                                   10.0 * (m / 8.0) ** (1.0 / 3.0),
                                   seed * 16 + k, system_id=k,
                                   name="c2_%de" % (16 * mult)))
    return out


def c3_system(n_walkers=2048, seed=BASE_SEED + 3):
    """32 C-like cores (Z_v=4 -> 128 electrons, 64 up + 64 down) in a 20 bohr
    box; 8 s + 4 p shells = 20 Gaussians per atom (640 basis functions,
    64 orbitals); a = 0.15 bohr."""
    return molecule_system(32, 0, 0, 8, 4, n_walkers, 0.15, 20.0, seed,
                           name="c3")


def c4_system(n_walkers=4096, seed=BASE_SEED + 1):
    """The 16-electron system of c1_system with electron-nucleus Pade terms
    switched on (A=-0.25, B=0, b=1 for every species): 15 Jastrow parameters."""
    d = molecule_system(1, 1, 6, 4, 2, n_walkers, 0.2, 10.0, seed, name="c4",
                        en_jastrow=(-0.25, 0.0, 1.0))
    return d


def hydrogenic_system(Z=1.0, zeta=1.0, n_walkers=64, a=0.2, seed=BASE_SEED + 7):
    """One electron around a bare nucleus of charge Z with a single Slater 1s
    function exp(-zeta r): an exact eigenstate when zeta = Z (e_L = -Z^2/2)."""
    rng = np.random.default_rng(seed)
    atom_pos = np.zeros((1, 3))
    init = 0.7 * rng.standard_normal((n_walkers, 1, 3)) + 0.05
    return _finish(dict(
        name="hydrogenic", atom_pos=atom_pos, atom_charge=np.array([Z]),
        atom_core=np.array([BARE]), core_rc=np.array([0.0]),
        atom_species=np.array([0]), basis_atom=np.array([0]),
        basis_type=np.array([STO1S]), basis_exp=np.array([zeta]),
        mo_coeff=np.ones((1, 1)), n_up=1, n_dn=0,
        jastrow=np.zeros((3, 3)), init_pos=init, a=a,
        tau=100.0 * a * a / 3.0, n_proj=100, n_walkers=n_walkers, seed=seed,
        system_id=0))


def one_electron_system(kind="gauss", n_walkers=256, a=0.4, seed=BASE_SEED + 8,
                        origin=(0.13, 0.07, 0.21)):
    """One electron around a bare proton.  kind='gauss': nodeless trial from
    two s Gaussians; kind='nodal': p_z trial (node on the plane z=0) from one
    p_z Gaussian, which exercises the fixed-node terms; kind='soft': the
    nodeless trial around a softened core -2/sqrt(r^2 + 0.25) (a smooth
    potential, so the lattice energy approaches the continuum one as a^2).
    Every walker starts on the same lattice origin + a*Z^3, so that all walkers
    sample one lattice Hamiltonian (used by the brute-force lowest-eigenvalue
    check)."""
    rng = np.random.default_rng(seed)
    atom_pos = np.zeros((1, 3))
    o = np.asarray(origin, np.float64)
    charge, core, rc = np.array([1.0]), np.array([BARE]), np.array([0.0])
    if kind == "soft":
        charge, core, rc = np.array([2.0]), np.array([SOFTCORE]), np.array([0.5])
    if kind in ("gauss", "soft"):
        batom = np.array([0, 0]); btype = np.array([S, S])
        bexp = np.array([0.2, 1.2]); C = np.array([[0.6], [0.5]])
        g = 1.0 * rng.standard_normal((n_walkers, 1, 3))
    else:
        batom = np.array([0]); btype = np.array([PZ])
        bexp = np.array([0.15]); C = np.array([[1.0]])
        g = 2.0 * rng.standard_normal((n_walkers, 1, 3))
        g[:, 0, 2] = np.abs(g[:, 0, 2]) + a      # start in the z>0 pocket
    init = o[None, None, :] + a * np.round(g / a)
    return _finish(dict(
        name="one_e_" + kind, atom_pos=atom_pos, atom_charge=charge,
        atom_core=core, core_rc=rc,
        atom_species=np.array([0]), basis_atom=batom, basis_type=btype,
        basis_exp=bexp, mo_coeff=C, n_up=1, n_dn=0,
        jastrow=np.zeros((3, 3)), init_pos=init, a=a,
        tau=20.0 * a * a / 3.0, n_proj=20, n_walkers=n_walkers, seed=seed,
        system_id=0, lattice_origin=o))


# Synthetic non-local channels (l, power, coefficient, exponent): a repulsive
# s channel with an attractive r^2 tail and an attractive p channel, so that
# both signs of the non-local elements occur; they decay below 1e-2 Ha by the
# cutoff radius 1.3 bohr.
ECP_TERMS = ((0, 0, 10.0, 5.0), (0, 2, -3.0, 4.0), (1, 0, -5.0, 4.5))


def with_ecp(d, atoms, terms=ECP_TERMS, rcut=1.3):
    """Copy of system d with the non-local channels `terms` on every atom in
    `atoms`, acting inside radius rcut (shrunk to 0.49 of the closest pair of
    those atoms, so that the spheres never overlap)."""
    d = dict(d)
    R = np.asarray(d["atom_pos"], np.float64)
    atoms = list(atoms)
    for a_ in range(len(atoms)):
        for b_ in range(a_ + 1, len(atoms)):
            rcut = min(rcut, 0.49 * float(np.linalg.norm(R[atoms[a_]] - R[atoms[b_]])))
    ea, el, ep, ec, ee = [], [], [], [], []
    for I in atoms:
        for (l, pw, c, b) in terms:
            ea.append(I); el.append(l); ep.append(pw); ec.append(c); ee.append(b)
    rc = np.zeros(R.shape[0])
    rc[atoms] = rcut
    d.update(ecp_atom=np.array(ea, np.int32), ecp_l=np.array(el, np.int32),
             ecp_pow=np.array(ep, np.int32), ecp_coef=np.array(ec, np.float64),
             ecp_exp=np.array(ee, np.float64), ecp_rcut=rc)
    d["name"] = d.get("name", "sys") + "_ecp"
    return d


def c1_ecp_system(n_walkers=4096, seed=BASE_SEED + 1):
    """The 16-electron system of c1_system with the synthetic non-local
    channels on its two smooth cores (C-like and O-like, 7.0 bohr apart),
    cutoff radius 1.3 bohr."""
    d = c1_system(n_walkers, seed)
    return with_ecp(d, np.where(d["atom_core"] == SOFTCORE)[0])


CONFIGS = {
    "h2": h2_system,
    "c1": c1_system,
    "c3": c3_system,
    "c4": c4_system,
}
