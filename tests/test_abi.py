"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates its inputs (no GPU needed: only pure host
functions are called)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2508_12033_amd import inputs as I
from paper_2508_12033_amd import lrdmc as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lrdmc.h")).read()
    return sorted(set(re.findall(r"\b(lrdmc_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    L = B.load()
    names = _declared()
    assert set(names) == set(B.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_workspace_bytes_and_validation():
    L = B.load()
    d = I.c1_system(n_walkers=4096)
    keep = []
    s = B._sys_struct(d, keep)
    prm = B.params_for(d)
    n = L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(prm))
    # walker state dominates: > positions + orbital rows of 4096 walkers
    assert n > 4096 * (16 * 3 * 8 + 96 * 8 * 8)
    assert n % 256 == 0
    bad = B.params_for(d, a=-1.0)
    assert L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(bad)) == 0
    assert b"lattice space" in L.lrdmc_last_error()
    h = ct.c_void_p()
    rc = L.lrdmc_init_system(ct.byref(s), 1, ct.byref(prm), None, None, 0, None, ct.byref(h))
    assert rc == -1 and not h.value
    bad = B.params_for(d, refresh_every=0)
    assert L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(bad)) == 0
    # empty phase and empty population are rejected before any device work
    bad = B.params_for(d, "lb", n_proj=0)
    assert L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(bad)) == 0
    assert b"n_proj" in L.lrdmc_last_error()
    d0 = dict(d)
    d0["n_walkers_run"] = 0
    s0 = B._sys_struct(d0, keep)
    assert s0.n_walkers == 0
    assert L.lrdmc_workspace_bytes(ct.byref(s0), 1, ct.byref(prm)) == 0
    assert b"n_walkers" in L.lrdmc_last_error()


def test_layout_rejects_oversized_system():
    """FP64: the 128-electron system fits the large-system layout (coefficient
    block and Slater rows in global memory); 256 electrons (128 per spin:
    256 KB of inverses alone) fit neither FP64 layout nor the mixed one."""
    L = B.load()
    d = I.c3_system(n_walkers=2)
    keep = []
    s = B._sys_struct(d, keep)
    assert L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(B.params_for(d))) > 0
    big = I.molecule_system(64, 0, 0, 4, 2, 2, 0.15, 25.0, I.BASE_SEED + 50)
    s = B._sys_struct(big, keep)
    for prec in ("fp64", "fp32"):
        assert L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(B.params_for(big, precision=prec))) == 0
        assert b"too large" in L.lrdmc_last_error()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_layout_accepts_large_system(prec):
    """The 128-electron, 640-function system fits the mixed-precision layout:
    per walker 6N x n_s + 4N x n_s orbital floats, the Slater rows and both
    inverses in HBM (about 393 KB), double-buffered for the reconfiguration."""
    L = B.load()
    d = I.c3_system(n_walkers=2)
    keep = []
    s = B._sys_struct(d, keep)
    prm = B.params_for(d, precision=prec)
    nb = L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(prm))
    per_walker = 4 * (2 * 64 * 6 * 64 + 2 * 64 * 4 * 64 + 128 * 64 + 2 * 64 * 64)
    assert nb >= 2 * 2 * per_walker
    assert nb < 2 * 2 * per_walker + (4 << 20)
    bad = B.params_for(d, precision=7)
    assert L.lrdmc_workspace_bytes(ct.byref(s), 1, ct.byref(bad)) == 0
    assert b"precision" in L.lrdmc_last_error()


def test_pseudopotential_validation():
    """Non-local pseudopotential arrays: accepted on the FP64 layout (12N
    proposals: the spilled orbital rows and the ratio arrays double), rejected
    with overlapping cutoff spheres, a bad channel or power, a term on an atom
    without a cutoff radius, or a mixed precision (not supported)."""
    L = B.load()
    d0 = I.c1_system(n_walkers=64)
    d = I.with_ecp(d0, np.where(d0["atom_core"] == I.SOFTCORE)[0])
    keep = []
    prm = B.params_for(d)
    n0 = L.lrdmc_workspace_bytes(ct.byref(B._sys_struct(d0, keep)), 1, ct.byref(prm))
    n1 = L.lrdmc_workspace_bytes(ct.byref(B._sys_struct(d, keep)), 1, ct.byref(prm))
    assert n0 > 0 and n1 > n0 + 64 * 96 * 8 * 8
    for key, val, msg in (("ecp_l", 3, b"ecp_l"), ("ecp_pow", -1, b"ecp_pow")):
        bad = dict(d)
        bad[key] = np.array(d[key]).copy()
        bad[key][0] = val
        assert L.lrdmc_workspace_bytes(ct.byref(B._sys_struct(bad, keep)), 1, ct.byref(prm)) == 0
        assert msg in L.lrdmc_last_error()
    bad = dict(d)
    bad["ecp_rcut"] = np.array(d["ecp_rcut"]).copy()
    bad["ecp_rcut"][bad["ecp_rcut"] > 0] = 3.6       # the two cores are 7.0 bohr apart
    assert L.lrdmc_workspace_bytes(ct.byref(B._sys_struct(bad, keep)), 1, ct.byref(prm)) == 0
    assert b"overlap" in L.lrdmc_last_error()
    bad = dict(d)
    bad["ecp_atom"] = np.array(d["ecp_atom"]).copy()
    bad["ecp_atom"][0] = 2                           # a proton: no cutoff radius
    assert L.lrdmc_workspace_bytes(ct.byref(B._sys_struct(bad, keep)), 1, ct.byref(prm)) == 0
    assert b"cutoff" in L.lrdmc_last_error()
    mixed = B.params_for(d, precision="fp32")
    assert L.lrdmc_workspace_bytes(ct.byref(B._sys_struct(d, keep)), 1, ct.byref(mixed)) == 0
    assert b"not supported" in L.lrdmc_last_error()
