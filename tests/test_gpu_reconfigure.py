"""Reconfiguration of a caller-held population (lrdmc_reconfigure) against the
oracle's comb and walker average (Sec. II.A comb; Sec. II.C load-balanced
weights w / (W - E_0)): selections bit-exact, log of the average weight and
walker-averaged e_L to 1e-12 relative, at one walker, ragged sizes, the
benchmark's 4096, a population of 2^20, with dead walkers (lw = -inf), and
the all-dead case."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_12033_amd import lrdmc as B
from parity_util import say

pytestmark = pytest.mark.gpu


def _population(nw, seed, dead_frac=0.1):
    rng = np.random.default_rng(seed)
    lw = rng.normal(0.0, 2.0, nw)
    lw[rng.random(nw) < dead_frac] = -np.inf
    if nw > 1 and np.all(~np.isfinite(lw)):
        lw[0] = 0.0
    eL = -20.0 + rng.normal(0.0, 0.5, nw)
    W = 1000.0 + rng.normal(0.0, 3.0, nw)
    return lw, eL, W


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("scheme", ["lb", "conv"])
@pytest.mark.parametrize("nw", [1, 37, 1000, 4096, 1 << 20])
def test_reconfigure_matches_oracle(scheme, nw):
    lw, eL, W = _population(nw, nw + (scheme == "lb"), dead_frac=0.0 if nw == 1 else 0.1)
    e0, seed, sysid, j = -20.3, 12033, 5, 17
    say("case reconfigure", scheme, nw)
    sel, out = B.reconfigure(_dev(lw), _dev(eL), _dev(W), e0=e0, scheme=scheme, seed=seed,
                             sysid=sysid, j=j)
    torch.cuda.synchronize()
    sel, out = sel.cpu().numpy(), out.cpu().numpy()
    xi = O.uniform(seed, sysid, 0, j, 0, O.RNG_COMB)
    osel, lwb, cnt = O.comb(lw, xi, follow=sel)
    assert cnt["hard_mismatch"] == 0 and cnt["ambig_adopted"] == 0, cnt
    assert np.array_equal(osel, sel)
    assert np.all(np.isfinite(lw[sel]))
    assert out[4] == 0.0
    assert abs(out[0] - lwb) < 1e-12 * max(1.0, abs(lwb))
    eb = O.walker_average(scheme, lw, eL, W, e0)
    assert abs(out[1] - eb) < 1e-12 * abs(eb)
    assert out[2] == np.max(lw)
    assert out[3] == len(np.unique(sel))


def test_reconfigure_all_dead_and_nonfinite():
    nw = 64
    lw = np.full(nw, -np.inf)
    eL = np.full(nw, -1.0)
    W = np.full(nw, 10.0)
    sel, out = B.reconfigure(_dev(lw), _dev(eL), _dev(W), e0=0.0)
    torch.cuda.synchronize()
    assert out[4].item() == 1.0 and np.all(sel.cpu().numpy() == 0)
    lw[3] = np.nan
    lw[5] = 0.0
    sel, out = B.reconfigure(_dev(lw), _dev(eL), _dev(W), e0=0.0)
    torch.cuda.synchronize()
    assert out[4].item() == 2.0


def test_reconfigure_rejects_bad_arguments():
    L = B.load()
    assert L.lrdmc_reconfigure_workspace_bytes(0) == 0
    x = _dev(np.zeros(4))
    sel = torch.empty(4, dtype=torch.int32, device="cuda")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    rc = L.lrdmc_reconfigure(0, 4, x.data_ptr(), x.data_ptr(), x.data_ptr(), 0.0, 1, 0, 0,
                             sel.data_ptr(), out.data_ptr(), None, 0, None)
    assert rc == -1
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    rc = L.lrdmc_reconfigure(0, 4, x.data_ptr(), x.data_ptr(), x.data_ptr(), 0.0, 1, 0, 0,
                             sel.data_ptr(), out.data_ptr(), ws.data_ptr(), 8, None)
    assert rc == -3
