"""lrdmc_reconfigure_noalloc (the reconfiguration of a caller-held population
with its scratch in the library's fixed device array) against
lrdmc_reconfigure (scratch in a caller workspace), through the C ABI: two
calls in a row, the second with a smaller population, each compared element
by element (selections bit-exact, the eight result doubles identical), and
the population bound rejected before any device work."""
import numpy as np
import pytest
import torch

from paper_2508_12033_amd import lrdmc as B

pytestmark = pytest.mark.gpu


def _population(nw, seed):
    rng = np.random.default_rng(seed)
    lw = rng.normal(0.0, 2.0, nw)
    lw[rng.random(nw) < 0.1] = -np.inf
    lw[0] = 0.5
    eL = -20.0 + rng.normal(0.0, 0.5, nw)
    W = 1000.0 + rng.normal(0.0, 3.0, nw)
    return [torch.from_numpy(x).cuda() for x in (lw, eL, W)]


def _call_noalloc(L, scheme, lw, eL, W, e0, seed, sysid, j):
    nw = int(lw.shape[0])
    sel = torch.full((nw,), -7, dtype=torch.int32, device="cuda")
    out = torch.full((8,), -7.0, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    rc = L.lrdmc_reconfigure_noalloc(scheme, nw, lw.data_ptr(), eL.data_ptr(), W.data_ptr(),
                                     float(e0), seed, sysid, j, sel.data_ptr(), out.data_ptr(),
                                     st.cuda_stream)
    assert rc == 0, L.lrdmc_last_error()
    return sel, out


@pytest.mark.parametrize("scheme", [B.SCHEME_LB, B.SCHEME_CONV])
def test_noalloc_matches_workspace_entry_point(scheme):
    L = B.load()
    for nw, seed, j in ((300000, 1, 3), (4099, 2, 4)):     # second call smaller
        lw, eL, W = _population(nw, seed + 10 * scheme)
        sel_n, out_n = _call_noalloc(L, scheme, lw, eL, W, -20.1, 12033, 2, j)
        sel_w, out_w = B.reconfigure(lw, eL, W, e0=-20.1, scheme="lb" if scheme == 0 else "conv",
                                     seed=12033, sysid=2, j=j)
        torch.cuda.synchronize()
        sn, sw = sel_n.cpu().numpy(), sel_w.cpu().numpy()
        on, ow = out_n.cpu().numpy(), out_w.cpu().numpy()
        assert np.array_equal(sn, sw)
        assert np.array_equal(on[:5], ow[:5])
        assert on[4] == 0.0 and np.all((sn >= 0) & (sn < nw))
        assert np.all(np.isfinite(lw.cpu().numpy()[sn]))


def test_noalloc_rejects_too_many_walkers():
    L = B.load()
    nw = 1048576 + 1
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    sel = torch.zeros(16, dtype=torch.int32, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = L.lrdmc_reconfigure_noalloc(0, nw, x.data_ptr(), x.data_ptr(), x.data_ptr(), 0.0, 1, 0, 0,
                                     sel.data_ptr(), out.data_ptr(), None)
    assert rc == -1 and b"LRDMC_NOALLOC_MAX_WALKERS" in L.lrdmc_last_error()
