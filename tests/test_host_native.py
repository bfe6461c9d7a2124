"""Host-side checks of device helpers compiled with hipcc and run on the CPU.

lw_block_update (blocked logarithm of the load-balanced weight factors
bbar / (W - E_0), Sec. II.C / Algorithm 2): sequences of factors that carry
the running product past the range of a double (a subnormal denominator, a
factor of 1e305, a subnormal numerator) must give the per-step sum of
logarithms, and the product kept between logarithms must stay in
[2^-600, 2^600].

Derivative formulas of the adjoint pass (lrdmc_deriv.hpp): basis gradients,
Hessians and Laplacian gradients and the Pade pair function's r- and
parameter derivatives against fourth-order central differences of values
written out from their definitions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _build_and_run(tmp_path, name):
    exe = str(tmp_path / name)
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_2508_12033_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", name + ".hip"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
def test_blocked_log_weight_update(tmp_path):
    _build_and_run(tmp_path, "lw_update_host")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
def test_adjoint_derivative_formulas(tmp_path):
    _build_and_run(tmp_path, "deriv_host")
