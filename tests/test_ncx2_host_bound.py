"""The exact chi-squared inverse's lambda bound, through its host build.

The library's sweeps are __host__ __device__ code; a tiny host program built
with hipcc calls the same inverse on the CPU: lambda in range gives the root,
lambda above the documented bound (1e8), negative lambda and NaN give NaN."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_09715_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include "ncx2_device.hpp"
int main() {
  const double lams[] = {10.0, 1.0e4, 1.0e8, 1.0000001e8, 1.0e12, -1.0, __builtin_nan("")};
  for (double lam : lams) std::printf("%.17g %.17g\n", lam, aicdf::ncx2_icdf(0.3, 0.9, lam));
  return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_lambda_bound_host_build(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "probe"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", f"-I{CSRC}",
                        f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    rows = [tuple(float(v) for v in line.split()) for line in out.stdout.split("\n") if line.strip()]
    got = {lam: x for lam, x in rows[:3]}
    for lam in (10.0, 1.0e4):
        ref = stats.ncx2.ppf(0.3, 0.9, lam)
        assert abs(got[lam] - ref) <= 1e-9 * ref
    # at the bound: finite and near the mean (the distribution is close to
    # normal with standard deviation 2 sqrt(lambda))
    x = got[1.0e8]
    assert np.isfinite(x) and abs(x - (1.0e8 + 0.9 + 2.0 * np.sqrt(1.0e8 + 0.9) * stats.norm.ppf(0.3))) < 10.0
    for lam, x in rows[3:]:
        assert np.isnan(x), (lam, x)
