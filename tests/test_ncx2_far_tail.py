"""The exact chi-squared inverse in the far lower tail (u from 1e-35 down to
1e-300), through the library's host build, against a 50-digit mpmath root of
the Poisson-mixture CDF (Section 5: C(x) = sum_j e^-mu mu^j / j! P(nu/2 + j,
x/2), A&S 26.4.25).  The oracle's windowed CDF is pinned for u >= 1e-30;
below, the dominant terms sit at j = 0 and the library's sweeps and final
scaling carry them, which this test checks.  Bound: the library's 5e-11
relative."""
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_09715_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# u down to 1e-300 where the root is a normal FP64 number (x ~ u^(2/nu):
# for nu = 0.889 the smallest u is 1e-130, x ~ 1e-292)
CASES = [(nu, lam, u) for nu in (0.889, 2.0, 5.0) for lam in (0.0, 3.0, 40.0)
         for u in ((1e-35, 1e-100, 1e-130) if nu < 1 else (1e-35, 1e-100, 1e-300))]
# roots below the FP64 range: 1e-300 at nu = 0.889 lies near 1e-675
UNDERFLOW = [(0.889, lam, 1e-300) for lam in (0.0, 3.0, 40.0)]

PROGRAM = r"""
#include <cstdio>
#include "ncx2_device.hpp"
int main() {
  double nu, lam, u;
  while (std::scanf("%lf %lf %lf", &nu, &lam, &u) == 3) std::printf("%.17g\n", aicdf::ncx2_icdf(u, nu, lam));
  return 0;
}
"""


def mp_cdf(x, nu, lam):
    """C(x) to ~50 digits: the Poisson mixture of regularised lower
    incomplete gamma functions, summed until the terms fall below 1e-60 of
    the sum (the terms decrease geometrically once j exceeds mu and y)."""
    a, mu, y = mp.mpf(nu) / 2, mp.mpf(lam) / 2, mp.mpf(x) / 2
    s, j = mp.mpf(0), 0
    while True:
        w = mp.exp(-mu) * mu ** j / mp.factorial(j) if mu > 0 else (mp.mpf(1) if j == 0 else mp.mpf(0))
        t = w * mp.gammainc(a + j, 0, y, regularized=True)
        s += t
        if j > mu + y + 10 and (t == 0 or t < s * mp.mpf(10) ** -60):
            return s
        if mu == 0:
            return s
        j += 1


def mp_icdf(u, nu, lam):
    """The root (an mpf) of log C(e^t) = log u in t = log x, bracketed by
    log x_lo - 1 and log x_lo + mu/a + 2, x_lo = 2 (u Gamma(a+1))^(1/a):
    C(x) <= P(a, x/2) <= (x/2)^a / Gamma(a+1) puts the root above x_lo, and
    C(x) >= e^-mu P(a, x/2), with P(a, y) close to y^a / Gamma(a+1) for the
    tiny y here, puts it below x_lo e^(mu/a) (widened until it holds)."""
    mp.mp.dps = 50
    a = mp.mpf(nu) / 2
    lu = mp.log(mp.mpf(u))
    tlo = mp.log(2) + (lu + mp.loggamma(a + 1)) / a
    f = lambda t: mp.log(mp_cdf(mp.exp(t), nu, lam)) - lu
    lo, hi = tlo - 1, tlo + (mp.mpf(lam) / 2) / a + 2
    while f(hi) < 0:
        hi += 1
    t = mp.findroot(f, (lo, hi), solver="anderson", tol=mp.mpf(10) ** -40, maxsteps=200)
    return mp.exp(t)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_far_lower_tail_against_mpmath(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "probe"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", f"-I{CSRC}",
                        f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    inp = "\n".join(f"{nu!r} {lam!r} {u!r}" for nu, lam, u in CASES + UNDERFLOW) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = [float(v) for v in out.stdout.split()]
    assert len(got) == len(CASES) + len(UNDERFLOW)
    for (nu, lam, u), x in zip(CASES, got):
        ref = mp_icdf(u, nu, lam)
        assert ref > 1e-300
        assert abs(x - ref) <= 5e-11 * ref, (nu, lam, u, x, float(ref), float(abs(x - ref) / ref))
    for x in got[len(CASES):]:
        assert 0.0 <= x < 1e-300, x


# The body and both tails at moderate and large lambda (the CIR levels' range
# and beyond, both sweep directions: upper-tail targets 1 - u < 2^-10, and
# every u > 1/2 once lambda > 4096), against the oracle's bisection in log x:
# the root iteration's third-order steps and its stopping rule, through the
# host build.  Bound: 5e-11 relative.
BODY = [(nu, lam, u) for nu in (0.889, 5.0) for lam in (0.0, 0.5, 20.0, 300.0, 5000.0)
        for u in (1e-8, 0.01, 0.3, 0.5, 0.7, 0.99, 1.0 - 1e-6)]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_body_and_upper_tail_against_oracle(tmp_path):
    from oracle import ncx2 as oracle_ncx2
    src = tmp_path / "probe.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "probe"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", f"-I{CSRC}",
                        f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    inp = "".join(f"{nu!r} {lam!r} {u!r}\n" for nu, lam, u in BODY)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split()
    got = np.array([float(v) for v in out])
    worst = 0.0
    for (nu, lam, u), x in zip(BODY, got):
        ref = float(oracle_ncx2.icdf(u, nu, lam)[0])
        rel = abs(x - ref) / ref
        worst = max(worst, rel)
        assert rel <= 5e-11, (nu, lam, u, x, ref, rel)
    assert worst > 0.0  # the two sides are computed independently
