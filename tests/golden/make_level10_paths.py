"""Writes level10_paths.txt: the oracle's per-path replay of CIR paths at
level 10 (1024 exact transitions per path; Section 5.2), for the GPU parity
tests at the finest level of the large fused run.  Calls only oracle/ (the
exact replay bisects the series CDF at every step: about a minute per pair
of paths, too slow to repeat inside every GPU test run).

Cases (CIR kappa = 0.5, theta = 0.04, xi = 0.3, v0 = 0.04, T = 1, the
trapezoidal time average):
  exact       kind EXACT, seed 93, paths 777 and 778
  correction  kind CORRECTION, seed 94, paths 31 and 32, with the damped
              test surrogate (mlp.init_params(21), W3 x 0.05, b3 = 0,
              parameters rounded to FP32, log lambda range [-8, 10], input
              feature the 16-row cubic dyadic approximation of Phi^-1(u24))

    python tests/golden/make_level10_paths.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cir, mlp, tables  # noqa: E402
from oracle.dtypes import round_f32  # noqa: E402
from oracle.transform import dyadic_transform_f32  # noqa: E402

CIR = dict(v0=0.04, kappa=0.5, theta=0.04, xi=0.3, T=1.0, functional=1)
NU = 4 * 0.5 * 0.04 / 0.3 ** 2
LO, HI = -8.0, 10.0


def damped_params():
    p = mlp.init_params(21)
    p["W3"] = p["W3"] * 0.05
    p["b3"] = np.array(0.0)
    return {k: np.asarray(v, float).astype(np.float32).astype(np.float64) for k, v in p.items()}


def surrogate_x(q):
    cubic = round_f32(tables.dyadic_table(16, 3))

    def f(u, lam):
        u, lam = np.asarray(u, float), np.asarray(lam, float)
        with np.errstate(divide="ignore"):
            ll = np.where(lam > 0, np.log(np.where(lam > 0, lam, 1.0)), -np.inf)
        llc = np.clip(ll, LO, HI)  # outside the range: the network at the nearer end
        w = dyadic_transform_f32(cubic, u.astype(np.float32))[0].astype(np.float64)
        P = mlp.forward(q, w, mlp.g_feature(llc, LO, HI), bf16=True)
        s = lam + NU
        return np.maximum(s + 2 * np.sqrt(s) * P, 0.0)
    return f


def main():
    rows = []
    Y, Pf, Pc = cir.level_replay(CIR, 10, cir.EXACT, 93, np.array([777, 778]))
    rows += [("exact", 93, p, y, a, b) for p, y, a, b in zip((777, 778), Y, Pf, Pc)]
    Y, Pf, Pc = cir.level_replay(CIR, 10, cir.CORRECTION, 94, np.array([31, 32]), surrogate_x=surrogate_x(damped_params()))
    rows += [("correction", 94, p, y, a, b) for p, y, a, b in zip((31, 32), Y, Pf, Pc)]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "level10_paths.txt")
    with open(out, "w") as f:
        f.write("# CIR level-10 paths from the oracle's replay (written by make_level10_paths.py)\n")
        f.write("# case seed path Y P_f P_c\n")
        for r in rows:
            f.write(f"{r[0]} {r[1]} {r[2]} {float(r[3])!r} {float(r[4])!r} {float(r[5])!r}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
