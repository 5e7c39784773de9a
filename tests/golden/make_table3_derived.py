"""Writes table3_derived.txt: the four-way variance drop of nested MLMC for
GBM with P = X and the Euler-Maruyama scheme (Section 4.1, Table 3),
predicted from each approximation's own mean-square error.  Calls only
oracle/.

Prediction.  With eps = Z - Z~ small, the coupled fine and coarse paths of
level l >= 1 respond to eps_n through sensitivities that differ by
sigma sqrt(delta) Z' (Z' the other normal of the coarse pair), so to leading
order Var(D_l) = sigma^4 delta T E(X^2) E(eps^2), while
Var(Y_l) = sigma^4 delta T E(X^2) / 2 (strong order 1/2): the ratio is
2 E(eps^2), and log2(V~_l / v^_l) = 1 + log2 E(eps^2), independent of l.
E(eps^2) is the mean over the u24 grid (the uniforms that drive the fused
paths: odd multiples of 2^-24) of (Phi^-1(u) - Z~(u))^2, Z~ the FP32
evaluation of the table (Code 1 / Code 2); the exact normal of a coupled draw
comes from the u53 whose leading bits are that u24, a difference worth
2^-29 in E(eps^2), negligible here.  The last column repeats the prediction
with the dyadic tables' singular intervals (t = min(u, 1-u) < 2^-15, one draw
in 8192) left out.

    python tests/golden/make_table3_derived.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import tables  # noqa: E402
from oracle.dtypes import round_f32  # noqa: E402
from oracle.normal import Phi_inv  # noqa: E402
from oracle.transform import const_transform, dyadic_transform_f32  # noqa: E402


def main():
    u = (np.arange(1 << 23, dtype=np.float64) + 0.5) * 2.0 ** -23
    z = Phi_inv(u)
    t = np.minimum(u, 1.0 - u)
    cases = {
        "rademacher": const_transform(np.array([-1.0, 1.0]), u),
        "const1024": const_transform(round_f32(tables.const_table(1024)), u),
        "linear16": dyadic_transform_f32(round_f32(tables.dyadic_table(16, 1)), u.astype(np.float32))[0],
        "cubic16": dyadic_transform_f32(round_f32(tables.dyadic_table(16, 3)), u.astype(np.float32))[0],
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table3_derived.txt")
    with open(out, "w") as f:
        f.write("# Table 3 (GBM, P = X, Euler-Maruyama): log2(V~/v^) predicted as 1 + log2 E(eps^2)\n")
        f.write("# (written by make_table3_derived.py)\n")
        f.write("# table mse_u24 predicted predicted_without_singular_rows\n")
        for name, za in cases.items():
            e2 = (np.asarray(za, np.float64) - z) ** 2
            keep = t >= 2.0 ** -15
            f.write(f"{name} {e2.mean():.6e} {1 + np.log2(e2.mean()):.3f} {1 + np.log2(e2[keep].mean()):.3f}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
