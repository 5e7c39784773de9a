#!/usr/bin/env python3
"""One GPU-filling call of each fused level kernel and of the surrogate's
training and inference, for collecting hardware counters per kernel
(rocprofv3 --pmc ... -- python3 paper_2012_09715_amd/profile_levels.py).

Calls (after one untimed warm-up of each):
  GBM Euler-Maruyama, discounted call, level 8, 2^20 paths: exact,
      approximate (16-row linear dyadic table) and correction kinds
  CIR time average, level 6: approximate kind with the linear chi-squared
      table (2^20 paths), the surrogate (2^20 paths), and the exact kind
      (2^17 paths)
  surrogate: one training epoch over 2^20 exact targets (batch 4096) and
      one forward pass over 2^22 inputs
Prints one line per call with its kernel time from the library's events.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

import paper_2012_09715_amd as A  # noqa: E402
from paper_2012_09715_amd import mlmc_driver as D  # noqa: E402


def main():
    lin = A.Table.dyadic(16, 1)
    chi = A.Chi2Table.create(D.NU_CIR, 1)
    sur = A.Surrogate.create(D.NU_CIR, *D.SURROGATE_RANGE, seed=1)
    u, ll, t = sur.make_data(1 << 20, 2)
    calls = [
        ("gbm exact l8", lambda: A.mlmc_level_gbm(D.GBM_CALL, 8, 1 << 20, A.KIND_EXACT, None, 3)),
        ("gbm approx l8", lambda: A.mlmc_level_gbm(D.GBM_CALL, 8, 1 << 20, A.KIND_APPROX, lin, 3)),
        ("gbm correction l8", lambda: A.mlmc_level_gbm(D.GBM_CALL, 8, 1 << 20, A.KIND_CORRECTION, lin, 3)),
        ("cir table approx l6", lambda: A.mlmc_level_cir_table(D.CIR_PARAMS, 6, 1 << 20, A.KIND_APPROX, chi, 4)),
        ("cir surrogate approx l6", lambda: A.mlmc_level_cir(D.CIR_PARAMS, 6, 1 << 20, A.KIND_APPROX, sur, 4)),
        ("cir exact l6", lambda: A.mlmc_level_cir(D.CIR_PARAMS, 6, 1 << 17, A.KIND_EXACT, None, 4)),
    ]
    for name, fn in calls:
        fn()
        s = fn()
        print(f"{name}: {s['kernel_ms']:.3f} ms", flush=True)
    ue, lle, _ = sur.make_data(1 << 22, 5)
    for rep in range(2):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        sur.train(u, ll, t, epochs=1, batch=4096, lr=1e-3, seed=rep)
        ev1.record()
        torch.cuda.synchronize()
        if rep:
            print(f"surrogate training epoch (2^20 samples): {ev0.elapsed_time(ev1):.3f} ms", flush=True)
        ev0.record()
        sur.forward(ue, lle)
        ev1.record()
        torch.cuda.synchronize()
        if rep:
            print(f"surrogate forward (2^22 inputs): {ev0.elapsed_time(ev1):.3f} ms", flush=True)


if __name__ == "__main__":
    main()
