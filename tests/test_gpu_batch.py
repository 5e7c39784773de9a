"""Level-batched calls (one launch for many levels of an estimator) against
the per-level stream-ordered calls: every job's 8 sums bit-identical to its
own level call, for exact-only, approximate-only and mixed batches, both
launch shapes and empty jobs."""
import pytest
import torch

import paper_2012_09715_amd as A
from paper_2012_09715_amd import mlmc_driver as D

pytestmark = pytest.mark.gpu

E, AP, C = A.KIND_EXACT, A.KIND_APPROX, A.KIND_CORRECTION


def per_level(params, jobs, table, seed):
    out = torch.zeros((len(jobs), 8), dtype=torch.float64, device="cuda")
    for j, (level, kind, n, off) in enumerate(jobs):
        A.mlmc_level_gbm_async(params, level, n, kind, table, seed, off, out[j])
    torch.cuda.synchronize()
    return out.cpu()


def batched(params, jobs, table, seed):
    out = torch.full((len(jobs), 8), -7.0, dtype=torch.float64, device="cuda")
    A.mlmc_levels_gbm(params, jobs, table, seed, out)
    torch.cuda.synchronize()
    return out.cpu()


JOBS = {
    "exact": [(10, E, 300, 0), (8, E, 5000, 11), (0, E, 200_000, 3), (4, E, 70_000, 1 << 33), (2, E, 0, 0),
              (9, E, 9000, 5)],
    "approx": [(10, AP, 700, 2), (6, AP, 100_000, 0), (0, AP, 1_500_000, 9), (3, AP, 1, 0)],
    "mixed": [(10, C, 40, 0), (9, C, 600, 1), (10, AP, 2000, 0), (0, C, 120_000, 0), (0, AP, 1_100_000, 0),
              (5, C, 3000, 17), (5, AP, 50_000, 0), (1, E, 10_000, 0), (8, AP, 0, 0)],
}


@pytest.mark.parametrize("name", list(JOBS))
@pytest.mark.parametrize("params", [D.GBM_CALL, dict(D.GBM_CALL, scheme=1, payoff=0)], ids=["em_call", "mil_x"])
@pytest.mark.parametrize("tabkind", ["dyadic", "const", "geometric"])
def test_batch_equals_level_calls(name, params, tabkind):
    tab = {"dyadic": lambda: A.Table.dyadic(16, 1), "const": lambda: A.Table.const(1024),
           "geometric": lambda: A.Table.geometric(0.7, 64, 3)}[tabkind]()
    jobs = JOBS[name]
    ref = per_level(params, jobs, tab, 4321)
    got = batched(params, jobs, tab, 4321)
    assert torch.equal(got, ref), (got - ref).abs().max()
    for j, job in enumerate(jobs):
        assert got[j, 7].item() == job[2]


def test_batch_full_size_estimator():
    # an allocation of ~10^7 paths over levels 0..10 (Milstein, the large
    # fused run's scheme), nested estimator in one launch
    p = dict(D.GBM_CALL, scheme=1)
    tab = A.Table.dyadic(16, 1)
    jobs = [(l, C, max(8_000_000 >> (2 * l), 2), 0) for l in range(10, -1, -1)] + \
           [(l, AP, max(8_000_000 >> l, 2), 0) for l in range(10, -1, -1)]
    assert torch.equal(batched(p, jobs, tab, 99), per_level(p, jobs, tab, 99))


def test_batch_errors():
    tab = A.Table.dyadic(16, 1)
    out = torch.zeros((30, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(A.AicdfError, match="ERANGE"):
        A.mlmc_levels_gbm(D.GBM_CALL, [(1, E, 10, 0)] * 25, tab, 1, out)
    with pytest.raises(A.AicdfError, match="job 1"):
        A.mlmc_levels_gbm(D.GBM_CALL, [(1, E, 10, 0), (21, E, 10, 0)], tab, 1, out)
    with pytest.raises(A.AicdfError, match="job 0"):
        A.mlmc_levels_gbm(D.GBM_CALL, [(1, 3, 10, 0)], tab, 1, out)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_levels_gbm(D.GBM_CALL, [(1, AP, 10, 0)], None, 1, out)
    with pytest.raises(A.AicdfError):
        A.mlmc_levels_gbm(D.GBM_CALL, [(1, E, 10, 0)] * 3, tab, 1, out[:2].reshape(-1)[:16].contiguous())
