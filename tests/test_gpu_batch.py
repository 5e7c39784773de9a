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


# ------------------------------------------------------------------ CIR
CIRP = dict(v0=0.04, kappa=0.5, theta=0.04, xi=0.3, T=1.0, functional=1)
NU = 4 * 0.5 * 0.04 / 0.3 ** 2

CIR_JOBS = {
    "exact": [(6, E, 200, 0), (2, E, 3000, 5), (0, E, 150_000, 0), (4, E, 0, 0), (8, E, 2, 77)],
    "approx": [(6, AP, 20_000, 0), (0, AP, 300_000, 3), (3, AP, 1, 0)],
    "mixed": [(8, C, 2, 0), (6, C, 300, 0), (6, AP, 5000, 0), (0, C, 140_000, 9), (0, AP, 400_000, 0),
              (3, E, 1000, 0), (2, C, 0, 0)],
}


def cir_level_async(params, level, n, kind, approx, seed, off, sums):
    if isinstance(approx, A.Chi2Table):
        return A.mlmc_level_cir_table_async(params, level, n, kind, approx, seed, off, sums)
    if approx == "em":
        return A.mlmc_level_cir_em_async(params, level, n, kind, seed, off, sums)
    if approx == "sankaran":
        return A.mlmc_level_cir_sankaran_async(params, level, n, kind, seed, off, sums)
    return A.mlmc_level_cir_async(params, level, n, kind, approx, seed, off, sums)


@pytest.fixture(scope="module")
def cir_approxes():
    return {"surrogate": A.Surrogate.create(NU, -8.0, 10.0, seed=3), "poly1": A.Chi2Table.create(NU, 1),
            "poly3": A.Chi2Table.create(NU, 3), "em": "em", "sankaran": "sankaran"}


@pytest.mark.parametrize("name", list(CIR_JOBS))
@pytest.mark.parametrize("apx", ["surrogate", "poly1", "poly3", "em", "sankaran"])
@pytest.mark.parametrize("functional", [0, 1])
def test_cir_batch_equals_level_calls(cir_approxes, name, apx, functional):
    if name == "exact" and apx != "surrogate":
        pytest.skip("the exact kind does not depend on the approximation")
    p = dict(CIRP, functional=functional)
    approx = cir_approxes[apx]
    jobs = CIR_JOBS[name]
    ref = torch.zeros((len(jobs), 8), dtype=torch.float64, device="cuda")
    for j, (level, kind, n, off) in enumerate(jobs):
        cir_level_async(p, level, n, kind, approx, 555, off, ref[j])
    got = torch.full((len(jobs), 8), -7.0, dtype=torch.float64, device="cuda")
    A.mlmc_levels_cir(p, jobs, None if name == "exact" else approx, 555, got)
    torch.cuda.synchronize()
    assert torch.equal(got.cpu(), ref.cpu()), (got.cpu() - ref.cpu()).abs().max()


def test_cir_batch_errors(cir_approxes):
    out = torch.zeros((30, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(A.AicdfError, match="two-way"):
        A.mlmc_levels_cir(CIRP, [(1, 3, 10, 0)], cir_approxes["poly1"], 1, out)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_levels_cir(CIRP, [(1, AP, 10, 0)], None, 1, out)
    with pytest.raises(A.AicdfError, match="job 1"):
        A.mlmc_levels_cir(CIRP, [(1, E, 10, 0), (13, E, 10, 0)], None, 1, out)
    other = A.Chi2Table.create(2.0, 1)
    with pytest.raises(A.AicdfError, match="nu"):
        A.mlmc_levels_cir(CIRP, [(1, AP, 10, 0)], other, 1, out)
