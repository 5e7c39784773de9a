"""The allocation-free GBM level (mlmc_level_gbm_noalloc) against the
stream-ordered call it mirrors (mlmc_level_gbm_async): the same kernels on
the same draws, so the 8 sums and the per-path values must be bit-identical.
Two calls in a row per case, the second smaller, so that the shared scratch
array still holds the first call's partials when the second runs."""
import pytest
import torch

import paper_2012_09715_amd as A
from paper_2012_09715_amd import mlmc_driver as D

pytestmark = pytest.mark.gpu

MIL = dict(D.GBM_CALL, scheme=1)


def pair(params, level, n, kind, table, seed, offset):
    s1 = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
    s2 = torch.full((8,), -2.0, dtype=torch.float64, device="cuda")
    p1 = torch.full((3 * n,), -1.0, dtype=torch.float64, device="cuda")
    p2 = torch.full((3 * n,), -2.0, dtype=torch.float64, device="cuda")
    A.mlmc_level_gbm_async(params, level, n, kind, table, seed, offset, s1, path_out=p1)
    A.mlmc_level_gbm_noalloc(params, level, n, kind, table, seed, offset, s2, path_out=p2)
    torch.cuda.synchronize()
    return s1.cpu(), s2.cpu(), p1.cpu(), p2.cpu()


@pytest.mark.parametrize("kind", [A.KIND_EXACT, A.KIND_APPROX, A.KIND_CORRECTION])
@pytest.mark.parametrize("params", [D.GBM_CALL, MIL], ids=["em", "milstein"])
def test_noalloc_matches_async(kind, params):
    tab = A.Table.dyadic(16, 1)
    # (level, paths): a GPU-filling call (4096 work-groups), then smaller
    # ones, the last in the one-path-per-wavefront shape (2^8 steps)
    for level, n, off in ((4, 1_100_000, 0), (3, 5000, 77), (8, 300, 1 << 33), (0, 1, 5)):
        a, b, pa, pb = pair(params, level, n, kind, tab, 1234 + level, off)
        assert torch.equal(a, b), (level, n, a, b)
        assert torch.equal(pa, pb)
        assert b[7].item() == n and b[6].item() == 0.0


def test_noalloc_zero_paths_and_errors():
    tab = A.Table.dyadic(16, 1)
    s = torch.full((8,), 5.0, dtype=torch.float64, device="cuda")
    A.mlmc_level_gbm_noalloc(D.GBM_CALL, 3, 0, A.KIND_APPROX, tab, 1, 0, s)
    torch.cuda.synchronize()
    assert torch.all(s.cpu() == 0.0)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_level_gbm_noalloc(D.GBM_CALL, 3, 10, A.KIND_APPROX, None, 1, 0, s)
    with pytest.raises(A.AicdfError, match="ERANGE"):
        A.mlmc_level_gbm_noalloc(D.GBM_CALL, 21, 10, A.KIND_EXACT, None, 1, 0, s)
