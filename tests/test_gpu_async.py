"""Stream-ordered level calls (mlmc_level_*_async): the same kernels as the
synchronous calls, with the sums written by the device into caller memory.
Every field must equal the synchronous call's bit for bit, for every level
family, launch shape and kind, when several calls share one stream (the
workspace and fallback counter are reused in stream order) and when they are
spread over several streams from one host thread."""
import numpy as np
import pytest
import torch

import paper_2012_09715_amd as A
from paper_2012_09715_amd import mlmc_driver as D

pytestmark = pytest.mark.gpu

GBM = dict(S0=1.0, r=0.05, sigma=0.2, T=1.0, K=1.0, scheme=1, payoff=1)
CIR = dict(v0=0.04, kappa=0.5, theta=0.04, xi=0.3, T=1.0, functional=1)
NU = 4 * 0.5 * 0.04 / 0.3 ** 2


@pytest.fixture(scope="module")
def approx():
    return dict(lin=A.Table.dyadic(16, 1), geo=A.Table.geometric(0.7, 64, 3), const=A.Table.const(64),
                chi=A.Chi2Table.create(NU, 3), sur=A.Surrogate.create(NU, -8.0, 10.0, seed=3),
                low=A.Surrogate.create(NU, -60.0, -59.0, seed=4))


def calls(ap):
    """(synchronous call, stream-ordered call) pairs covering every family:
    dense and one-path-per-wavefront launch shapes, every kind, zero paths,
    and surrogate calls that fall back to the exact inverse."""
    out = []
    for l, n in ((0, 5000), (3, 777), (8, 3000), (8, 20000), (10, 300)):
        for k, tab in ((0, None), (1, ap["lin"]), (2, ap["geo"]), (2, ap["const"])):
            out.append((lambda s=None, l=l, n=n, k=k, tab=tab: A.mlmc_level_gbm(GBM, l, n, k, tab, 7, 11, stream=s),
                        lambda sums, l=l, n=n, k=k, tab=tab: A.mlmc_level_gbm_async(GBM, l, n, k, tab, 7, 11, sums)))
    out.append((lambda s=None: A.mlmc_level_gbm(GBM, 4, 0, 1, ap["lin"], 7, 0, stream=s),
                lambda sums: A.mlmc_level_gbm_async(GBM, 4, 0, 1, ap["lin"], 7, 0, sums)))
    for l, n in ((0, 3000), (2, 300), (5, 5000)):
        for k in (0, 1, 2, 3):
            out.append((lambda s=None, l=l, n=n, k=k: A.mlmc_level_cir_table(CIR, l, n, k, ap["chi"], 8, 3, stream=s),
                        lambda sums, l=l, n=n, k=k: A.mlmc_level_cir_table_async(CIR, l, n, k, ap["chi"], 8, 3,
                                                                                 sums)))
            out.append((lambda s=None, l=l, n=n, k=k: A.mlmc_level_cir_sankaran(CIR, l, n, k, 9, 0, stream=s),
                        lambda sums, l=l, n=n, k=k: A.mlmc_level_cir_sankaran_async(CIR, l, n, k, 9, 0, sums)))
            out.append((lambda s=None, l=l, n=n, k=k: A.mlmc_level_cir_em(CIR, l, n, k, 10, 0, stream=s),
                        lambda sums, l=l, n=n, k=k: A.mlmc_level_cir_em_async(CIR, l, n, k, 10, 0, sums)))
        for k, sur in ((1, "sur"), (2, "sur"), (1, "low"), (2, "low")):
            out.append((lambda s=None, l=l, n=n, k=k, sur=sur: A.mlmc_level_cir(CIR, l, n, k, ap[sur], 12, 0,
                                                                               stream=s),
                        lambda sums, l=l, n=n, k=k, sur=sur: A.mlmc_level_cir_async(CIR, l, n, k, ap[sur], 12, 0,
                                                                                   sums)))
    out.append((lambda s=None: A.mlmc_level_cir(CIR, 3, 0, 0, None, 12, 0, stream=s),
                lambda sums: A.mlmc_level_cir_async(CIR, 3, 0, 0, None, 12, 0, sums)))
    return out


def same(a, b):
    return (a["n"] == b["n"] and a["sum"] == b["sum"] and a["sum_pf"] == b["sum_pf"]
            and a["sum_pc"] == b["sum_pc"] and a["fallbacks"] == b["fallbacks"])


def test_one_stream_matches_sync(approx):
    pairs = calls(approx)
    ref = [p[0]() for p in pairs]
    assert any(r["fallbacks"] > 0 for r in ref)
    # all calls back to back on one stream, one wait at the end; NaN marks
    # rows that were never written
    st = torch.cuda.Stream()
    sums = torch.full((len(pairs), 8), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        for i, p in enumerate(pairs):
            p[1](sums[i])
    st.synchronize()
    host = sums.cpu()
    for i, r in enumerate(ref):
        got = A.sums_dict(host[i])
        assert same(got, r), (i, got, r)
    # a synchronous call on the same stream afterwards sees a clear counter
    again = pairs[-2][0](st)
    assert same(again, ref[-2])


@pytest.mark.parametrize("n_streams", [2, 5])
def test_several_streams_match_sync(approx, n_streams):
    pairs = calls(approx)
    ref = [p[0]() for p in pairs]
    jobs = [p[1] for p in pairs]
    costs = [float(len(pairs) - i) for i in range(len(pairs))]
    D.warm_streams(lambda: A.mlmc_level_gbm(GBM, 0, 2, 0, None, 1), n_streams)
    for rep in range(2):
        res, wall = D.run_async(jobs, costs, n_streams)
        assert wall > 0
        for i, (a, b) in enumerate(zip(res, ref)):
            assert same(a, b), (rep, i, a, b)


def test_path_out_matches_sync(approx):
    n = 4000
    po_s = torch.zeros(n * 3, dtype=torch.float64, device="cuda")
    po_a = torch.full((n * 3,), float("nan"), dtype=torch.float64, device="cuda")
    sums = torch.zeros(8, dtype=torch.float64, device="cuda")
    r = A.mlmc_level_cir_table(CIR, 4, n, 2, approx["chi"], 5, 17, path_out=po_s)
    A.mlmc_level_cir_table_async(CIR, 4, n, 2, approx["chi"], 5, 17, sums, path_out=po_a)
    torch.cuda.synchronize()
    assert torch.equal(po_s, po_a)
    assert same(A.sums_dict(sums.cpu()), r)
    g_s = torch.zeros(n * 3, dtype=torch.float64, device="cuda")
    g_a = torch.full((n * 3,), float("nan"), dtype=torch.float64, device="cuda")
    r = A.mlmc_level_gbm(GBM, 6, n, 2, approx["lin"], 5, 0, path_out=g_s)
    A.mlmc_level_gbm_async(GBM, 6, n, 2, approx["lin"], 5, 0, sums, path_out=g_a)
    torch.cuda.synchronize()
    assert torch.equal(g_s, g_a)
    assert same(A.sums_dict(sums.cpu()), r)


def test_zero_paths_written_and_errors(approx):
    sums = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    A.mlmc_level_cir_em_async(CIR, 2, 0, 1, 0, 0, sums)
    torch.cuda.synchronize()
    assert np.array_equal(sums.cpu().numpy(), np.zeros(8))
    sums.fill_(float("nan"))
    # argument errors come back before anything is enqueued
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_level_gbm_async(GBM, 2, 100, 1, None, 1, 0, sums)
    with pytest.raises(A.AicdfError, match="ERANGE"):
        A.mlmc_level_cir_table_async(CIR, 13, 100, 0, None, 1, 0, sums)
    with pytest.raises(A.AicdfError, match="nu"):
        A.mlmc_level_cir_async(CIR, 2, 100, 1, A.Surrogate.create(2.0, -8.0, 10.0, seed=0), 1, 0, sums)
    with pytest.raises(A.AicdfError):
        A.mlmc_level_gbm_async(GBM, 2, 100, 0, None, 1, 0, torch.zeros(8, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert torch.isnan(sums).all()
