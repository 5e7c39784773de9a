"""Level calls on several streams from several host threads (the library
keeps one workspace per stream): the sums equal those of the same calls made
one after another, bit for bit, and the nested-MLMC driver's concurrent pass
reproduces its sequential pass."""
import pytest
import torch

import paper_2012_09715_amd as A
from paper_2012_09715_amd import mlmc_driver as D

pytestmark = pytest.mark.gpu

GBM = dict(S0=1.0, r=0.05, sigma=0.2, T=1.0, K=1.0, scheme=1, payoff=1)
CIR = dict(v0=0.04, kappa=0.5, theta=0.04, xi=0.3, T=1.0, functional=1)


def test_concurrent_level_calls_match_sequential():
    lin = A.Table.dyadic(16, 1)
    chi = A.Chi2Table.create(4 * 0.5 * 0.04 / 0.09, 1)
    jobs = []
    for l in range(0, 9):
        for k in (0, 1, 2):
            jobs.append(lambda l=l, k=k: A.mlmc_level_gbm(GBM, l, 3000 + 17 * l, k, lin, 11, 5))
    for l in range(0, 6):
        for k in (0, 1, 2):
            # few-path exact and correction calls run one path per wavefront
            jobs.append(lambda l=l, k=k: A.mlmc_level_cir_table(CIR, l, 300 + l, k, chi, 12, 0))
        jobs.append(lambda l=l: A.mlmc_level_cir_sankaran(CIR, l, 200, 2, 13, 0))
    seq = [j() for j in jobs]
    for n_streams in (2, 4, 8):
        par, wall = D.run_concurrent(jobs[::-1], n_streams)
        par = par[::-1]
        assert wall > 0
        for a, b in zip(seq, par):
            assert a["n"] == b["n"] and a["sum"] == b["sum"]
            assert a["sum_pf"] == b["sum_pf"] and a["sum_pc"] == b["sum_pc"]


def test_concurrent_errors_propagate():
    jobs = [lambda: A.mlmc_level_gbm(GBM, 2, 100, 0, None, 1),
            lambda: A.mlmc_level_gbm(GBM, 2, 100, 1, None, 1)]  # approximate kind without a table
    with pytest.raises(A.AicdfError, match="EINVAL"):
        D.run_concurrent(jobs, 2)


def test_nested_driver_concurrent_pass():
    lin = A.Table.dyadic(16, 1)
    r = D.nested_mlmc("gbm", D.GBM_CALL, 6, 2e-3, lin, seed=5, n_pilot=1 << 14)
    assert r["concurrent_sums_identical"]
    assert r["wall_ms_hat_concurrent"] > 0 and r["wall_ms_tilde_concurrent"] > 0
    assert r["measured_speedup_concurrent"] > 0
