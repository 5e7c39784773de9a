"""GPU parity of the Sankaran approximation (Section 5.1's comparator): the
transform and the CIR level that uses it, against the oracle.

Transform tolerance: FP32 arithmetic around the same exact normal; the
relative error of B (a few eps32, |z| <= 5.6 on the u24 grid) is amplified
by the power 1/c1 <= 3, so |x - x_oracle| <= 1e-5 x + 1e-6 (nu + lambda).
"""
import numpy as np
import pytest
import torch

import paper_2012_09715_amd as A
from oracle import cir, sankaran
from tests.inputs import edge_uniforms, random_u24

pytestmark = pytest.mark.gpu
DEV = "cuda"
CIR = dict(v0=0.04, kappa=0.5, theta=0.04, xi=0.3, T=1.0, functional=1)
NU_CIR = 4 * 0.5 * 0.04 / 0.3 ** 2


def run(nu, u, lam):
    ug = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float32)).to(DEV)
    lg = torch.from_numpy(np.ascontiguousarray(lam, dtype=np.float32)).to(DEV)
    return A.approx_ncx2_sankaran(nu, ug, lg).cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("nu", [NU_CIR, 1.0, 5.0, 100.0])
def test_transform_parity(nu):
    n = 4096 * 3 + 29
    u = random_u24(n, seed=int(nu * 7))
    rng = np.random.default_rng(3)
    lam = np.exp(rng.uniform(np.log(1e-6), np.log(1e5), n)).astype(np.float32)
    lam[:50] = 0.0
    e = edge_uniforms(np.float32)
    e = e[(e > 0) & (e < 1)]
    u = np.concatenate([u, e]).astype(np.float32)
    lam = np.concatenate([lam, np.full(e.shape, 3.0, np.float32)])
    x = run(nu, u, lam)
    ref = sankaran.approx_x(u.astype(np.float64), nu, lam.astype(np.float64))
    tol = 1e-5 * ref + 1e-6 * (nu + lam)
    bad = ~(np.abs(x - ref) <= tol)
    assert not bad.any(), (int(bad.sum()), u[bad][:4], lam[bad][:4], x[bad][:4], ref[bad][:4])


def test_transform_benchmark_size_sampled():
    # 2^28 device-resident pairs in the benchmark's launch, checked on a sample
    n = 1 << 28
    u = torch.empty(n, dtype=torch.float32, device=DEV)
    A.uniform_fill(u, 20201217, 3, 0)
    g = torch.Generator(device=DEV)
    g.manual_seed(20201217)
    lam = torch.exp(torch.rand(n, device=DEV, generator=g) * 18.0 - 8.0)
    x = torch.empty(n, dtype=torch.float32, device=DEV)
    A.approx_ncx2_sankaran(NU_CIR, u, lam, x=x)
    pick = torch.from_numpy(np.unique(np.concatenate([np.random.default_rng(4).integers(0, n, 40_000),
                                                      [0, n - 1]]))).to(DEV)
    us, ls = u[pick].cpu().numpy(), lam[pick].cpu().numpy()
    xs = x[pick].cpu().numpy().astype(np.float64)
    ref = sankaran.approx_x(us.astype(np.float64), NU_CIR, ls.astype(np.float64))
    tol = 1e-5 * ref + 1e-6 * (NU_CIR + ls)
    assert np.all(np.abs(xs - ref) <= tol)
    del u, lam, x


def test_transform_errors_and_nan():
    u = torch.rand(16, device=DEV)
    lam = torch.rand(16, device=DEV)
    with pytest.raises(A.AicdfError, match="EALIAS"):
        A.approx_ncx2_sankaran(1.0, u, lam, x=u)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.approx_ncx2_sankaran(-1.0, u, lam)
    lam[0] = -1.0
    assert torch.isnan(A.approx_ncx2_sankaran(1.0, u, lam)[0])


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_cir_level_parity(kind):
    level, n, seed = 3, 200, 90 + kind
    out = torch.zeros(n * 3, dtype=torch.float64, device=DEV)
    A.mlmc_level_cir_sankaran(CIR, level, n, kind, seed, 0, path_out=out)
    got = out.cpu().numpy().reshape(n, 3)
    f = lambda u, lam: sankaran.approx_x(u, NU_CIR, lam)
    ref = cir.level_replay(CIR, level, kind, seed, np.arange(n), surrogate_x=f)
    scale = np.maximum(np.abs(ref[1]), 1e-3)
    for j in range(3):
        assert np.all(np.abs(got[:, j] - ref[j]) <= 2e-4 * 8 * scale), j
