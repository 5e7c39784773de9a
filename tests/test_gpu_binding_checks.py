"""The Python binding rejects wrong caller buffers before anything is
launched: wrong dtype, too few elements, another device (an undersized or
mistyped buffer must never reach a kernel, which would write past it)."""
import pytest
import torch

import paper_2012_09715_amd as A
from paper_2012_09715_amd import mlmc_driver as D

pytestmark = pytest.mark.gpu


def _cuda(n, dtype):
    return torch.rand(n, device="cuda", dtype=torch.float64).to(dtype).clamp_(1e-6, 1 - 1e-6)


def test_transform_output_too_small():
    u = _cuda(1000, torch.float32)
    tab = A.Table.dyadic(16, 1)
    for fn in (lambda z: A.approx_icdf_linear(tab, u, z=z), lambda z: A.approx_icdf_const(A.Table.const(), u, z=z),
               lambda z: A.exact_icdf(u, z=z)):
        with pytest.raises(A.AicdfError):
            fn(torch.empty(999, dtype=torch.float32, device="cuda"))


def test_ncx2_exact_dtype_and_size():
    u = _cuda(256, torch.float64)
    lam = torch.full((256,), 10.0, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AicdfError):
        A.ncx2_icdf_exact(D.NU_CIR, u.float(), lam)       # float32 u
    with pytest.raises(A.AicdfError):
        A.ncx2_icdf_exact(D.NU_CIR, u, lam.float())       # float32 lambda
    with pytest.raises(A.AicdfError):
        A.ncx2_icdf_exact(D.NU_CIR, u, lam[:255])         # lambda too short
    with pytest.raises(A.AicdfError):
        A.ncx2_icdf_exact(D.NU_CIR, u, lam, x=torch.empty(256, dtype=torch.float32, device="cuda"))
    with pytest.raises(A.AicdfError):
        A.ncx2_icdf_exact(D.NU_CIR, u, lam, x=torch.empty(255, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    x = A.ncx2_icdf_exact(D.NU_CIR, u, lam)
    assert torch.isfinite(x).all()


def test_exact_inverse_lambda_bound_gives_nan():
    u = torch.full((8,), 0.3, dtype=torch.float64, device="cuda")
    lam = torch.tensor([10.0, 1e8, 1.0000001e8, 1e12, -1.0, float("nan"), 0.0, 1e3], dtype=torch.float64,
                       device="cuda")
    for n in (8, 9000):  # one inverse per wavefront / per thread
        uu, ll = u.repeat(n // 8 + 1)[:n].contiguous(), lam.repeat(n // 8 + 1)[:n].contiguous()
        x = A.ncx2_icdf_exact(D.NU_CIR, uu, ll).cpu()[:8]
        assert torch.isfinite(x[[0, 1, 6, 7]]).all()
        assert torch.isnan(x[2:6]).all()


def test_level_path_out_checks():
    tab = A.Table.dyadic(16, 1)
    for bad in (torch.empty(3 * 100 - 1, dtype=torch.float64, device="cuda"),
                torch.empty(3 * 100, dtype=torch.float32, device="cuda")):
        with pytest.raises(A.AicdfError):
            A.mlmc_level_gbm(D.GBM_CALL, 2, 100, A.KIND_APPROX, tab, 1, 0, path_out=bad)
        with pytest.raises(A.AicdfError):
            A.mlmc_level_cir_em(D.CIR_PARAMS, 2, 100, A.KIND_APPROX, 1, 0, path_out=bad)


def test_surrogate_buffer_checks():
    s = A.Surrogate.create(D.NU_CIR, -8.0, 10.0, seed=1)
    u = _cuda(512, torch.float32)
    g = torch.zeros(512, dtype=torch.float32, device="cuda")
    with pytest.raises(A.AicdfError):
        s.forward(u.double(), g)
    with pytest.raises(A.AicdfError):
        s.forward(u, g[:511])
    with pytest.raises(A.AicdfError):
        s.forward(u, g, p=torch.empty(511, dtype=torch.float32, device="cuda"))
    with pytest.raises(A.AicdfError):
        s.train(u, g, torch.zeros(511, dtype=torch.float32, device="cuda"), epochs=1)


def test_bw_probe_size_checks():
    a = torch.empty(1024, dtype=torch.float32, device="cuda")
    b = torch.empty(512, dtype=torch.float32, device="cuda")
    with pytest.raises(A.AicdfError):
        A.bw_probe(0, a, b, n_bytes=4096)
