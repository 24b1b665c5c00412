"""The allocation-free forward pass of the surrogate network
(mlp_predict_device_noalloc) against mlp_predict, through the C ABI.

Both run the same GEMM kernels on the same parameters, so the outputs must be
identical; two calls in a row, the second with fewer rows, check that the
shared static scratch array carries nothing from one call to the next."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_0459_amd import lbcap
    return lbcap


def test_noalloc_predict_matches_predict(L):
    import torch
    net = L.MLP(seed=5)
    rng = np.random.default_rng(77)
    for rows in (L.MLP_NOALLOC_MAX_ROWS - 187, 301):
        X = rng.normal(0.0, 1.0, (rows, L.MLP.N_IN)).astype(np.float32)
        ref = net.predict(X)
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.full((rows, L.MLP.N_OUT), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        net.predict_device_noalloc(Xd, Yd)
        torch.cuda.synchronize()
        got = Yd.cpu().numpy()
        print(f"rows {rows}: max |noalloc - predict| = {np.abs(got - ref).max():.3e}")
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref)


def test_noalloc_predict_rejects_too_many_rows(L):
    import torch
    net = L.MLP(seed=5)
    n = L.MLP_NOALLOC_MAX_ROWS + 1
    Xd = torch.zeros((n, L.MLP.N_IN), dtype=torch.float32, device="cuda")
    Yd = torch.zeros((n, L.MLP.N_OUT), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LbError) as e:
        net.predict_device_noalloc(Xd, Yd)
    assert e.value.code == L.LB_EINVAL
    assert "MLP_NOALLOC_MAX_ROWS" in str(e.value)
