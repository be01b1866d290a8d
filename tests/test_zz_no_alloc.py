"""The allocation-free MSE entry point (cmbx_mlp_mse_noalloc) against cmbx_mlp_mse with a
caller's workspace: the same gradient and loss, bit for bit, on two calls in a row (the
second smaller, so it reads partial sums the first left in the static array only if it
were wrong), through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx
    return cmbx.lib()


def _ref(L, Y, T):
    n = Y.numel()
    dY = torch.empty_like(Y)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    part = torch.empty(int(L.cmbx_mlp_mse_partials(n)), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.cmbx_mlp_mse(Y.data_ptr(), T.data_ptr(), n, dY.data_ptr(), part.data_ptr(), loss.data_ptr(), s) == 0
    return dY, loss


def test_noalloc_matches_workspace_version(L):
    g = torch.Generator(device="cuda").manual_seed(7)
    s = torch.cuda.current_stream().cuda_stream
    for n in (3_000_001, 70_000, 1):
        Y = torch.randn(n, generator=g, device="cuda")
        T = torch.randn(n, generator=g, device="cuda")
        dY = torch.full_like(Y, float("nan"))
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        assert L.cmbx_mlp_mse_noalloc(Y.data_ptr(), T.data_ptr(), n, dY.data_ptr(), loss.data_ptr(), s) == 0
        rdY, rloss = _ref(L, Y, T)
        torch.cuda.synchronize()
        assert torch.equal(dY, rdY), n
        assert torch.equal(loss, rloss), n
        exact = float(np.mean((Y.double() - T.double()).cpu().numpy() ** 2))
        assert abs(float(loss.item()) - exact) <= 1e-5 * exact, n


def test_noalloc_limit(L):
    from paper_2507_15703_amd import cmbx
    Y = torch.zeros(4, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    big = 65536 * 256 + 1   # one partial sum beyond the static array: refused before any launch
    assert L.cmbx_mlp_mse_noalloc(Y.data_ptr(), Y.data_ptr(), big, Y.data_ptr(), Y.data_ptr(), s) == cmbx.EINVAL
    assert "exceeds" in cmbx.last_error()
    assert L.cmbx_mlp_mse_noalloc(None, Y.data_ptr(), 4, Y.data_ptr(), Y.data_ptr(), s) == cmbx.EINVAL
