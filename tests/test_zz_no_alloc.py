"""The allocation-free loss and gradient entry point
(lbm_mlp_loss_grad_noalloc) against lbm_mlp_loss_grad, through the C ABI:
two calls in a row, the second with a smaller batch, each equal bit for bit
to the allocating entry point's result (same kernels, same summation order),
in both precisions; a batch above the scratch array's limit is refused."""
import numpy as np
import pytest

from paper_2510_14712_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_loss_grad_matches_allocating_entry_point(precision):
    import torch
    from paper_2510_14712_amd import lbm
    lbm.load()
    params = inputs.mlp_params(51, scale=1.2).astype(np.float32)
    rng = np.random.default_rng(52)
    for B in (4096, 1024):  # the second call uses less of the scratch array than the first
        xn = rng.uniform(-1, 1, (B, 2)).astype(np.float32)
        tn = rng.normal(size=(B, 3)).astype(np.float32)
        print(f"case noalloc loss_grad precision={precision} B={B}", flush=True)
        l0, g0 = lbm.mlp_loss_grad(params, xn, tn, precision=precision)
        l1, g1 = lbm.mlp_loss_grad_noalloc(params, xn, tn, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(g0, g1) and torch.equal(l0, l1)
        assert float(g1.abs().max()) > 0


def test_noalloc_batch_limit():
    from paper_2510_14712_amd import lbm
    L = lbm.load()
    B = 8192 + 64  # LBM_MLP_NOALLOC_MAX_BATCH + 64
    assert L.lbm_mlp_loss_grad_noalloc(None, None, None, B, None, None, 0, None) == lbm.LBM_EINVAL
