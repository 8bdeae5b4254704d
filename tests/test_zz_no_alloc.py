"""The selector network's loss gradient through the entry point that
allocates nothing (a fixed device workspace for batches of up to 512
samples), against the allocating entry point, on two calls in a row, the
second with a smaller batch."""
import ctypes

import numpy as np
import pytest

import paper_1203_2739_amd as spx
from gpu_util import dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_no_alloc_loss_grad_matches_allocating_entry_point():
    L = spx.lib()
    rng = np.random.default_rng(77)
    theta = dev((rng.standard_normal(spx.MLP_PARAMS) * 0.2).astype(np.float32))
    for B in (300, 37):
        X = dev(rng.standard_normal((B, spx.NFEATURES)).astype(np.float32))
        lab = dev(rng.integers(0, spx.NCHOICES, B).astype(np.int32))
        loss_a = torch.zeros(1, dtype=torch.float32, device="cuda")
        grad_a = torch.zeros(spx.MLP_PARAMS, dtype=torch.float32, device="cuda")
        spx.mlp_loss_grad(theta, X, lab, loss_a, grad_a)
        loss_b = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
        grad_b = torch.full((spx.MLP_PARAMS,), np.nan, dtype=torch.float32, device="cuda")
        spx.mlp_loss_grad_noalloc(theta, X, lab, loss_b, grad_b)
        # same kernels, same order of operations: identical bits
        assert np.array_equal(host(loss_a), host(loss_b)), B
        assert np.array_equal(host(grad_a), host(grad_b)), B


def test_no_alloc_rejects_batches_over_its_workspace():
    theta = torch.zeros(spx.MLP_PARAMS, dtype=torch.float32, device="cuda")
    X = torch.zeros((513, spx.NFEATURES), dtype=torch.float32, device="cuda")
    lab = torch.zeros(513, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(spx.MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(spx.SpxError):
        spx.mlp_loss_grad_noalloc(theta, X, lab, loss, grad)
