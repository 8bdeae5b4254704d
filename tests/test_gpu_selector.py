"""Selector network kernels against the binary64 oracle (forward, loss,
gradient, Adam), training on the GPU, and the exhaustive timing of the 24
choices.  The held-out study of the learned choice is in
test_study_selector.py."""
import numpy as np
import pytest

import paper_1203_2739_amd as spx
from gpu_util import dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rand_net(seed, B):
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(spx.MLP_PARAMS) * 0.2).astype(np.float32)
    X = rng.standard_normal((B, spx.NFEATURES)).astype(np.float32)
    labels = rng.integers(0, spx.NCHOICES, B).astype(np.int32)
    return theta, X, labels


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("B", [1, 37, 256])
def test_forward_and_gradient_match_oracle(orc, B):
    import torch
    theta, X, labels = rand_net(B, B)
    logits = torch.empty((B, spx.NCHOICES), dtype=torch.float32, device="cuda")
    spx.mlp_forward(dev(theta), dev(X), logits)
    z = orc.mlp_forward(theta.astype(np.float64), X.astype(np.float64))
    assert relmax(host(logits).astype(np.float64), z) < 1e-5
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(spx.MLP_PARAMS, dtype=torch.float32, device="cuda")
    spx.mlp_loss_grad(dev(theta), dev(X), dev(labels), loss, grad)
    l64, g64 = orc.mlp_grad(theta.astype(np.float64), X.astype(np.float64), labels)
    assert abs(float(host(loss)[0]) - l64) <= 1e-5 * max(1.0, abs(l64))
    assert relmax(host(grad).astype(np.float64), g64) < 1e-4


def test_adam_step_matches_oracle(orc):
    import torch
    theta, X, labels = rand_net(3, 64)
    rng = np.random.default_rng(4)
    m0 = (rng.standard_normal(spx.MLP_PARAMS) * 1e-3).astype(np.float32)
    v0 = (rng.random(spx.MLP_PARAMS) * 1e-5).astype(np.float32)
    g = (rng.standard_normal(spx.MLP_PARAMS) * 1e-2).astype(np.float32)
    th_d, m_d, v_d = dev(theta.copy()), dev(m0.copy()), dev(v0.copy())
    spx.mlp_adam(th_d, dev(g), m_d, v_d, 5, lr=1e-3)
    th64, m64, v64 = orc.adam_step(theta.astype(np.float64), g.astype(np.float64), m0.astype(np.float64),
                                   v0.astype(np.float64), 5, lr=1e-3)
    assert np.max(np.abs(host(th_d) - th64)) < 1e-6
    # binary32 carries 1 - beta2 with a relative error near 5e-5; the
    # optimizer step is held to the gradient's 1e-4 bound
    assert relmax(host(m_d).astype(np.float64), m64) < 1e-4
    assert relmax(host(v_d).astype(np.float64), v64) < 1e-4


def test_training_fits_a_teacher(orc):
    """Labels from a fixed random teacher network: GPU training reaches high
    accuracy, so forward, backward and the optimizer work together."""
    from paper_1203_2739_amd import selector
    rng = np.random.default_rng(11)
    teacher = (rng.standard_normal(spx.MLP_PARAMS) * 0.3)
    X = rng.standard_normal((512, spx.NFEATURES))
    labels = orc.mlp_forward(teacher, X).argmax(axis=1).astype(np.int32)
    theta, curve = selector.train(X.astype(np.float32), labels, epochs=150, batch=64, lr=3e-3, seed=1)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    logits = torch.empty((X.shape[0], spx.NCHOICES), dtype=torch.float32, device="cuda")
    spx.mlp_forward(theta, Xd, logits)
    acc = np.mean(host(logits).argmax(axis=1) == labels)
    assert curve[-1] < 0.5 * curve[0] and acc > 0.85, (curve[0], curve[-1], acc)


def test_exhaustive_timing_from_given_trees():
    """The selector's timing with the three K = 256 partitions computed
    beforehand on the host (spx_partition_tree, then
    spx_select_exhaustive_trees) times all 24 choices and returns the fastest;
    a tree with a part out of range is refused before anything runs."""
    from paper_1203_2739_amd import selector
    from synth import gen_family
    A = gen_family("F2", 77, 15000)
    trees = selector.partition_trees(A, seed=3)
    assert trees["seconds"] > 0
    T, tp = selector.measure(A, seed=3, reps=3, trees=trees)
    assert T.shape == (spx.NCHOICES,) and np.all(T > 0) and tp == trees["seconds"]
    M = spx.from_csr(A)
    x = torch.ones(A.n, dtype=torch.float64, device="cuda")
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    c, ms = spx.select_exhaustive_trees(M, trees, x, y, reps=2)
    assert c == int(np.argmin(ms))
    bad = dict(trees)
    bad["db"] = trees["db"].copy()
    bad["db"][0] = 257
    with pytest.raises(spx.SpxError):
        spx.select_exhaustive_trees(M, bad, x, y, reps=1)
