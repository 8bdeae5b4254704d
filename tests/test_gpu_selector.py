"""Selector network kernels against the binary64 oracle (forward, loss,
gradient, Adam), training on the GPU, and the learned choice on measured
timings against the best single fixed choice."""
import numpy as np
import pytest

import paper_1203_2739_amd as spx
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


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
    acc = np.mean(selector.predict(theta, X.astype(np.float32)) == labels)
    assert curve[-1] < 0.5 * curve[0] and acc > 0.85, (curve[0], curve[-1], acc)


def test_selector_on_measured_timings():
    """Small end-to-end run: every choice timed on a handful of matrices of
    the four families; the network trained on them picks choices whose
    regret on those matrices is no worse than the best fixed choice's."""
    from paper_1203_2739_amd import selector
    from synth import gen_family
    mats = [gen_family(f, 100 + s, 2500 + 700 * s) for s in range(2) for f in ("F1", "F2", "F3", "F4")]
    T = np.stack([selector.measure(A, seed=i, warmup=1, steps=5)[0] for i, A in enumerate(mats)])
    assert np.all(T > 0)
    F = selector.feature_matrix(mats)
    norm = selector.Normalizer(F)
    labels = T.argmin(axis=1)
    theta, curve = selector.train(norm(F), labels, epochs=300, batch=16, lr=3e-3)
    chosen = selector.predict(theta, norm(F))
    fixed = selector.best_fixed(T)
    r_net = selector.regret(T, chosen).mean()
    r_fix = selector.regret(T, np.full(len(mats), fixed)).mean()
    print(f"mean regret: network {r_net:.3f}, best fixed choice {selector.choice_name(fixed)} {r_fix:.3f}")
    assert r_net <= r_fix + 1e-9
