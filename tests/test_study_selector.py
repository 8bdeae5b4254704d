"""The learned choice on measured timings, evaluated on matrices it never saw.

A statistical end-to-end study rather than a parity check, so it sits in a
file of its own that is collected after the parity tests."""
import numpy as np
import pytest

import paper_1203_2739_amd as spx

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.timeout(1200)
def test_selector_gains_on_held_out_matrices():
    """48 matrices of the four families (n from 9,000 to 45,000), every
    choice timed by the library (spx_select_exhaustive).  Six-fold
    cross-validation: the network is trained on 40 matrices and chooses,
    through spx_select, for the 8 others; every matrix is held out once.
    Pooled over the 48 held-out choices, its mean regret must not exceed
    that of plain CSR, nor that of the best fixed choice (picked on each
    fold's training matrices) by more than 0.05.

    Eight held-out matrices alone are too few: replaying the protocol on
    the timings of 600 measured matrices of the same families, one split of
    16 + 8 failed "at most best fixed + 0.03 and at most plain" in about a
    third of the draws.  The pooled six-fold form failed those bounds in 2
    of 160 draws and the bounds asserted here in none (mean regret: network
    0.068, best fixed 0.091, plain 0.127; the network beat plain CSR in
    every draw)."""
    from paper_1203_2739_amd import selector
    from synth import gen_family
    fams = ("F1", "F2", "F3", "F4")
    sizes = [12000, 20000, 30000, 45000, 16000, 26000, 9000, 36000, 14000, 24000, 18000, 40000]
    mats = [gen_family(f, 300 + 10 * s + k, n) for s, n in enumerate(sizes) for k, f in enumerate(fams)]
    T = np.stack([selector.measure(A, seed=i, reps=5)[0] for i, A in enumerate(mats)])
    assert np.all(T > 0)
    F = selector.feature_matrix(mats)
    N = len(mats)
    folds = np.array_split(np.random.default_rng(0).permutation(N), 6)
    r_net, r_fix, r_plain = [], [], []
    for k, te in enumerate(folds):
        tr = np.setdiff1d(np.arange(N), te)
        norm = selector.Normalizer(F[tr])
        theta, settings, _ = selector.fit(F[tr], T[tr], norm, epochs=200, check_every=40, lrs=(3e-3,))
        chosen = selector.predict(theta, F[te], norm)
        if k == 0:
            # the library's selection from the matrix itself agrees
            lib = [spx.select(spx.from_csr(mats[i], device=False), theta, norm.mu, norm.sd)[0] for i in te]
            assert np.array_equal(np.array(lib), chosen)
        fixed = selector.best_fixed(T[tr])
        r_net.append(selector.regret(T[te], chosen))
        r_fix.append(selector.regret(T[te], np.full(te.size, fixed)))
        r_plain.append(selector.regret(T[te], np.zeros(te.size, int)))
        print(f"fold {k}: network {r_net[-1].mean():.3f}, best fixed {selector.choice_name(fixed)} "
              f"{r_fix[-1].mean():.3f}, plain {r_plain[-1].mean():.3f}; settings {settings}", flush=True)
    rn, rf, rp = (float(np.concatenate(r).mean()) for r in (r_net, r_fix, r_plain))
    print(f"held-out mean regret over {N} matrices: network {rn:.3f}, best fixed {rf:.3f}, plain {rp:.3f}")
    assert rn <= rf + 0.05 and rn <= rp, (rn, rf, rp)
