"""Precision mode on the host: the library's rounding of the stored values
to binary32 and bfloat16 equals the oracle's bit for bit, in every form's
storage order, including ties, subnormals, overflow and NaN."""
import numpy as np
import pytest

import paper_1203_2739_amd as spx
from synth import CSR, gen_c1


def special_csr():
    rng = np.random.default_rng(12)
    m = n = 40
    rp = np.arange(0, 4 * m + 1, 4, dtype=np.int64)
    cols = np.concatenate([np.sort(rng.choice(n, 4, replace=False)) for _ in range(m)]).astype(np.int32)
    special = [1 + 2.0**-8, 1 + 3 * 2.0**-8, -(1 + 2.0**-8), 1e-40, -1e-45, 3.5e38, -1e300, 1e300,
               np.nan, np.inf, -np.inf, 0.0, -0.0, 1 + 2.0**-24, 1 + 3 * 2.0**-24, 1.0 + 2.0**-25,
               65504.0, 2.0**-126, 2.0**-149, 1.00390625]
    v = np.concatenate([special, rng.standard_normal(4 * m - len(special)) * 10.0 ** rng.integers(-30, 30, 4 * m - len(special))])
    return CSR(m, n, rp, cols, v)


@pytest.mark.parametrize("which", ["special", "c1"])
def test_rounding_matches_oracle(orc, which):
    A = special_csr() if which == "special" else gen_c1()
    M = spx.from_csr(A, device=False)
    plans = [(spx.plan_plain(M), None)]
    if which == "c1":
        plans += [(spx.reorder_sb(M, 8, 0, 1)[0], "sb"), (spx.reorder_db(M, 8, 0, 1)[0], "db")]
    for P, form in plans:
        vals = A.vals if form is None else P.export_csr()[2]
        for prec in ("f32", "bf16"):
            spx.plan_add_lowp(P, prec)
            got = P.export_lowp(prec)
            f = orc.to_f32(vals)
            ref = f if prec == "f32" else orc.f32_to_bf16(f)
            assert np.array_equal(got.view(np.uint32 if prec == "f32" else np.uint16),
                                  ref.view(np.uint32 if prec == "f32" else np.uint16)), (form, prec)


def test_lowp_errors():
    A = gen_c1()
    M = spx.from_csr(A, device=False)
    P = spx.plan_plain(M)
    with pytest.raises(spx.SpxError):
        P.export_lowp("f32")          # not added yet
    with pytest.raises(spx.SpxError):
        spx.plan_add_lowp(P, 7)
    S = spx.split(M, 2, 0, 0)[0]
    with pytest.raises(spx.SpxError) as e:
        spx.plan_add_lowp(S, "f32")
    assert e.value.code == -5


def test_generator_dense_rows():
    """Members of the uneven batch with rows as long as the matrix is wide
    still get distinct, sorted columns in every row."""
    from synth import gen_c4_one
    for j in (4, 5, 6):
        A, k = gen_c4_one(j, base_seed=7001, n_hi=20_000)
        for i in range(A.m):
            c = A.colidx[A.rowptr[i]:A.rowptr[i + 1]]
            assert np.all(np.diff(c) > 0) and (c.size == 0 or (c[0] >= 0 and c[-1] < A.n))


@pytest.mark.parametrize("which", ["c1", "zipf", "family", "empty"])
def test_features_match_oracle(orc, which):
    """The library's selector features equal the oracle's: histograms and
    counted fractions exactly, sums within binary32 rounding."""
    from synth import gen_family, gen_uniform_zipf
    if which == "c1":
        A = gen_c1()
    elif which == "zipf":
        A = gen_uniform_zipf(5, 3000, 40000, 900)
    elif which == "family":
        A = gen_family("F3", 9, 5000)
    else:
        A = CSR(6, 4, np.array([0, 0, 2, 2, 3, 3, 3]), np.array([1, 3, 0], np.int32), np.ones(3))
    M = spx.from_csr(A, device=False)
    got = spx.features(M).astype(np.float64)
    ref = orc.features(A)
    assert np.array_equal(got[2:34], ref[2:34].astype(np.float32).astype(np.float64))
    assert np.allclose(got, ref.astype(np.float32), rtol=2e-7, atol=1e-30)


def test_selector_host_logic():
    """Regret, the best fixed choice, near-optimal label augmentation and the
    hierarchical coarsening of a bisection tree, on hand-made timings."""
    from paper_1203_2739_amd import selector
    T = np.array([[1.0, 2.0, 1.01] + [9.0] * 21,
                  [3.0, 1.5, 1.0] + [9.0] * 21])
    assert np.allclose(selector.regret(T, np.array([0, 0])), [0.0, 2.0])
    assert selector.best_fixed(T) == 2          # regrets 0.01 and 0: the best mean
    X, lab = selector.augment(np.eye(2, 40, dtype=np.float32), T, tol=0.02)
    assert sorted(lab[:2]) == [0, 2] and list(lab[2:]) == [2]
    assert selector.choice_name(23) == "split256" and selector.choice_name(6) == "sb8"
    assert [spx.choice_info(c)[0] for c in range(24)] == ["plain"] * 6 + ["sb"] * 6 + ["db"] * 6 + ["split"] * 6
    assert [spx.choice_info(c)[1] for c in range(6, 24)] == [8, 16, 32, 64, 128, 256] * 3
    with pytest.raises(spx.SpxError):
        spx.choice_info(24)
    # part p of a K = 256 tree lies in part p >> (8 - log2 K) of the tree cut at K
    parts = np.arange(256)
    assert np.array_equal(np.unique(parts >> 5), np.arange(8))
