"""Precision mode on the GPU through the C interface: binary32 and bfloat16
products against the oracle (bit-exact on integer data, within the binary32
summation bound otherwise), and the binary64-refined CG solve."""
import numpy as np
import pytest

import paper_1203_2739_amd as spx
from gpu_util import dev, host, integer_problem
from synth import CSR, gen_c3_spd, gen_uniform_zipf, gen_vectors

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def lowp_y(P, prec, x32, m):
    import torch
    yd = torch.full((max(m, 1),), np.nan, dtype=torch.float32, device="cuda")
    spx.spmv_lowp(P, prec, dev(x32.astype(np.float32)), yd)
    return host(yd)[:m]


def oracle_lowp(orc, A, vals, x32, prec):
    f = orc.to_f32(vals)
    if prec == "f32":
        return orc.spmv_lowp(A, f, x32), f.astype(np.float64)
    h = orc.f32_to_bf16(f)
    return orc.spmv_lowp(A, None, x32, vals16=h), orc.bf16_bits_to_f32(h).astype(np.float64)


def plans(A, form):
    M = spx.from_csr(A)
    if form == "plain":
        return spx.plan_plain(M), A, np.arange(A.n)
    P, rp, cp, _ = {"sb": spx.reorder_sb, "db": spx.reorder_db}[form](M, 8, 0, 2)
    from oracle import permute_csr
    r, c, v = permute_csr(A, rp, cp)
    return P, CSR(A.m, A.n, r, c.astype(np.int32), v), cp


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("form", ["plain", "sb", "db"])
@pytest.mark.parametrize("tune", [None, dict(wg_size=64), dict(wg_size=512), dict(reduce_iters=2, wg_size=256),
                                  dict(wg_size=512, scan_reduce=1), dict(wg_size=128, scan_reduce=1)])
def test_lowp_integer_exact(orc, prec, form, tune):
    A0 = gen_uniform_zipf(51, 20_000, 300_000, 4000, diagonal=True)
    A, x = integer_problem(A0, 13)
    P, Ah, cp = plans(A, form)
    if tune:
        spx.plan_retune(P, tune)
    spx.plan_add_lowp(P, prec)
    xh = x[cp].astype(np.float32)
    y = lowp_y(P, prec, xh, A.m)
    ref, _ = oracle_lowp(orc, Ah, Ah.vals, xh, prec)
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("tune", [None, dict(wg_size=1024, scan_reduce=1)])
def test_lowp_rounding_bound(orc, prec, tune):
    A = gen_uniform_zipf(52, 30_000, 500_000, 5000, diagonal=True)
    x = gen_vectors(120, A.n)[0].astype(np.float32)
    P, Ah, cp = plans(A, "plain")
    if tune:
        spx.plan_retune(P, tune)
    spx.plan_add_lowp(P, prec)
    y = lowp_y(P, prec, x, A.m).astype(np.float64)
    ref, vq = oracle_lowp(orc, Ah, Ah.vals, x, prec)
    # both sides sum binary32 products of the same rounded values: each is
    # within m_i u sum |a_q x| of the exact sum (u = 2^-24)
    absq = orc.abs_rowsum(CSR(A.m, A.n, A.rowptr, A.colidx, vq), x.astype(np.float64))
    deg = np.diff(A.rowptr)
    lim = 2.0 * (deg + 2) * U32 * absq
    assert np.all(np.abs(y - ref.astype(np.float64)) <= lim)
    # against the binary64 product of the unrounded values: value rounding
    # (unit roundoff 2^-24 for binary32, 2^-8 more for bfloat16, whose
    # significand has 8 bits) plus the
    # binary32 summation
    y64 = orc.spmv(A, x.astype(np.float64))
    abs64 = orc.abs_rowsum(A, x.astype(np.float64))
    uval = U32 if prec == "f32" else 2.0 ** -8 + U32
    assert np.all(np.abs(y - y64) <= (uval + 2.0 * (deg + 2) * U32) * abs64 * (1 + 1e-6))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_cg_ir_solves_spd(orc, prec):
    """C3-style SPD system at n = 20,000 from b = A 1: the refined solve
    reaches relative residual 1e-10 (recomputed by the oracle in binary64)
    and the solution is close to ones."""
    import torch
    A = gen_c3_spd(seed=3, n=20_000)
    b = orc.spmv(A, np.ones(A.n))
    M = spx.from_csr(A)
    P = spx.plan_plain(M)
    if prec != "f64":
        spx.plan_add_lowp(P, prec)
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st = spx.cg_ir(P, prec, dev(b), xd, tol=1e-10, inner_tol=1e-3 if prec != "bf16" else 1e-2,
                   max_outer=60, max_inner=2000)
    assert st["converged"], st
    x = host(xd)
    res = np.linalg.norm(b - orc.spmv(A, x))
    assert res / np.linalg.norm(b) <= 2e-10, res
    # A is strictly diagonally dominant with margin 1, so its smallest
    # eigenvalue is at least 1 (Gershgorin) and ||x - 1|| <= ||b - A x||
    assert np.linalg.norm(x - 1.0) <= res * (1 + 1e-6)
    if prec != "f64":
        assert st["outer"] >= 2  # binary32 or bfloat16 alone cannot reach 1e-10


def test_cg_ir_not_converged_reports():
    import torch
    A = gen_c3_spd(seed=4, n=5_000)
    M = spx.from_csr(A)
    P = spx.plan_plain(M)
    spx.plan_add_lowp(P, "bf16")
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    xd = torch.zeros_like(b)
    st = spx.cg_ir(P, "bf16", b, xd, tol=1e-14, inner_tol=1e-2, max_outer=1, max_inner=3)
    assert not st["converged"] and st["outer"] == 1 and st["inner"] <= 3


def test_cg_ir_rejects_reordered_plans():
    import torch
    A = gen_c3_spd(seed=5, n=3_000)
    M = spx.from_csr(A)
    P = spx.reorder_sb(M, 4, 0, 0)[0]
    spx.plan_add_lowp(P, "f32")
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(spx.SpxError) as e:
        spx.cg_ir(P, "f32", b, torch.zeros_like(b))
    assert e.value.code == -5


def test_cg_schedules(orc):
    """Binary64 CG runs under any schedule, gather-sorted blocks included;
    the binary32 refined solve refuses a schedule the precision mode does
    not run."""
    import torch
    A = gen_c3_spd(seed=5, n=8_000)
    b = orc.spmv(A, np.ones(A.n))
    M = spx.from_csr(A)
    P = spx.plan_plain(M, tune=dict(wg_size=512, sort_gathers=1))
    spx.plan_add_lowp(P, "f32")
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st = spx.cg_ir(P, "f64", dev(b), xd, tol=1e-10, max_inner=2000)
    assert st["converged"]
    assert np.linalg.norm(b - orc.spmv(A, host(xd))) <= 2e-10 * np.linalg.norm(b)
    xd.zero_()
    with pytest.raises(spx.SpxError):
        spx.cg_ir(P, "f32", dev(b), xd, tol=1e-10)
