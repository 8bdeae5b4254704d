"""Helpers shared by the GPU parity tests."""
import numpy as np

TOL = 1e-12  # per-entry bound: |y - y_ref| <= TOL * sum_j |a_ij x_j|


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_close_rowwise(y, ref, bound, what=""):
    """The parity rule for binary64 products: per-entry error at most
    TOL * sum_j |a_ij x_j|; rows with a zero bound must be exactly zero."""
    y = np.asarray(y)
    err = np.abs(y - ref)
    lim = TOL * bound
    zero = bound == 0
    assert np.all(y[zero] == 0.0), f"{what}: nonzero result on an all-zero row"
    bad = np.flatnonzero(err > lim)
    assert bad.size == 0, (f"{what}: {bad.size} rows over the bound; worst "
                           f"{(err[bad] / np.maximum(bound[bad], 1e-300)).max():.3e} at row {bad[0]}")


def integer_problem(A, seed):
    """Replace values and x by small integers: every summation order is exact."""
    rng = np.random.default_rng(seed)
    v = rng.integers(-8, 9, size=A.nnz).astype(np.float64)
    v[v == 0] = 3.0
    x = rng.integers(-8, 9, size=A.n).astype(np.float64)
    from synth import CSR
    return CSR(A.m, A.n, A.rowptr, A.colidx, v), x
