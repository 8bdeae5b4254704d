"""Python binding of libspx (argument marshalling only).

Every computation runs in the HIP library ``libspx.so`` built from
``csrc/``; this module converts numpy arrays and torch tensors to pointers and
raises :class:`SpxError` for a failed call.  Importing works without a GPU;
loading the library fails loudly if it has not been built.

Function names follow the C interface in ``include/spx.h`` without the
``spx_`` prefix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspx.so")

FORM_PLAIN, FORM_SB, FORM_DB, FORM_SPLIT = 0, 1, 2, 3
FORM_NAMES = {0: "plain", 1: "sb", 2: "db", 3: "split", 4: "order"}

_lib = None


class SpxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spx error {code}: {msg}")
        self.code = code


class Tune(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("nnz_per_block", ctypes.c_int32),
                ("blocks_per_tile", ctypes.c_int32), ("window_entries", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("reduce_iters", ctypes.c_int32),
                ("tiles_per_group", ctypes.c_int32), ("wave_blocks", ctypes.c_int32),
                ("pipeline", ctypes.c_int32), ("scan_reduce", ctypes.c_int32), ("sort_gathers", ctypes.c_int32),
                ("compact_index", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("K", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("nleaves", ctypes.c_int32),
                ("nblocks", ctypes.c_int32), ("ntiles", ctypes.c_int32), ("nslots", ctypes.c_int32),
                ("row_border_begin", ctypes.c_int32), ("row_empty_begin", ctypes.c_int32),
                ("col_border_begin", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("nnz_per_block", ctypes.c_int32), ("blocks_per_tile", ctypes.c_int32),
                ("window_entries", ctypes.c_int32), ("sum_lambda_col", ctypes.c_int64),
                ("sum_lambda_row", ctypes.c_int64), ("border_row_nnz", ctypes.c_int64),
                ("cut_connectivity", ctypes.c_int64), ("bytes_matrix", ctypes.c_int64),
                ("bytes_window", ctypes.c_int64), ("window_nnz", ctypes.c_int64),
                ("partition_seconds", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("reduce_iters", ctypes.c_int32), ("nlong_rows", ctypes.c_int32),
                ("tiles_per_group", ctypes.c_int32), ("wave_blocks", ctypes.c_int32),
                ("pipeline", ctypes.c_int32), ("scan_reduce", ctypes.c_int32), ("sort_gathers", ctypes.c_int32),
                ("compact_index", ctypes.c_int32), ("nnz_compact", ctypes.c_int64)]


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

_SIGS = {
    "spx_last_error": ([], ctypes.c_char_p),
    "spx_version": ([], ctypes.c_char_p),
    "spx_set_num_threads": ([_I32], _I32),
    "spx_csr_upload": ([_I32, _I32, _I64, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_csr_create_host": ([_I32, _I32, _I64, _VP, _VP, _VP, _VP], _I32),
    "spx_mat_destroy": ([_VP], None),
    "spx_plan_plain": ([_VP, _VP, _VP], _I32),
    "spx_reorder_sb": ([_VP, _I32, _I64, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_reorder_db": ([_VP, _I32, _I64, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_split": ([_VP, _I32, _I64, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_split_ex": ([_VP, _I32, _I64, ctypes.c_uint64, _I32, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_reorder_rn": ([_VP, _I32, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_plan_retune": ([_VP, _VP], _I32),
    "spx_plan_autotune": ([_VP, _I32, _VP, _VP, _I32, _VP, _VP, _VP, _VP], _I32),
    "spx_autotune_candidate": ([_I32, _VP], _I32),
    "spx_choice_info": ([_I32, _VP, _VP, _VP], _I32),
    "spx_mlp_loss_grad_noalloc": ([_VP, _VP, _VP, _I32, _VP, _VP, _VP], _I32),
    "spx_order_bfs": ([_VP, _VP, _VP], _I32),
    "spx_order_rcm": ([_VP, _VP, _VP], _I32),
    "spx_plan_from_perm": ([_VP, _VP, _VP, _VP, _VP], _I32),
    "spx_select": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_select_features": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_plan_for_choice": ([_VP, _I32, ctypes.c_uint64, _VP, _VP, _VP], _I32),
    "spx_select_exhaustive": ([_VP, _VP, _VP, _I32, ctypes.c_uint64, _VP, _VP, _VP, _VP], _I32),
    "spx_partition_tree": ([_VP, _I32, ctypes.c_uint64, _VP, _VP], _I32),
    "spx_select_exhaustive_trees": ([_VP, _VP, _VP, _VP, _VP, _VP, _I32, _VP, _VP, _VP], _I32),
    "spx_plan_destroy": ([_VP], None),
    "spx_plan_info_get": ([_VP, _VP], _I32),
    "spx_spmv": ([_VP, _VP, _VP, _VP], _I32),
    "spx_spmv_split": ([_VP, _VP, _VP, _I32, _VP], _I32),
    "spx_split_prepare_y": ([_VP, _VP, _VP], _I32),
    "spx_permute_x": ([_VP, _VP, _VP, _VP], _I32),
    "spx_unpermute_y": ([_VP, _VP, _VP, _VP], _I32),
    "spx_plan_export_csr": ([_VP, _VP, _VP, _VP], _I32),
    "spx_plan_export_split": ([_VP, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_plan_export_parts": ([_VP, _VP, _VP], _I32),
    "spx_plan_export_perm": ([_VP, _VP, _VP], _I32),
    "spx_plan_export_sched": ([_VP, _VP, _VP], _I32),
    "spx_plan_export_gather_order": ([_VP, _VP, _VP, _VP, _VP], _I32),
    "spx_plan_export_compact": ([_VP, _VP, _VP], _I32),
    "spx_stream_sink_len": ([_I64], _I64),
    "spx_stream_read": ([_VP, _I64, _VP, _VP], _I32),
    "spx_stream_copy": ([_VP, _VP, _I64, _VP], _I32),
    "spx_plan_add_lowp": ([_VP, _I32], _I32),
    "spx_plan_export_lowp": ([_VP, _I32, _VP], _I32),
    "spx_spmv_lowp": ([_VP, _I32, _VP, _VP, _VP], _I32),
    "spx_cg_ir": ([_VP, _I32, _VP, _VP, ctypes.c_double, ctypes.c_double, _I32, _I32, _VP, _VP], _I32),
    "spx_batch_create": ([_I32, _VP, _VP, _VP], _I32),
    "spx_batch_destroy": ([_VP], None),
    "spx_batch_bind": ([_VP, _VP, _VP, _VP, _VP], _I32),
    "spx_batch_run": ([_VP, _VP], _I32),
    "spx_batch_capture": ([_VP], _I32),
    "spx_batch_replay": ([_VP, _VP], _I32),
    "spx_batch_autotune": ([_VP, _I32, _VP, _VP], _I32),
    "spx_batch_configure": ([_VP, _VP], _I32),
    "spx_batch_info": ([_VP, _VP, _VP, _VP], _I32),
    "spx_spmv_batched": ([_I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_features": ([_VP, _VP], _I32),
    "spx_plan_from_parts": ([_VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP], _I32),
    "spx_mlp_forward": ([_VP, _VP, _I32, _VP, _VP], _I32),
    "spx_mlp_loss_grad": ([_VP, _VP, _VP, _I32, _VP, _VP, _VP], _I32),
    "spx_mlp_adam": ([_VP, _VP, _VP, _VP, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, _VP], _I32),
}

NFEATURES, NCHOICES, MLP_PARAMS = 40, 24, 8344


class BatchConfig(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("span_div", ctypes.c_int32),
                ("reduce_iters", ctypes.c_int32), ("ms", ctypes.c_float)]

PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2
_PREC = {"f64": PREC_F64, "f32": PREC_F32, "bf16": PREC_BF16}


class CgStats(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


def declared_symbols():
    """Names of the functions declared in include/*.h."""
    import re
    inc = os.path.join(os.path.dirname(HERE), "include")
    names = set()
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            names |= set(re.findall(r"\b(spx_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def _device_first():
    """PyTorch for ROCm carries its own HIP runtime beside the one libspx
    links; the device must be opened by PyTorch's runtime before libspx makes
    its first HIP call, or that call finds no device."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()
        torch.empty(1, device="cuda")


def lib():
    """Load libspx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1203_2739_amd.build.build()")
        _device_first()
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _extra_signatures(L)
        _lib = L
    return _lib


_EXTRA_SIGS = {}


def _extra_signatures(L):
    for name, (args, res) in _EXTRA_SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


def _check(rc):
    if rc != 0:
        raise SpxError(rc, lib().spx_last_error().decode())


def last_error():
    return lib().spx_last_error().decode()


def version():
    return lib().spx_version().decode()


def set_num_threads(n):
    _check(lib().spx_set_num_threads(int(n)))


def _host_i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _host_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _hp(a):
    return a.ctypes.data_as(_VP) if a is not None else None


def _dev(t, dtype=None, numel=None):
    """Device pointer of a torch tensor (or an integer address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return _VP(t)
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} elements, needs {numel}")
    return _VP(t.data_ptr())


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return _VP(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return _VP(stream)
    return _VP(stream.cuda_stream)


def make_tune(**kw):
    t = Tune()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


class Mat:
    """A CSR matrix handle (host copy, and a device copy after upload)."""

    def __init__(self, handle, m, n, nnz, on_device):
        self._h = _VP(handle)
        self.m, self.n, self.nnz, self.on_device = m, n, nnz, on_device

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.spx_mat_destroy(self._h)
            self._h = None


def _csr_args(rowptr, colidx, vals):
    rowptr = _host_i32(rowptr)
    colidx = _host_i32(colidx)
    vals = _host_f64(vals)
    if colidx.size != vals.size:
        raise ValueError("colidx and vals differ in length")
    return rowptr, colidx, vals


def csr_upload(m, n, rowptr, colidx, vals, stream=None) -> Mat:
    """Validate a CSR matrix and copy it to the current device."""
    rp, ci, v = _csr_args(rowptr, colidx, vals)
    if rp.size != int(m) + 1:
        raise ValueError("rowptr must have m + 1 entries")
    h = _VP()
    _check(lib().spx_csr_upload(int(m), int(n), int(ci.size), _hp(rp), _hp(ci),
                                _hp(v), _stream(stream), ctypes.byref(h)))
    return Mat(h.value, int(m), int(n), int(ci.size), True)


def csr_create_host(m, n, rowptr, colidx, vals) -> Mat:
    """Validate a CSR matrix and keep a host copy only."""
    rp, ci, v = _csr_args(rowptr, colidx, vals)
    if rp.size != int(m) + 1:
        raise ValueError("rowptr must have m + 1 entries")
    h = _VP()
    _check(lib().spx_csr_create_host(int(m), int(n), int(ci.size), _hp(rp),
                                     _hp(ci), _hp(v), ctypes.byref(h)))
    return Mat(h.value, int(m), int(n), int(ci.size), False)


def from_csr(A, device=True, stream=None) -> Mat:
    """Matrix handle from any object with m, n, rowptr, colidx, vals."""
    if device:
        return csr_upload(A.m, A.n, A.rowptr, A.colidx, A.vals, stream)
    return csr_create_host(A.m, A.n, A.rowptr, A.colidx, A.vals)


class Plan:
    """A matrix in plain, SB, DB or split form."""

    def __init__(self, handle, mat):
        self._h = _VP(handle)
        self.mat_dims = (mat.m, mat.n, mat.nnz)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.spx_plan_destroy(self._h)
            self._h = None

    def info(self) -> dict:
        i = PlanInfo()
        _check(lib().spx_plan_info_get(self._h, ctypes.byref(i)))
        d = {f: getattr(i, f) for f, _ in PlanInfo._fields_}
        d["form_name"] = FORM_NAMES[d["form"]]
        return d

    def export_csr(self):
        m, n, nnz = self.mat_dims
        rp = np.empty(m + 1, np.int32)
        ci = np.empty(max(nnz, 1), np.int32)
        v = np.empty(max(nnz, 1), np.float64)
        _check(lib().spx_plan_export_csr(self._h, _hp(rp), _hp(ci), _hp(v)))
        return rp, ci[:nnz], v[:nnz]

    def export_split(self):
        inf = self.info()
        L, S, nnz = inf["nleaves"], inf["nslots"], inf["nnz"]
        lsp = np.empty(L + 1, np.int32)
        sr = np.empty(max(S, 1), np.int32)
        sp = np.empty(S + 1, np.int32)
        ci = np.empty(max(nnz, 1), np.int32)
        v = np.empty(max(nnz, 1), np.float64)
        _check(lib().spx_plan_export_split(self._h, _hp(lsp), _hp(sr), _hp(sp), _hp(ci), _hp(v)))
        return dict(leaf_slot_ptr=lsp, slot_row=sr[:S], slot_ptr=sp, colidx=ci[:nnz], vals=v[:nnz])

    def export_lowp(self, precision):
        """Rounded values: float32 array (f32) or uint16 bfloat16 bit patterns (bf16)."""
        prec = _PREC.get(precision, precision)
        nnz = self.info()["nnz"]
        out = np.empty(max(nnz, 1), np.float32 if prec == PREC_F32 else np.uint16)
        _check(lib().spx_plan_export_lowp(self._h, int(prec), _hp(out)))
        return out[:nnz]

    def export_parts(self):
        inf = self.info()
        size = inf["nnz"] if inf["form"] == FORM_SPLIT else inf["m"]
        a = np.empty(max(size, 1), np.int32)
        b = np.empty(max(size, 1), np.int32)
        _check(lib().spx_plan_export_parts(self._h, _hp(a), _hp(b)))
        return a[:size], b[:size]

    def export_perm(self):
        m, n, _ = self.mat_dims
        rp = np.empty(max(m, 1), np.int32)
        cp = np.empty(max(n, 1), np.int32)
        _check(lib().spx_plan_export_perm(self._h, _hp(rp), _hp(cp)))
        return rp[:m], cp[:n]

    def export_sched(self):
        """(blk_desc[nblocks, 4], tiles[ntiles, 4])."""
        inf = self.info()
        bd = np.empty(max(4 * inf["nblocks"], 1), np.int32)
        tl = np.empty(max(4 * inf["ntiles"], 1), np.int32)
        _check(lib().spx_plan_export_sched(self._h, _hp(bd), _hp(tl)))
        return bd[:4 * inf["nblocks"]].reshape(-1, 4), tl[:4 * inf["ntiles"]].reshape(-1, 4)

    def export_compact(self):
        """(colidx16 uint16[nnz], cbase int32[nblocks]) of a compact_index plan."""
        inf = self.info()
        c = np.empty(max(inf["nnz"], 1), np.uint16)
        b = np.empty(max(inf["nblocks"], 1), np.int32)
        _check(lib().spx_plan_export_compact(self._h, _hp(c), _hp(b)))
        return c[:inf["nnz"]], b[:inf["nblocks"]]

    def export_gather_order(self):
        """(ofs[nblocks], colidx uint32[len], vals[len]) of the gather-sorted copy."""
        n = ctypes.c_int64()
        _check(lib().spx_plan_export_gather_order(self._h, ctypes.byref(n), None, None, None))
        nb = self.info()["nblocks"]
        o = np.empty(max(nb, 1), np.int32)
        c = np.empty(max(n.value, 1), np.uint32)
        v = np.empty(max(n.value, 1), np.float64)
        _check(lib().spx_plan_export_gather_order(self._h, None, _hp(o), _hp(c), _hp(v)))
        return o[:nb], c[:n.value], v[:n.value]


def _tune_ptr(tune):
    if tune is None:
        return None
    if isinstance(tune, dict):
        tune = make_tune(**tune)
    return ctypes.byref(tune)


def plan_plain(A: Mat, tune=None) -> Plan:
    h = _VP()
    _check(lib().spx_plan_plain(A.handle, _tune_ptr(tune), ctypes.byref(h)))
    return Plan(h.value, A)


def _reorder(fn, A, K, window_bytes, seed, tune, part_len):
    rp = np.empty(max(A.m, 1), np.int32)
    cp = np.empty(max(A.n, 1), np.int32)
    pp = np.empty(max(part_len, 1), np.int32)
    h = _VP()
    _check(fn(A.handle, int(K), int(window_bytes), ctypes.c_uint64(int(seed)), _hp(rp), _hp(cp),
              _hp(pp), _tune_ptr(tune), ctypes.byref(h)))
    return Plan(h.value, A), rp[:A.m], cp[:A.n], pp[:part_len]


def reorder_sb(A: Mat, K, window_bytes=0, seed=0, tune=None):
    """SB form (Eq. 1): returns (plan, row_perm, col_perm, part_ptr[K+1])."""
    return _reorder(lib().spx_reorder_sb, A, K, window_bytes, seed, tune, K + 1)


def reorder_db(A: Mat, K, window_bytes=0, seed=0, tune=None):
    """DB form (Eq. 5): returns (plan, row_perm, col_perm, part_ptr[K+2])."""
    return _reorder(lib().spx_reorder_db, A, K, window_bytes, seed, tune, K + 2)


def reorder_rn(A: Mat, K, window_bytes=0, seed=0, tune=None):
    """sHP_RN (row-net model, Section 5.1) as a DB-shaped plan: returns
    (plan, row_perm, col_perm, part_ptr[K+2]).  window_bytes is ignored."""
    fn = lambda a, k, wb, sd, *rest: lib().spx_reorder_rn(a, k, sd, *rest)  # noqa: E731
    return _reorder(fn, A, K, window_bytes, seed, tune, K + 2)


def split(A: Mat, K, window_bytes=0, seed=0, tune=None, row_net_cost=None):
    """Splitting (Section 4): returns (plan, row_perm, col_perm, nz_part[nnz]).
    row_net_cost: cost of a row net relative to a column net (None: the
    library's default, 32; 1 is Corollary 4's objective as written)."""
    if row_net_cost is None:
        return _reorder(lib().spx_split, A, K, window_bytes, seed, tune, A.nnz)
    fn = lambda *a: lib().spx_split_ex(a[0], a[1], a[2], a[3], int(row_net_cost), *a[4:])  # noqa: E731
    return _reorder(fn, A, K, window_bytes, seed, tune, A.nnz)


def plan_retune(P: Plan, tune=None):
    _check(lib().spx_plan_retune(P.handle, _tune_ptr(tune)))


_TUNE_FIELDS = ("wg_size", "nnz_per_block", "blocks_per_tile", "window_entries", "xcd_remap", "reduce_iters",
                "tiles_per_group", "wave_blocks", "pipeline", "scan_reduce", "sort_gathers", "compact_index")


def autotune_candidates():
    """The library's candidate schedules, as dicts, in the order tried."""
    n = int(lib().spx_autotune_candidate(-1, None))
    out = []
    for i in range(n):
        t = make_tune()
        lib().spx_autotune_candidate(i, ctypes.byref(t))
        out.append({f: getattr(t, f) for f in _TUNE_FIELDS if getattr(t, f)})
    return out


def plan_autotune(P: Plan, x, y, reps=10, precision="f64", stream=None, report=False):
    """Time the library's candidate schedules on x -> y and keep the fastest
    (binary64 products, or the "f32"/"bf16" products on binary32 vectors).
    Returns (schedule dict, milliseconds per product), plus with report=True
    the milliseconds of every candidate (-1: not run)."""
    import torch
    m, n, _ = P.mat_dims
    prec = {"f64": 0}.get(precision, _PREC.get(precision, precision))
    dt = torch.float64 if prec == 0 else torch.float32
    t = make_tune()
    ms = ctypes.c_float()
    nc = int(lib().spx_autotune_candidate(-1, None))
    cm = np.empty(max(nc, 1), np.float32)
    _check(lib().spx_plan_autotune(P.handle, int(prec), _dev(x, dt, n), _dev(y, dt, m), int(reps),
                                   ctypes.byref(t), ctypes.byref(ms), _hp(cm), _stream(stream)))
    chosen = {f: getattr(t, f) for f in _TUNE_FIELDS}
    return (chosen, ms.value, cm[:nc].tolist()) if report else (chosen, ms.value)


def spmv(P: Plan, x, y, stream=None):
    """y <- A x (reordered space for SB/DB/split plans)."""
    import torch
    m, n, _ = P.mat_dims
    _check(lib().spx_spmv(P.handle, _dev(x, torch.float64, n), _dev(y, torch.float64, m),
                          _stream(stream)))


def spmv_split(P: Plan, x, y, accumulate=0, stream=None):
    """y <- y + A^k x for k = 1..K.  accumulate: 0 = y starts at zero,
    1 = add to y, 2 = y starts at zero and its shared rows are already zero."""
    import torch
    m, n, _ = P.mat_dims
    _check(lib().spx_spmv_split(P.handle, _dev(x, torch.float64, n), _dev(y, torch.float64, m),
                                int(accumulate), _stream(stream)))


def split_prepare_y(P: Plan, y, stream=None):
    """Zero the rows of y shared by several leaves of a split plan."""
    import torch
    m, n, _ = P.mat_dims
    _check(lib().spx_split_prepare_y(P.handle, _dev(y, torch.float64, m), _stream(stream)))


def permute_x(P: Plan, x, x_hat, stream=None):
    import torch
    m, n, _ = P.mat_dims
    _check(lib().spx_permute_x(P.handle, _dev(x, torch.float64, n), _dev(x_hat, torch.float64, n),
                               _stream(stream)))


def unpermute_y(P: Plan, y_hat, y, stream=None):
    import torch
    m, n, _ = P.mat_dims
    _check(lib().spx_unpermute_y(P.handle, _dev(y_hat, torch.float64, m), _dev(y, torch.float64, m),
                                 _stream(stream)))


def stream_sink_len(nbytes):
    return int(lib().spx_stream_sink_len(int(nbytes)))


def stream_read(src, nbytes, sink, stream=None):
    _check(lib().spx_stream_read(_dev(src), int(nbytes), _dev(sink), _stream(stream)))


def stream_copy(src, dst, nbytes, stream=None):
    _check(lib().spx_stream_copy(_dev(src), _dev(dst), int(nbytes), _stream(stream)))


# ---------------------------------------------------------------- precision mode

def plan_add_lowp(P: Plan, precision):
    """Store the plan's values rounded to binary32 ("f32") or bfloat16 ("bf16")."""
    _check(lib().spx_plan_add_lowp(P.handle, int(_PREC.get(precision, precision))))


def spmv_lowp(P: Plan, precision, x, y, stream=None):
    """y <- A_low x with binary32 device vectors (binary32 accumulation)."""
    import torch
    m, n, _ = P.mat_dims
    _check(lib().spx_spmv_lowp(P.handle, int(_PREC.get(precision, precision)), _dev(x, torch.float32, n),
                               _dev(y, torch.float32, m), _stream(stream)))


def cg_ir(P: Plan, precision, b, x, tol=1e-10, inner_tol=1e-3, max_outer=50, max_inner=1000,
          stream=None):
    """Solve A x = b by CG in the given precision inside binary64 iterative
    refinement.  Returns a dict of statistics with "converged"."""
    import torch
    m, n, _ = P.mat_dims
    st = CgStats()
    rc = lib().spx_cg_ir(P.handle, int(_PREC.get(precision, precision)), _dev(b, torch.float64, n),
                         _dev(x, torch.float64, n), float(tol), float(inner_tol), int(max_outer),
                         int(max_inner), ctypes.byref(st), _stream(stream))
    if rc not in (0, -4):
        _check(rc)
    return {"outer": st.outer, "inner": st.inner, "rel_residual": st.rel_residual,
            "seconds": st.seconds, "converged": rc == 0}


# ---------------------------------------------------------------- batched products

def _vec_table(tensors, ks, rows):
    """Pointer and leading-dimension tables of row-major (rows, k) tensors.

    ``rows[i]`` is the number of rows the i-th matrix reads (X: its n) or
    writes (Y: its m); a tensor with fewer rows, or with rows closer than k
    entries apart, is refused before any pointer reaches the library, which
    cannot check raw device pointers."""
    import torch
    n = len(tensors)
    if len(ks) != n or len(rows) != n:
        raise ValueError("one tensor per matrix is needed")
    ptrs = (ctypes.c_void_p * max(n, 1))()
    lds = (ctypes.c_int64 * max(n, 1))()
    for i, (t, k, r) in enumerate(zip(tensors, ks, rows)):
        if t.dtype != torch.float64:
            raise ValueError("batched vectors must be float64 device tensors")
        if t.dim() == 1:
            if k != 1 or t.stride(0) != 1:
                raise ValueError("a 1-D tensor needs k = 1 and unit stride")
            if t.shape[0] < r:
                raise ValueError(f"tensor {i} has {t.shape[0]} entries, the matrix needs {r}")
            lds[i] = 1
        elif t.dim() == 2:
            if t.shape[1] != k or t.stride(1) != 1:
                raise ValueError("expected a (rows, k) tensor with unit column stride")
            if t.shape[0] < r:
                raise ValueError(f"tensor {i} has {t.shape[0]} rows, the matrix needs {r}")
            if t.shape[0] > 1 and t.stride(0) < k:
                raise ValueError(f"tensor {i}: rows overlap (leading dimension {t.stride(0)} < k = {k})")
            lds[i] = t.stride(0) if t.shape[0] > 1 else k
        else:
            raise ValueError("batched vectors must be 1-D or 2-D tensors")
        if not t.is_cuda:
            raise ValueError("batched vectors must be float64 device tensors")
        ptrs[i] = t.data_ptr()
    return ptrs, lds


class Batch:
    """Y_i = A_i X_i for many plans in one persistent launch."""

    def __init__(self, plans, nrhs):
        self.plans = list(plans)  # kept alive: the batch uses their device arrays
        self.nrhs = [int(k) for k in nrhs]
        arr = (ctypes.c_void_p * max(len(self.plans), 1))(*[p.handle.value for p in self.plans])
        ks = np.ascontiguousarray(self.nrhs, dtype=np.int32)
        h = _VP()
        _check(lib().spx_batch_create(len(self.plans), arr, _hp(ks), ctypes.byref(h)))
        self._h = h
        self._bound = None

    def __del__(self):
        try:
            if self._h:
                lib().spx_batch_destroy(self._h)
        except Exception:
            pass

    def bind(self, X, Y):
        xp, xl = _vec_table(X, self.nrhs, [p.mat_dims[1] for p in self.plans])
        yp, yl = _vec_table(Y, self.nrhs, [p.mat_dims[0] for p in self.plans])
        _check(lib().spx_batch_bind(self._h, xp, xl, yp, yl))
        self._bound = (list(X), list(Y))

    def run(self, stream=None):
        _check(lib().spx_batch_run(self._h, _stream(stream)))

    def capture(self):
        _check(lib().spx_batch_capture(self._h))

    def replay(self, stream=None):
        _check(lib().spx_batch_replay(self._h, _stream(stream)))

    def autotune(self, reps=3, stream=None):
        c = BatchConfig()
        _check(lib().spx_batch_autotune(self._h, int(reps), ctypes.byref(c), _stream(stream)))
        return {"order": c.order, "span_div": c.span_div, "reduce_iters": c.reduce_iters, "ms": c.ms}

    def configure(self, order=0, span_div=1, reduce_iters=64):
        c = BatchConfig(order, span_div, reduce_iters, 0.0)
        _check(lib().spx_batch_configure(self._h, ctypes.byref(c)))

    def info(self):
        ni, gr = ctypes.c_int32(), ctypes.c_int32()
        nb = ctypes.c_int64()
        _check(lib().spx_batch_info(self._h, ctypes.byref(ni), ctypes.byref(nb), ctypes.byref(gr)))
        return {"nitems": ni.value, "bytes": nb.value, "grid": gr.value}


def spmv_batched(plans, nrhs, X, Y, stream=None):
    """One-shot batched products (create, bind, run, wait, destroy)."""
    arr = (ctypes.c_void_p * max(len(plans), 1))(*[p.handle.value for p in plans])
    ks = [int(k) for k in nrhs]
    kk = np.ascontiguousarray(ks, dtype=np.int32)
    xp, xl = _vec_table(X, ks, [p.mat_dims[1] for p in plans])
    yp, yl = _vec_table(Y, ks, [p.mat_dims[0] for p in plans])
    _check(lib().spx_spmv_batched(len(plans), arr, _hp(kk), xp, xl, yp, yl, _stream(stream)))


# ---------------------------------------------------------------- selector network

def features(A: Mat):
    """The 40 selector features of a matrix (host computation, float32)."""
    out = np.empty(NFEATURES, np.float32)
    _check(lib().spx_features(A.handle, _hp(out)))
    return out


def mlp_forward(theta, X, logits, stream=None):
    import torch
    B = X.shape[0]
    _check(lib().spx_mlp_forward(_dev(theta, torch.float32, MLP_PARAMS), _dev(X, torch.float32, B * NFEATURES),
                                 int(B), _dev(logits, torch.float32, B * NCHOICES), _stream(stream)))


def mlp_loss_grad(theta, X, labels, loss, grad, stream=None):
    import torch
    B = X.shape[0]
    if labels.numel() < B:
        raise ValueError(f"{labels.numel()} labels for {B} samples")
    if B > 0:
        lo, hi = int(labels[:B].min()), int(labels[:B].max())
        if lo < 0 or hi >= NCHOICES:
            raise ValueError(f"labels must lie in [0, {NCHOICES}), got [{lo}, {hi}]")
    _check(lib().spx_mlp_loss_grad(_dev(theta, torch.float32, MLP_PARAMS), _dev(X, torch.float32, B * NFEATURES),
                                   _dev(labels, torch.int32, B), int(B), _dev(loss, torch.float32, 1),
                                   _dev(grad, torch.float32, MLP_PARAMS), _stream(stream)))


def mlp_loss_grad_noalloc(theta, X, labels, loss, grad, stream=None):
    """mlp_loss_grad through the entry point that allocates nothing (batches of
    at most 512 samples share one fixed device workspace per GPU)."""
    import torch
    B = X.shape[0]
    if labels.numel() < B:
        raise ValueError(f"{labels.numel()} labels for {B} samples")
    if 0 < B <= 512:
        lo, hi = int(labels[:B].min()), int(labels[:B].max())
        if lo < 0 or hi >= NCHOICES:
            raise ValueError(f"labels must lie in [0, {NCHOICES}), got [{lo}, {hi}]")
    _check(lib().spx_mlp_loss_grad_noalloc(_dev(theta, torch.float32, MLP_PARAMS),
                                           _dev(X, torch.float32, B * NFEATURES), _dev(labels, torch.int32, B),
                                           int(B), _dev(loss, torch.float32, 1),
                                           _dev(grad, torch.float32, MLP_PARAMS), _stream(stream)))


def mlp_adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    _check(lib().spx_mlp_adam(_dev(theta, torch.float32, MLP_PARAMS), _dev(grad, torch.float32, MLP_PARAMS),
                              _dev(m, torch.float32, MLP_PARAMS), _dev(v, torch.float32, MLP_PARAMS), int(t),
                              float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


def plan_from_parts(A: Mat, form, K, parts, tune=None):
    """Plan of form "sb", "db" or "split" for a given partition (SB: parts[m]
    in 0..K-1; DB: 0..K with K the row border; split: parts[nnz]).  Returns
    (plan, row_perm, col_perm)."""
    f = {"sb": FORM_SB, "db": FORM_DB, "split": FORM_SPLIT}[form]
    pa = np.ascontiguousarray(parts, dtype=np.int32)
    rp = np.empty(max(A.m, 1), np.int32)
    cp = np.empty(max(A.n, 1), np.int32)
    h = _VP()
    _check(lib().spx_plan_from_parts(A.handle, f, int(K), _hp(pa), _tune_ptr(tune), _hp(rp), _hp(cp),
                                     ctypes.byref(h)))
    return Plan(h.value, A), rp[:A.m], cp[:A.n]


# ---------------------------------------------------------------- selection

def choice_info(choice):
    """(form name, K, schedule dict) of one of the 24 choices."""
    f, k = ctypes.c_int32(), ctypes.c_int32()
    t = make_tune()
    _check(lib().spx_choice_info(int(choice), ctypes.byref(f), ctypes.byref(k), ctypes.byref(t)))
    return FORM_NAMES[f.value], k.value, {n: getattr(t, n) for n in _TUNE_FIELDS if getattr(t, n)}


def _norm_arrays(mu, sd):
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    sd = np.ascontiguousarray(sd, dtype=np.float64)
    if mu.size != NFEATURES or sd.size != NFEATURES:
        raise ValueError(f"mu and sd need {NFEATURES} entries")
    return mu, sd


def select(A: Mat, theta, mu, sd, stream=None):
    """The network's choice for matrix A: (choice, logits[24])."""
    import torch
    mu, sd = _norm_arrays(mu, sd)
    c = ctypes.c_int32()
    lg = np.empty(NCHOICES, np.float32)
    _check(lib().spx_select(A.handle, _dev(theta, torch.float32, MLP_PARAMS), _hp(mu), _hp(sd), ctypes.byref(c),
                            _hp(lg), _stream(stream)))
    return c.value, lg


def select_features(f, theta, mu, sd, stream=None):
    """The network's choice for raw features f[40] (from features()): (choice, logits)."""
    import torch
    mu, sd = _norm_arrays(mu, sd)
    f = np.ascontiguousarray(f, dtype=np.float32)
    if f.size != NFEATURES:
        raise ValueError(f"features need {NFEATURES} entries")
    c = ctypes.c_int32()
    lg = np.empty(NCHOICES, np.float32)
    _check(lib().spx_select_features(_hp(f), _dev(theta, torch.float32, MLP_PARAMS), _hp(mu), _hp(sd),
                                     ctypes.byref(c), _hp(lg), _stream(stream)))
    return c.value, lg


def plan_for_choice(A: Mat, choice, seed=0):
    """(plan, row_perm, col_perm) of a choice for A."""
    rp = np.empty(max(A.m, 1), np.int32)
    cp = np.empty(max(A.n, 1), np.int32)
    h = _VP()
    _check(lib().spx_plan_for_choice(A.handle, int(choice), ctypes.c_uint64(int(seed)), _hp(rp), _hp(cp),
                                     ctypes.byref(h)))
    return Plan(h.value, A), rp[:A.m], cp[:A.n]


def select_exhaustive(A: Mat, x, y, reps=10, seed=0, stream=None):
    """Every choice timed on x -> y: (fastest choice, ms[24], partition seconds)."""
    import torch
    ms = np.empty(NCHOICES, np.float32)
    c = ctypes.c_int32()
    tp = ctypes.c_double()
    _check(lib().spx_select_exhaustive(A.handle, _dev(x, torch.float64, A.n), _dev(y, torch.float64, A.m),
                                       int(reps), ctypes.c_uint64(int(seed)), _hp(ms), ctypes.byref(c),
                                       ctypes.byref(tp), _stream(stream)))
    return c.value, ms.astype(np.float64), tp.value


_TREE_FORMS = {"sb": 1, "db": 2, "split": 3}


def partition_tree(A: Mat, form, seed=0):
    """The K = 256 bisection the reordered choices of form ("sb", "db",
    "split") are cut from, computed on the host: (parts int32, seconds)."""
    n = A.nnz if form == "split" else A.m
    parts = np.empty(max(n, 1), np.int32)
    sec = ctypes.c_double()
    _check(lib().spx_partition_tree(A.handle, _TREE_FORMS[form], ctypes.c_uint64(int(seed)), _hp(parts),
                                    ctypes.byref(sec)))
    return parts[:n], sec.value


def select_exhaustive_trees(A: Mat, trees, x, y, reps=10, stream=None):
    """select_exhaustive with the three trees given (dict form -> parts as
    partition_tree returns them): (fastest choice, ms[24])."""
    import torch
    ts = [np.ascontiguousarray(trees[f], dtype=np.int32) for f in ("sb", "db", "split")]
    ms = np.empty(NCHOICES, np.float32)
    c = ctypes.c_int32()
    _check(lib().spx_select_exhaustive_trees(A.handle, _hp(ts[0]), _hp(ts[1]), _hp(ts[2]),
                                             _dev(x, torch.float64, A.n), _dev(y, torch.float64, A.m), int(reps),
                                             _hp(ms), ctypes.byref(c), _stream(stream)))
    return c.value, ms.astype(np.float64)


# ---------------------------------------------------------------- comparison orderings

def order_bfs(A: Mat):
    """sBFS (Section 5.1): (row_perm, col_perm) from breadth-first search on
    the bipartite graph of A."""
    rp = np.empty(max(A.m, 1), np.int32)
    cp = np.empty(max(A.n, 1), np.int32)
    _check(lib().spx_order_bfs(A.handle, _hp(rp), _hp(cp)))
    return rp[:A.m], cp[:A.n]


def order_rcm(A: Mat):
    """sRCM (Section 5.1): (row_perm, col_perm) from reverse Cuthill-McKee on
    the bipartite graph of A."""
    rp = np.empty(max(A.m, 1), np.int32)
    cp = np.empty(max(A.n, 1), np.int32)
    _check(lib().spx_order_rcm(A.handle, _hp(rp), _hp(cp)))
    return rp[:A.m], cp[:A.n]


def plan_from_perm(A: Mat, row_perm, col_perm, tune=None):
    """Plan holding A[row_perm][:, col_perm] in CSR (form "order")."""
    rp = np.ascontiguousarray(row_perm, dtype=np.int32)
    cp = np.ascontiguousarray(col_perm, dtype=np.int32)
    if rp.size != A.m or cp.size != A.n:
        raise ValueError("row_perm needs m entries and col_perm n entries")
    h = _VP()
    _check(lib().spx_plan_from_perm(A.handle, _hp(rp), _hp(cp), _tune_ptr(tune), ctypes.byref(h)))
    return Plan(h.value, A)
