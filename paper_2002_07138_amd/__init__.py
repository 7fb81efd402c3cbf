"""Python binding of libpowerlu (PowerLU / PowerLU_FP on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library (``libpowerlu.so`` next to this file, built by ``build.py``).  torch is
used for device memory and the current stream.  If the library is missing the
import of any entry point raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpowerlu.so")

PLU_OK = 0
PLU_WARN_ZERO_PIVOT = 1
PLU_TOL_NOT_REACHED = 2
PLU_ERR_NONFINITE = 3
PLU_ERR_OOM = 4
PLU_ERR_HIP = 5
PLU_ERR_NOT_IMPLEMENTED = 6
PLU_ERR_TIMEOUT = 7
PLU_PENDING = 8
PLU_ERR_TOO_LARGE = 9
PREC_FP32 = 0
PREC_BF16 = 1
PREC_FP8_E4M3 = 2
PREC_REFINE_LAST = 16
PREC_REFINE_TWO = 32
PREC_A_UNCHANGED = 64
PREC_FP64_INDICATOR = 128
LAYOUT_ROW = 0
LAYOUT_COL = 1
PEAK_MFMA_FP32 = 0
PEAK_MFMA_BF16 = 1
PEAK_MFMA_FP8 = 2
PEAK_HBM_READ = 3

_ENTRY_POINTS = [
    "plu_create", "plu_destroy", "plu_set_stream", "plu_workspace_size", "plu_status_string",
    "plu_fixed_rank", "plu_fixed_precision", "plu_residual", "plu_gaussian", "plu_pass",
    "plu_getrf", "plu_thin_qr", "plu_range_basis", "plu_rank_rule", "plu_quantize",
    "plu_batched", "plu_set_pivot_trace", "plu_pivot_trace", "plu_single_pass",
    "plu_randlu", "plu_randsvd", "plu_sparse_create", "plu_sparse_destroy", "plu_sparse_pass",
    "plu_sparse_fixed_rank", "plu_sparse_fixed_precision", "plu_sparse_randlu",
    "plu_sparse_randsvd", "plu_server_create",
    "plu_server_submit", "plu_server_poll",
    "plu_server_wait", "plu_server_destroy", "plu_fixed_rank_static", "plu_measure_peak",
]
BATCH_GRAPH = 1
BATCH_ONE_STREAM = 2


class PluInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("rank", ctypes.c_int32), ("passes", ctypes.c_int32),
        ("zero_pivot_step", ctypes.c_int32), ("tol_reached", ctypes.c_int32),
        ("l", ctypes.c_int32), ("normA2", ctypes.c_double), ("E_final", ctypes.c_double),
        ("min_pivot_gap", ctypes.c_float), ("pad_", ctypes.c_float),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


class PluRequest(ctypes.Structure):
    """Mirror of plu_request (include/powerlu.h)."""
    _fields_ = [
        ("mode", ctypes.c_int32), ("column_exact", ctypes.c_int32),
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("k", ctypes.c_int32), ("p_over", ctypes.c_int32), ("v", ctypes.c_int32),
        ("b", ctypes.c_int32), ("l", ctypes.c_int32),
        ("eps", ctypes.c_double), ("prec", ctypes.c_int32),
        ("Omega", ctypes.c_void_p), ("seed", ctypes.c_uint64),
        ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
        ("L", ctypes.c_void_p), ("ldl", ctypes.c_int64),
        ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
        ("layout", ctypes.c_int32),
        ("rank", ctypes.c_int32), ("status", ctypes.c_int32),
        ("info", PluInfo),
    ]


class PluResult(ctypes.Structure):
    """Mirror of plu_result (include/powerlu.h)."""
    _fields_ = [
        ("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("rank", ctypes.c_int32),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
        ("info", PluInfo),
    ]


class PowerLUError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib().plu_status_string(code).decode() if code > 0 else f"invalid argument {-code}"
        super().__init__(f"{where}: status {code} ({msg})")


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpowerlu.so not found at {LIB_PATH}; run build.py "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_double)
        pinfo = ctypes.POINTER(PluInfo)
        sig = {
            "plu_create": [ctypes.POINTER(vp), ctypes.c_int, vp],
            "plu_destroy": [vp],
            "plu_set_stream": [vp, vp],
            "plu_workspace_size": [vp, i64, i64, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
            "plu_status_string": [ctypes.c_int],
            "plu_fixed_rank": [vp, i32, i64, i64, vp, i64, i32, i32, i32, i32, vp, u64,
                               vp, vp, vp, i64, vp, i64, vp, ctypes.c_size_t, pinfo],
            "plu_fixed_rank_static": [vp, i32, i64, i64, vp, i64, i32, i32, i32, i32, vp, u64,
                                      vp, vp, vp, i64, vp, i64, pinfo],
            "plu_fixed_precision": [vp, i32, i64, i64, vp, i64, dbl, i32, i32, i32, i32, i32, i32, vp,
                                    u64, vp, vp, vp, i64, vp, i64, vp, vp, ctypes.c_size_t,
                                    pinfo],
            "plu_residual": [vp, i32, i64, i64, vp, i64, vp, vp, i32, vp, i64, vp, i64,
                             ctypes.POINTER(dbl)],
            "plu_gaussian": [vp, i64, i64, u64, vp, i64],
            "plu_pass": [vp, i32, i64, i64, vp, i64, i32, vp, i64, vp, i64, i32, vp],
            "plu_getrf": [vp, i64, i32, vp, i64, vp, vp, i64, pinfo],
            "plu_thin_qr": [vp, i64, i32, vp, i64],
            "plu_range_basis": [vp, i32, i64, i64, vp, i64, i32, i32, i32, vp, u64, vp, i64],
            "plu_rank_rule": [vp, i64, i32, vp, i64, dbl, dbl, i32, i32, ctypes.POINTER(i32),
                              ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
            "plu_quantize": [vp, i32, i64, i64, vp, i64, i32, vp, i64, vp],
            "plu_batched": [vp, i32, ctypes.POINTER(PluRequest), i32],
            "plu_set_pivot_trace": [vp, i64],
            "plu_single_pass": [vp, i32, i64, i64, vp, i64, i32, vp, u64, vp, vp, vp, i64, vp, i64,
                                pinfo],
            "plu_randlu": [vp, i32, i64, i64, vp, i64, i32, i32, i32, vp, u64, vp, vp, vp, i64, vp,
                           i64, pinfo],
            "plu_randsvd": [vp, i32, i64, i64, vp, i64, i32, i32, i32, vp, u64, vp, i64, vp, vp,
                            i64, pinfo],
            "plu_sparse_create": [vp, i64, i64, i64, vp, vp, vp, ctypes.POINTER(vp)],
            "plu_sparse_destroy": [vp],
            "plu_sparse_pass": [vp, vp, i32, vp, i64, i32, vp, i64],
            "plu_sparse_fixed_rank": [vp, vp, i32, i32, i32, i32, vp, u64, vp, vp, vp, i64, vp, i64,
                                      pinfo],
            "plu_sparse_fixed_precision": [vp, vp, dbl, i32, i32, i32, i32, i32, i32, vp, u64, vp,
                                           vp, vp, i64, vp, i64, vp, pinfo],
            "plu_sparse_randlu": [vp, vp, i32, i32, i32, vp, u64, vp, vp, vp, i64, vp, i64, pinfo],
            "plu_sparse_randsvd": [vp, vp, i32, i32, i32, vp, u64, vp, i64, vp, vp, i64, pinfo],
            "plu_pivot_trace": [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), i32,
                                ctypes.POINTER(i32)],
            "plu_server_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t, i32],
            "plu_server_submit": [vp, ctypes.POINTER(PluRequest), ctypes.POINTER(u64)],
            "plu_server_poll": [vp, u64, ctypes.POINTER(PluResult)],
            "plu_server_wait": [vp, u64, ctypes.POINTER(PluResult)],
            "plu_server_destroy": [vp],
            "plu_measure_peak": [vp, i32, vp, i64, i32, ctypes.POINTER(dbl)],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "plu_status_string" else ctypes.c_int
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (raises if it was not built)."""
    return _lib()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_mat(t, name, dtype="float32", allow_col=False):
    import torch
    if t is None:
        return
    want = {"float32": torch.float32, "int32": torch.int32, "float64": torch.float64}[dtype]
    if t.dtype != want:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError(f"{name}: expected a device tensor")
    if t.dim() == 2 and t.stride(1) != 1:
        if not (allow_col and t.stride(0) == 1):
            raise ValueError(f"{name}: rows must be contiguous (row-major)"
                             + (" or columns contiguous (column-major)" if allow_col else ""))


def _ld(t):
    return t.stride(0) if t.dim() == 2 else 1


def _a_layout(shape, strides):
    """Storage order of A from its element strides: rows contiguous gives
    (LAYOUT_ROW, lda = row stride); columns contiguous gives (LAYOUT_COL,
    lda = column stride)."""
    m, n = shape
    if strides[1] == 1 and (m == 1 or strides[0] >= n):
        return LAYOUT_ROW, max(strides[0], n)
    if strides[0] == 1 and (n == 1 or strides[1] >= m):
        return LAYOUT_COL, max(strides[1], m)
    raise ValueError("A: rows or columns must be contiguous")


def _layout_of(A):
    _check_mat(A, "A", allow_col=True)
    return _a_layout(tuple(A.shape), (A.stride(0), A.stride(1)))


@dataclass
class Factors:
    p: "object"
    q: "object"
    L: "object"
    U: "object"
    rank: int
    info: dict


class SparseMatrix:
    """A sparse matrix in compressed rows bound to a handle's device
    (plu_sparse_create).  rowptr (int64, m + 1), colidx (int32) and vals
    (float32) are device tensors; they are kept referenced (the library
    borrows them) until close()."""

    def __init__(self, handle, rowptr, colidx, vals, shape):
        t = handle._torch
        m, n = (int(shape[0]), int(shape[1]))
        for x, name, dt in ((rowptr, "rowptr", t.int64), (colidx, "colidx", t.int32),
                            (vals, "vals", t.float32)):
            if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == dt and x.dim() == 1
                    and x.is_contiguous()):
                raise TypeError(f"{name}: a contiguous 1-D {dt} device tensor is needed")
        if rowptr.numel() != m + 1 or colidx.numel() != vals.numel():
            raise ValueError("rowptr needs m + 1 entries and colidx, vals one per stored entry")
        self.shape = (m, n)
        self.nnz = int(vals.numel())
        self.device = vals.device
        self._keep = (rowptr, colidx, vals)
        sp = ctypes.c_void_p()
        rc = _lib().plu_sparse_create(handle._h, m, n, self.nnz, _ptr(rowptr), _ptr(colidx),
                                      _ptr(vals), ctypes.byref(sp))
        if rc != PLU_OK:
            raise PowerLUError(rc, "plu_sparse_create")
        self._sp = sp

    def close(self):
        if getattr(self, "_sp", None):
            _lib().plu_sparse_destroy(self._sp)
            self._sp = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Handle:
    """One libpowerlu handle bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        lib = _lib()
        h = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        rc = lib.plu_create(ctypes.byref(h), device, ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise PowerLUError(rc, "plu_create")
        self._h = h
        self._stream = s

    def close(self):
        if getattr(self, "_h", None):
            _lib().plu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._stream = stream
        rc = _lib().plu_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise PowerLUError(rc, "plu_set_stream")

    def _rc(self, rc, where, ok=(PLU_OK,)):
        if rc not in ok:
            raise PowerLUError(rc, where)
        return rc

    # ---------------------------------------------------------------- steps
    def gaussian(self, rows, cols, seed, out=None):
        t = self._torch
        if out is None:
            out = t.empty((rows, cols), dtype=t.float32, device=f"cuda:{self.device}")
        _check_mat(out, "out")
        self._rc(_lib().plu_gaussian(self._h, rows, cols, seed, _ptr(out), _ld(out)), "plu_gaussian")
        return out

    def pass_(self, A, X, trans=False, out=None, prec=PREC_FP32, normA2=None):
        t = self._torch
        _check_mat(A, "A"); _check_mat(X, "X")
        m, n = A.shape
        l = X.shape[1]
        rows = n if trans else m
        if out is None:
            out = t.empty((rows, l), dtype=t.float32, device=A.device)
        _check_mat(out, "out")
        if normA2 is not None:
            _check_mat(normA2, "normA2", "float64")
        self._rc(_lib().plu_pass(self._h, 1 if trans else 0, m, n, _ptr(A), _ld(A), l, _ptr(X),
                                 _ld(X), _ptr(out), _ld(out), prec, _ptr(normA2)), "plu_pass")
        return out

    def quantize(self, src, fmt=PREC_BF16, transpose=False):
        """Rounded copy of src (the operand rounding of the precision form).
        BF16: returns the codes as int16 (bfloat16 bit patterns), row length
        padded to a multiple of 64 with zeros.  FP8_E4M3: returns (codes
        uint8, scale bytes uint8), row length padded to a multiple of 128."""
        t = self._torch
        _check_mat(src, "src")
        rows, cols = src.shape
        out_rows, row_len = (cols, rows) if transpose else (rows, cols)
        if fmt == PREC_FP8_E4M3:
            ldd = (row_len + 127) // 128 * 128
            dst = t.empty((out_rows, ldd), dtype=t.uint8, device=src.device)
            sc = t.empty((out_rows, ldd // 32), dtype=t.uint8, device=src.device)
        else:
            ldd = (row_len + 63) // 64 * 64
            dst = t.empty((out_rows, ldd), dtype=t.int16, device=src.device)
            sc = None
        self._rc(_lib().plu_quantize(self._h, fmt, rows, cols, _ptr(src), _ld(src),
                                     1 if transpose else 0, _ptr(dst), ldd, _ptr(sc)),
                 "plu_quantize")
        return dst if sc is None else (dst, sc)

    def getrf(self, F, want_perm=True, want_u=True, sync_info=True):
        """In place: F -> V = P^T L.  Returns (perm, U, info)."""
        t = self._torch
        _check_mat(F, "F")
        M, c = F.shape
        perm = t.empty(M, dtype=t.int32, device=F.device) if want_perm else None
        U = t.empty((c, c), dtype=t.float32, device=F.device) if want_u else None
        info = PluInfo()
        rc = _lib().plu_getrf(self._h, M, c, _ptr(F), _ld(F), _ptr(perm), _ptr(U),
                              _ld(U) if U is not None else 0,
                              ctypes.byref(info) if sync_info else None)
        self._rc(rc, "plu_getrf", ok=(PLU_OK, PLU_WARN_ZERO_PIVOT))
        return perm, U, (info.as_dict() if sync_info else None)

    def thin_qr(self, X):
        _check_mat(X, "X")
        M, c = X.shape
        self._rc(_lib().plu_thin_qr(self._h, M, c, _ptr(X), _ld(X)), "plu_thin_qr")
        return X

    def range_basis(self, A, l, v, Omega=None, seed=0, prec=PREC_FP32):
        t = self._torch
        _check_mat(Omega, "Omega")
        m, n = A.shape
        V = t.empty((n, l), dtype=t.float32, device=A.device)
        lay, lda = _layout_of(A)
        self._rc(_lib().plu_range_basis(self._h, lay, m, n, _ptr(A), lda, l, v, prec,
                                        _ptr(Omega), seed, _ptr(V), _ld(V)), "plu_range_basis")
        return V

    def rank_rule(self, G, normA2, eps, b, column_exact=True):
        _check_mat(G, "G")
        m, l = G.shape
        k = ctypes.c_int32()
        E = ctypes.c_double()
        cn = (ctypes.c_double * l)()
        rc = _lib().plu_rank_rule(self._h, m, l, _ptr(G), _ld(G), float(normA2), float(eps), b,
                                  1 if column_exact else 0, ctypes.byref(k), ctypes.byref(E), cn)
        self._rc(rc, "plu_rank_rule", ok=(PLU_OK, PLU_TOL_NOT_REACHED))
        return k.value, E.value, list(cn), rc == PLU_OK

    # ------------------------------------------------------------- sparse A
    def sparse_matrix(self, rowptr, colidx, vals, shape):
        """Bind a device matrix in compressed rows (see SparseMatrix)."""
        return SparseMatrix(self, rowptr, colidx, vals, shape)

    def sparse_pass(self, S, X, trans=False, out=None):
        """out = S X (trans False) or S^T X (trans True) for a SparseMatrix S."""
        _check_mat(X, "X")
        m, n = S.shape
        rows = n if trans else m
        l = X.shape[1]
        if out is None:
            out = self._torch.empty((rows, l), dtype=self._torch.float32, device=X.device)
        rc = _lib().plu_sparse_pass(self._h, S._sp, 1 if trans else 0, _ptr(X), _ld(X), l,
                                    _ptr(out), _ld(out))
        self._rc(rc, "plu_sparse_pass")
        return out

    # ------------------------------------------------------------- problems
    def workspace_size(self, m, n, l, prec=PREC_FP32, max_rounds=1):
        """Bytes of caller workspace a call of this shape needs (plu_workspace_size)."""
        b = ctypes.c_size_t()
        self._rc(_lib().plu_workspace_size(self._h, m, n, l, int(max_rounds), prec,
                                           ctypes.byref(b)), "plu_workspace_size")
        return b.value

    def fixed_rank(self, A, k, p_over, v, Omega=None, seed=0, prec=PREC_FP32, sync_info=True,
                   out=None, work=None):
        """PowerLU (Alg. 5 with Alg. 7); A is a device tensor or a SparseMatrix."""
        t = self._torch
        _check_mat(Omega, "Omega")
        sparse = isinstance(A, SparseMatrix)
        lay, lda = (0, 0) if sparse else _layout_of(A)
        m, n = A.shape
        dev = A.device
        if out is None:
            p = t.empty(m, dtype=t.int32, device=dev)
            q = t.empty(n, dtype=t.int32, device=dev)
            L = t.empty((m, k), dtype=t.float32, device=dev)
            U = t.empty((k, n), dtype=t.float32, device=dev)
        else:
            p, q, L, U = out
        info = PluInfo()
        pinfo = ctypes.byref(info) if sync_info else None
        if sparse:
            rc = _lib().plu_sparse_fixed_rank(self._h, A._sp, k, p_over, v, prec, _ptr(Omega),
                                              seed, _ptr(p), _ptr(q), _ptr(L), _ld(L), _ptr(U),
                                              _ld(U), pinfo)
        else:
            rc = _lib().plu_fixed_rank(self._h, lay, m, n, _ptr(A), lda, k, p_over, v, prec,
                                       _ptr(Omega), seed, _ptr(p), _ptr(q), _ptr(L), _ld(L),
                                       _ptr(U), _ld(U), _ptr(work),
                                       0 if work is None else work.numel() * work.element_size(),
                                       pinfo)
        self._rc(rc, "plu_fixed_rank", ok=(PLU_OK, PLU_WARN_ZERO_PIVOT))
        return Factors(p, q, L, U, k, info.as_dict() if sync_info else {})

    def fixed_rank_static(self, A, k, p_over, v, Omega=None, seed=0, prec=PREC_FP32,
                          sync_info=True, out=None):
        """plu_fixed_rank_static: PowerLU on the library's static scratch (no
        allocation by the library; out = (p, q, L, U) preallocated by the
        caller, or allocated here by torch)."""
        t = self._torch
        _check_mat(Omega, "Omega")
        lay, lda = _layout_of(A)
        m, n = A.shape
        if out is None:
            dev = A.device
            out = (t.empty(m, dtype=t.int32, device=dev), t.empty(n, dtype=t.int32, device=dev),
                   t.empty((m, k), dtype=t.float32, device=dev),
                   t.empty((k, n), dtype=t.float32, device=dev))
        p, q, L, U = out
        info = PluInfo()
        rc = _lib().plu_fixed_rank_static(self._h, lay, m, n, _ptr(A), lda, k, p_over, v, prec,
                                          _ptr(Omega), seed, _ptr(p), _ptr(q), _ptr(L), _ld(L),
                                          _ptr(U), _ld(U), ctypes.byref(info) if sync_info else None)
        self._rc(rc, "plu_fixed_rank_static", ok=(PLU_OK, PLU_WARN_ZERO_PIVOT))
        return Factors(p, q, L, U, k, info.as_dict() if sync_info else {})

    def single_pass(self, A, k, Omega=None, seed=0, sync_info=True):
        """Single-pass randomized LU (Alg. 10): one pass over a column-major A
        (two over a row-major one)."""
        t = self._torch
        _check_mat(Omega, "Omega")
        lay, lda = _layout_of(A)
        m, n = A.shape
        dev = A.device
        p = t.empty(m, dtype=t.int32, device=dev)
        q = t.empty(n, dtype=t.int32, device=dev)
        L = t.empty((m, k), dtype=t.float32, device=dev)
        U = t.empty((k, n), dtype=t.float32, device=dev)
        info = PluInfo()
        rc = _lib().plu_single_pass(self._h, lay, m, n, _ptr(A), lda, k, _ptr(Omega), seed,
                                    _ptr(p), _ptr(q), _ptr(L), _ld(L), _ptr(U), _ld(U),
                                    ctypes.byref(info) if sync_info else None)
        self._rc(rc, "plu_single_pass", ok=(PLU_OK, PLU_WARN_ZERO_PIVOT))
        return Factors(p, q, L, U, k, info.as_dict() if sync_info else {})

    def randlu(self, A, k, p_over, pw, Omega=None, seed=0, sync_info=True):
        """RandLU (Alg. 3 with the Alg. 4 power iteration, exponent pw):
        2 pw + 2 passes over A; Omega is n x (k + p_over)."""
        t = self._torch
        _check_mat(Omega, "Omega")
        sparse = isinstance(A, SparseMatrix)
        lay, lda = (0, 0) if sparse else _layout_of(A)
        m, n = A.shape
        dev = A.device
        p = t.empty(m, dtype=t.int32, device=dev)
        q = t.empty(n, dtype=t.int32, device=dev)
        L = t.empty((m, k), dtype=t.float32, device=dev)
        U = t.empty((k, n), dtype=t.float32, device=dev)
        info = PluInfo()
        pinfo = ctypes.byref(info) if sync_info else None
        if sparse:
            rc = _lib().plu_sparse_randlu(self._h, A._sp, k, p_over, pw, _ptr(Omega), seed,
                                          _ptr(p), _ptr(q), _ptr(L), _ld(L), _ptr(U), _ld(U),
                                          pinfo)
        else:
            rc = _lib().plu_randlu(self._h, lay, m, n, _ptr(A), lda, k, p_over, pw, _ptr(Omega),
                                   seed, _ptr(p), _ptr(q), _ptr(L), _ld(L), _ptr(U), _ld(U),
                                   pinfo)
        self._rc(rc, "plu_randlu", ok=(PLU_OK, PLU_WARN_ZERO_PIVOT))
        return Factors(p, q, L, U, k, info.as_dict() if sync_info else {})

    def randsvd(self, A, k, p_over, pw, Omega=None, seed=0, sync_info=True):
        """RandSVD (Alg. 1 with the Alg. 2 power iteration, exponent pw):
        returns (U m x k, S (k,), V n x k, info); 2 pw + 2 passes over A."""
        t = self._torch
        _check_mat(Omega, "Omega")
        sparse = isinstance(A, SparseMatrix)
        lay, lda = (0, 0) if sparse else _layout_of(A)
        m, n = A.shape
        dev = A.device
        U = t.empty((m, k), dtype=t.float32, device=dev)
        S = t.empty(k, dtype=t.float32, device=dev)
        V = t.empty((n, k), dtype=t.float32, device=dev)
        info = PluInfo()
        pinfo = ctypes.byref(info) if sync_info else None
        if sparse:
            rc = _lib().plu_sparse_randsvd(self._h, A._sp, k, p_over, pw, _ptr(Omega), seed,
                                           _ptr(U), _ld(U), _ptr(S), _ptr(V), _ld(V), pinfo)
        else:
            rc = _lib().plu_randsvd(self._h, lay, m, n, _ptr(A), lda, k, p_over, pw, _ptr(Omega),
                                    seed, _ptr(U), _ld(U), _ptr(S), _ptr(V), _ld(V), pinfo)
        self._rc(rc, "plu_randsvd")
        return U, S, V, (info.as_dict() if sync_info else {})

    def fixed_precision(self, A, eps, b, l=0, v=4, column_exact=True, Omega=None, seed=0,
                        prec=PREC_FP32, max_rounds=1, sync_info=True, out=None, work=None):
        """PowerLU_FP (Alg. 9); A is a device tensor or a SparseMatrix.

        sync_info=True: synchronizes and returns Factors trimmed to the rank.
        sync_info=False: returns at once (max_rounds = 1): Factors with the
        full-capacity L, U and rank = the device int32 tensor (1,) the call
        writes the rank into.  out = (p, q, L, U, rank) reuses buffers."""
        t = self._torch
        _check_mat(Omega, "Omega")
        sparse = isinstance(A, SparseMatrix)
        lay, lda = (0, 0) if sparse else _layout_of(A)
        m, n = A.shape
        dev = A.device
        lcap = (l if l else min(50 * b, b * ((min(m, n) - 1) // b))) * max(int(max_rounds), 1)
        if out is None:
            p = t.empty(m, dtype=t.int32, device=dev)
            q = t.empty(n, dtype=t.int32, device=dev)
            L = t.empty((m, lcap), dtype=t.float32, device=dev)
            U = t.empty((lcap, n), dtype=t.float32, device=dev)
            k = t.zeros(1, dtype=t.int32, device=dev)
        else:
            p, q, L, U, k = out
        info = PluInfo()
        pinfo = ctypes.byref(info) if sync_info else None
        if sparse:
            rc = _lib().plu_sparse_fixed_precision(self._h, A._sp, float(eps), b, l, v,
                                                   1 if column_exact else 0, int(max_rounds), prec,
                                                   _ptr(Omega), seed, _ptr(p), _ptr(q), _ptr(L),
                                                   _ld(L), _ptr(U), _ld(U), _ptr(k), pinfo)
        else:
            rc = _lib().plu_fixed_precision(self._h, lay, m, n, _ptr(A), lda, float(eps), b, l, v,
                                            1 if column_exact else 0, int(max_rounds), prec,
                                            _ptr(Omega), seed,
                                            _ptr(p), _ptr(q), _ptr(L), _ld(L), _ptr(U), _ld(U),
                                            _ptr(k), _ptr(work),
                                            0 if work is None else work.numel() * work.element_size(),
                                            pinfo)
        self._rc(rc, "plu_fixed_precision", ok=(PLU_OK, PLU_WARN_ZERO_PIVOT, PLU_TOL_NOT_REACHED))
        if not sync_info:
            return Factors(p, q, L, U, k, {})
        kk = int(info.rank)
        return Factors(p, q, L[:, :kk], U[:kk], kk, info.as_dict())

    def batched(self, problems, graph=False, one_stream=False):
        """Solve many problems in one batched call (plu_batched).  Each
        problem is a dict with A (device fp32 matrix) and either
        mode=0, k, p_over, v or mode=1, eps, b, l (0: default), v,
        column_exact; optional Omega, seed, prec (any form but
        PREC_FP64_INDICATOR), out = (p, q, L, U) device buffers.
        one_stream: every problem on the handle's stream (no side streams).
        Returns a list of Factors (the fixed-precision ones trimmed to their
        rank)."""
        t = self._torch
        reqs = (PluRequest * len(problems))()
        keep = []
        for r, pr in zip(reqs, problems):
            A = pr["A"]
            lay, lda = _layout_of(A)
            m, n = A.shape
            mode = int(pr.get("mode", 0))
            r.mode = mode
            r.column_exact = 1 if pr.get("column_exact", True) else 0
            r.m, r.n, r.lda, r.layout = m, n, lda, lay
            r.A = A.data_ptr()
            r.v = int(pr["v"])
            r.prec = int(pr.get("prec", PREC_FP32))
            if mode == 0:
                r.k, r.p_over = int(pr["k"]), int(pr["p_over"])
                cap = r.k
            else:
                r.b, r.l, r.eps = int(pr["b"]), int(pr.get("l", 0)), float(pr["eps"])
                cap = r.l if r.l else min(50 * r.b, r.b * ((min(m, n) - 1) // r.b))
            Om = pr.get("Omega")
            if Om is not None:
                _check_mat(Om, "Omega")
            r.Omega = Om.data_ptr() if Om is not None else None
            r.seed = int(pr.get("seed", 0))
            if pr.get("out") is not None:
                p, q, L, U = pr["out"]
                _check_mat(L, "L")
                _check_mat(U, "U")
                if L.shape[1] < cap or U.shape[0] < cap:
                    raise ValueError("out: L needs >= %d columns and U >= %d rows" % (cap, cap))
            else:
                p = t.empty(m, dtype=t.int32, device=A.device)
                q = t.empty(n, dtype=t.int32, device=A.device)
                L = t.empty((m, cap), dtype=t.float32, device=A.device)
                U = t.empty((cap, n), dtype=t.float32, device=A.device)
            r.p, r.q, r.L, r.ldl, r.U, r.ldu = p.data_ptr(), q.data_ptr(), L.data_ptr(), \
                _ld(L), U.data_ptr(), _ld(U)
            keep.append((p, q, L, U, A, Om))
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_ONE_STREAM if one_stream else 0)
        rc = _lib().plu_batched(self._h, len(problems), reqs, flags)
        if rc != PLU_OK:
            bad = [(i, r.status) for i, r in enumerate(reqs) if r.status != 0]
            raise PowerLUError(rc, f"plu_batched (request statuses {bad})")
        out = []
        for r, (p, q, L, U, A, Om) in zip(reqs, keep):
            if r.status not in (PLU_OK, PLU_WARN_ZERO_PIVOT, PLU_TOL_NOT_REACHED):
                raise PowerLUError(r.status, "plu_batched request")
            k = r.rank
            out.append(Factors(p, q, L[:, :k], U[:k], k, r.info.as_dict()))
        return out

    def set_pivot_trace(self, capacity):
        """Record the pivots of every GETRF of each following call (up to
        `capacity` entries); 0 turns recording off."""
        self._rc(_lib().plu_set_pivot_trace(self._h, int(capacity)), "plu_set_pivot_trace")

    def pivot_trace(self):
        """(pivot rows, gaps) of every GETRF of the last call, in order, as
        numpy arrays."""
        import numpy as np
        n = ctypes.c_int32()
        self._rc(_lib().plu_pivot_trace(self._h, None, None, 0, ctypes.byref(n)),
                 "plu_pivot_trace", ok=(PLU_OK, PLU_ERR_OOM))
        piv = np.zeros(n.value, np.int32)
        gaps = np.zeros(n.value, np.float32)
        self._rc(_lib().plu_pivot_trace(
            self._h, piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            gaps.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n.value, ctypes.byref(n)),
            "plu_pivot_trace")
        return piv, gaps

    def measure_peak(self, kind: int, buf=None, reps: int = 5) -> float:
        """plu_measure_peak: TFLOP/s of a matrix-core loop (PEAK_MFMA_*) or
        GB/s of a streaming read of the device tensor buf (PEAK_HBM_READ)."""
        r = ctypes.c_double()
        nbytes = 0 if buf is None else buf.numel() * buf.element_size()
        self._rc(_lib().plu_measure_peak(self._h, kind, None if buf is None else _ptr(buf),
                                         nbytes, reps, ctypes.byref(r)), "plu_measure_peak")
        return r.value

    def residual(self, A, f: Factors):
        lay, lda = _layout_of(A)
        m, n = A.shape
        r = ctypes.c_double()
        L, U = f.L, f.U
        self._rc(_lib().plu_residual(self._h, lay, m, n, _ptr(A), lda, _ptr(f.p), _ptr(f.q), f.rank,
                                     _ptr(L), _ld(L), _ptr(U), _ld(U), ctypes.byref(r)),
                 "plu_residual")
        return r.value


class Server:
    """The request loop of libpowerlu (plu_server_*).  Inputs and outputs are
    host memory: pass torch CPU tensors (pinned recommended) or numpy arrays;
    they are kept alive here until the request completes."""

    def __init__(self, device=0, hbm_budget_bytes=8 << 30, max_slots=64):
        lib = _lib()
        s = ctypes.c_void_p()
        rc = lib.plu_server_create(ctypes.byref(s), device, hbm_budget_bytes, max_slots)
        if rc != 0:
            raise PowerLUError(rc, "plu_server_create")
        self._s = s
        self._keep = {}

    @staticmethod
    def _hptr(x):
        if hasattr(x, "data_ptr"):
            if x.is_cuda:
                raise TypeError("server inputs and outputs are host memory")
            return x.data_ptr()
        return x.ctypes.data

    def submit(self, A, mode=0, k=0, p_over=0, v=4, eps=0.0, b=1, l=0, column_exact=True,
               seed=0, out=None, prec=PREC_FP32):
        """A: host fp32 m x n, rows or columns contiguous.  out: optional
        (p, q, L, U) host arrays (int32 m, int32 n, fp32 m x cap, fp32 cap x n);
        allocated (numpy) when omitted.  prec: as for the single calls (not
        PREC_FP64_INDICATOR).  Returns the ticket."""
        import numpy as np
        m, n = A.shape
        cap = k if mode == 0 else (l if l else min(50 * b, b * ((min(m, n) - 1) // b)))
        if out is None:
            out = (np.empty(m, np.int32), np.empty(n, np.int32), np.empty((m, max(cap, 1)), np.float32),
                   np.empty((max(cap, 1), n), np.float32))
        p, q, L, U = out
        r = PluRequest()
        r.mode, r.column_exact = mode, 1 if column_exact else 0
        r.m, r.n = m, n
        if hasattr(A, "stride") and callable(A.stride):
            strides = (A.stride(0), A.stride(1))
        else:
            strides = (A.strides[0] // 4, A.strides[1] // 4)
        r.layout, r.lda = _a_layout((m, n), strides)
        r.A = self._hptr(A)
        r.k, r.p_over, r.v, r.b, r.l, r.eps = k, p_over, v, b, l, float(eps)
        r.prec, r.Omega, r.seed = int(prec), None, seed
        r.p, r.q, r.L, r.U = self._hptr(p), self._hptr(q), self._hptr(L), self._hptr(U)
        r.ldl = max(cap, 1)
        r.ldu = n
        t = ctypes.c_uint64()
        rc = _lib().plu_server_submit(self._s, ctypes.byref(r), ctypes.byref(t))
        if rc != 0:
            raise PowerLUError(rc, "plu_server_submit")
        self._keep[t.value] = (A, out)
        return t.value

    def poll(self, ticket):
        res = PluResult()
        rc = _lib().plu_server_poll(self._s, ticket, ctypes.byref(res))
        if rc == PLU_PENDING:
            return None
        if rc != 0:
            raise PowerLUError(rc, "plu_server_poll")
        return self._finish(ticket, res)

    def wait(self, ticket):
        res = PluResult()
        rc = _lib().plu_server_wait(self._s, ticket, ctypes.byref(res))
        if rc != 0:
            raise PowerLUError(rc, "plu_server_wait")
        return self._finish(ticket, res)

    def _finish(self, ticket, res):
        A, (p, q, L, U) = self._keep.pop(ticket)
        k = res.rank
        return dict(p=p, q=q, L=L[:, :k], U=U[:k], rank=k, status=res.status,
                    t_submit=res.t_submit, t_admit=res.t_admit, t_done=res.t_done,
                    info=res.info.as_dict())

    def close(self):
        if getattr(self, "_s", None):
            _lib().plu_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
