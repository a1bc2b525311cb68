"""MI355X (gfx950) inexact-Krylov exponential discriminant analysis.

Thin ctypes binding of ``libeda.so`` (C ABI in ``include/eda.h``).  Every
step of the computation runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory and the stream.  There
is no CPU fallback: if the library is missing, loading fails loudly.

Problem (arXiv 1512.06500, eq. (1.7)): the t dominant eigenpairs of
exp(S_B) x = lambda exp(S_W) x with S_W = H_W H_W^T, S_B = H_B H_B^T.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

__all__ = [
    "EDAError", "Handle", "SolveResult", "load_library", "library_path", "colmajor",
    "EDA_OK", "EDA_ERR_ARG", "EDA_ERR_NOMEM", "EDA_ERR_HIP", "EDA_ERR_NOCONV",
    "EDA_ERR_RANGE", "EDA_ERR_NONFINITE", "EDA_ERR_STATE", "EXPORTED_SYMBOLS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))

EDA_OK, EDA_ERR_ARG, EDA_ERR_NOMEM, EDA_ERR_HIP = 0, 1, 2, 3
EDA_ERR_NOCONV, EDA_ERR_RANGE, EDA_ERR_NONFINITE, EDA_ERR_STATE = 4, 5, 6, 7
EDA_F64, EDA_F32, EDA_BF16, EDA_FP8_E4M3 = 0, 1, 2, 3
EDA_W, EDA_B = 0, 1
EDA_FORM_LANCZOS_M, EDA_FORM_ARNOLDI_A, EDA_FORM_JD_M = 0, 1, 2
EDA_RES_REL_THETA, EDA_RES_NORMWISE = 0, 1
EDA_WARN_DEGENERATE, EDA_WARN_FLOOR, EDA_WARN_REPAIRED, EDA_WARN_FALLBACK = 1, 2, 4, 8

_DTYPES = {"f64": EDA_F64, "f32": EDA_F32, "bf16": EDA_BF16, "fp8": EDA_FP8_E4M3}

EXPORTED_SYMBOLS = [
    "eda_create", "eda_destroy", "eda_strerror", "eda_last_error", "eda_scatter_factors",
    "eda_prepare", "eda_expmv", "eda_opmv", "eda_solve", "eda_solve_direct", "eda_solve_batched",
    "eda_gram", "eda_factor_codes", "eda_opmv_noalloc",
    "eda_syev", "eda_autotune", "eda_nn_classify",
]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("form", ctypes.c_int), ("block", ctypes.c_int32), ("max_basis", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("resmode", ctypes.c_int), ("krylov_dtype", ctypes.c_int),
        ("refine_dtype", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("start_block", ctypes.c_void_p), ("ld_start", ctypes.c_int64),
        ("check_every", ctypes.c_int32), ("max_refine", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 6),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("H_W", ctypes.c_void_p), ("ldw", ctypes.c_int64),
        ("H_B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
        ("t", ctypes.c_int32), ("tol", ctypes.c_double),
        ("ritz", ctypes.POINTER(ctypes.c_double)), ("ritz_log", ctypes.POINTER(ctypes.c_double)),
        ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
        ("resid", ctypes.POINTER(ctypes.c_double)),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("refine_passes", ctypes.c_int32), ("flags", ctypes.c_int32), ("ops", ctypes.c_int64),
        ("bytes_moved", ctypes.c_double), ("t_prepare_ms", ctypes.c_double),
        ("t_krylov_ms", ctypes.c_double), ("t_refine_ms", ctypes.c_double),
        ("shift_s", ctypes.c_double), ("op_calls", ctypes.c_int64),
        ("t_op_ms", ctypes.c_double), ("op_bytes", ctypes.c_double),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class EDAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[eda status {status}] {msg}")
        self.status = status


_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "libeda.so")


def load_library():
    """Load libeda.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1512_06500_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.eda_create.argtypes = [ctypes.POINTER(vp), vp]
    L.eda_create.restype = ctypes.c_int
    L.eda_destroy.argtypes = [vp]
    L.eda_destroy.restype = None
    L.eda_strerror.argtypes = [ctypes.c_int]
    L.eda_strerror.restype = ctypes.c_char_p
    L.eda_last_error.argtypes = [vp]
    L.eda_last_error.restype = ctypes.c_char_p
    L.eda_scatter_factors.argtypes = [vp, i64, i64, i64, vp, i64, ctypes.POINTER(i64), vp, i64,
                                      vp, i64]
    L.eda_scatter_factors.restype = ctypes.c_int
    L.eda_prepare.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, ctypes.c_int]
    L.eda_prepare.restype = ctypes.c_int
    L.eda_expmv.argtypes = [vp, ctypes.c_int, dbl, i64, vp, i64, vp, i64, ctypes.c_int,
                            ctypes.POINTER(dbl)]
    L.eda_expmv.restype = ctypes.c_int
    L.eda_opmv.argtypes = [vp, ctypes.c_int, i64, vp, i64, vp, i64, ctypes.c_int,
                           ctypes.POINTER(dbl)]
    L.eda_opmv.restype = ctypes.c_int
    L.eda_solve.argtypes = [vp, i32, dbl, ctypes.POINTER(SolveOpts), ctypes.POINTER(dbl),
                            ctypes.POINTER(dbl), vp, i64, ctypes.POINTER(dbl),
                            ctypes.POINTER(Info)]
    L.eda_solve.restype = ctypes.c_int
    L.eda_solve_direct.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp, i64,
                                   ctypes.POINTER(dbl), ctypes.POINTER(Info)]
    L.eda_solve_direct.restype = ctypes.c_int
    L.eda_solve_batched.argtypes = [vp, i32, ctypes.POINTER(Problem), ctypes.c_int,
                                    ctypes.POINTER(SolveOpts), ctypes.POINTER(Info),
                                    ctypes.POINTER(ctypes.c_int)]
    L.eda_solve_batched.restype = ctypes.c_int
    L.eda_gram.argtypes = [vp, vp, i64]
    L.eda_gram.restype = ctypes.c_int
    L.eda_factor_codes.argtypes = [vp, vp, i64, vp]
    L.eda_factor_codes.restype = ctypes.c_int
    L.eda_opmv_noalloc.argtypes = [vp, ctypes.c_int, i64, vp, i64, vp, i64, ctypes.c_int,
                                   ctypes.POINTER(dbl)]
    L.eda_opmv_noalloc.restype = ctypes.c_int
    L.eda_syev.argtypes = [vp, i64, vp, i64, vp, vp, i64]
    L.eda_syev.restype = ctypes.c_int
    L.eda_autotune.argtypes = [vp, i64, i64, i32, ctypes.c_int, ctypes.POINTER(i32),
                               ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.eda_autotune.restype = ctypes.c_int
    L.eda_nn_classify.argtypes = [vp, i64, i64, vp, i64, i64, vp, i64, vp, i64, vp, i64, vp, vp,
                                  vp]
    L.eda_nn_classify.restype = ctypes.c_int
    _lib = L
    return L


def colmajor(t):
    """Return a column-major (Fortran-order) view/copy of a 2-D tensor."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.stride(0) == 1 and (t.shape[1] <= 1 or t.stride(1) >= max(1, t.shape[0])):
        return t
    return t.t().contiguous().t()


def _ld(t) -> int:
    return max(int(t.stride(1)) if t.shape[1] > 1 else int(t.shape[0]), int(t.shape[0]), 1)


def _empty_cm(rows: int, cols: int, dtype, device):
    import torch
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


@dataclasses.dataclass
class SolveResult:
    ritz: list
    ritz_log: list
    X: object           # torch tensor d x t (column-major), float64
    resid: list
    info: dict
    status: int
    message: str


class Handle:
    """One libeda handle bound to the current device and a torch stream."""

    def __init__(self, stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = ctypes.c_void_p()
        st = self.lib.eda_create(ctypes.byref(h), ctypes.c_void_p(raw))
        self._h = h
        if st != EDA_OK:
            msg = self.lib.eda_last_error(h).decode()
            self.lib.eda_destroy(h)
            self._h = None
            raise EDAError(st, msg)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.d = self.n = self.k = None

    def close(self):
        if getattr(self, "_h", None):
            self.lib.eda_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != EDA_OK:
            raise EDAError(st, self.lib.eda_last_error(self._h).decode())

    def _f64(self, t):
        t = colmajor(t)
        if t.dtype != self._torch.float64 or t.device.type != "cuda":
            raise TypeError("expected a float64 CUDA tensor")
        return t

    # --- calls ---------------------------------------------------------------
    def scatter_factors(self, X, counts: Sequence[int]):
        """H_W, H_B of eqs. (1.1)-(1.2) from class-contiguous samples X (d x n)."""
        X = self._f64(X)
        d, n = X.shape
        k = len(counts)
        H_W = _empty_cm(d, n, self._torch.float64, X.device)
        H_B = _empty_cm(d, k, self._torch.float64, X.device)
        arr = (ctypes.c_int64 * k)(*[int(c) for c in counts])
        self._check(self.lib.eda_scatter_factors(self._h, d, n, k, X.data_ptr(), _ld(X), arr,
                                                 H_W.data_ptr(), _ld(H_W), H_B.data_ptr(),
                                                 _ld(H_B)))
        return H_W, H_B

    def prepare(self, H_W, H_B, storage: str = "f64"):
        H_W, H_B = self._f64(H_W), self._f64(H_B)
        d, n = H_W.shape
        k = H_B.shape[1]
        if H_B.shape[0] != d:
            raise ValueError("H_W and H_B need the same number of rows")
        self._check(self.lib.eda_prepare(self._h, d, n, k, H_W.data_ptr(), _ld(H_W),
                                         H_B.data_ptr(), _ld(H_B), _DTYPES[storage]))
        self.d, self.n, self.k = d, n, k
        self.storage = storage
        return self

    def _vblock(self, V, vdtype):
        V = colmajor(V)
        want = {"f64": self._torch.float64, "f32": self._torch.float32,
                "bf16": self._torch.bfloat16}[vdtype]
        if V.dtype != want or V.device.type != "cuda":
            raise TypeError(f"expected a {want} CUDA tensor")
        return V

    def expmv(self, which: str, c: float, V, out=None, vdtype: str = "f64"):
        """Out = e^{-s} exp(c S_which) V; returns (Out, s)."""
        V = self._vblock(V, vdtype)
        d, b = V.shape
        if out is None:
            out = _empty_cm(d, b, V.dtype, V.device)
        ls = ctypes.c_double()
        self._check(self.lib.eda_expmv(self._h, EDA_W if which == "W" else EDA_B, float(c), b,
                                       V.data_ptr(), _ld(V), out.data_ptr(), _ld(out),
                                       _DTYPES[vdtype], ctypes.byref(ls)))
        return out, ls.value

    def opmv(self, form: str, V, out=None, vdtype: str = "f64"):
        """Out = e^{-s} M V (form 'M') or e^{-s} A V (form 'A'); returns (Out, s)."""
        V = self._vblock(V, vdtype)
        d, b = V.shape
        if out is None:
            out = _empty_cm(d, b, V.dtype, V.device)
        ls = ctypes.c_double()
        f = EDA_FORM_LANCZOS_M if form == "M" else EDA_FORM_ARNOLDI_A
        self._check(self.lib.eda_opmv(self._h, f, b, V.data_ptr(), _ld(V), out.data_ptr(),
                                      _ld(out), _DTYPES[vdtype], ctypes.byref(ls)))
        return out, ls.value

    def opmv_noalloc(self, form: str, V, out, vdtype: str = "f64"):
        """eda_opmv_noalloc: the product of opmv with the library's static
        scratch instead of allocated workspaces; `out` must be given.
        Returns s (Out = e^{-s} M V or e^{-s} A V)."""
        V = self._vblock(V, vdtype)
        d, b = V.shape
        ls = ctypes.c_double()
        f = EDA_FORM_LANCZOS_M if form == "M" else EDA_FORM_ARNOLDI_A
        self._check(self.lib.eda_opmv_noalloc(self._h, f, b, V.data_ptr(), _ld(V),
                                              out.data_ptr(), _ld(out), _DTYPES[vdtype],
                                              ctypes.byref(ls)))
        return ls.value

    def solve(self, t: int, tol: float, block: int = 8, max_basis: int = 0, max_iter: int = 0,
              seed: int = 0, start_block=None, check_every: int = 0, resmode: str = "rel",
              krylov_dtype: str = "f64", max_refine: int = 0, raise_on_error: bool = True,
              X=None, form: str = "M") -> SolveResult:
        """form 'M': block Lanczos on the symmetric e^{-s} M, then the
        back-transform; form 'A': the eigenvectors of A = exp(-S_W) exp(S_B)
        directly, by block Lanczos in the exp(S_W) inner product (float64);
        form 'JD': the pairs of e^{-s} M by block Jacobi-Davidson (float64)."""
        torch = self._torch
        forms = {"M": EDA_FORM_LANCZOS_M, "A": EDA_FORM_ARNOLDI_A, "JD": EDA_FORM_JD_M}
        if form not in forms:
            raise ValueError("form must be 'M', 'A' or 'JD'")
        o = SolveOpts()
        o.form = forms[form]
        o.block = block
        o.max_basis = max_basis
        o.max_iter = max_iter
        o.resmode = EDA_RES_REL_THETA if resmode == "rel" else EDA_RES_NORMWISE
        o.krylov_dtype = _DTYPES[krylov_dtype]
        o.refine_dtype = EDA_F64
        o.max_refine = max_refine
        o.seed = seed
        o.check_every = check_every
        if start_block is not None:
            start_block = self._f64(start_block)
            o.start_block = start_block.data_ptr()
            o.ld_start = _ld(start_block)
        if X is None:
            X = _empty_cm(self.d, t, torch.float64, self.device)
        ritz = (ctypes.c_double * t)()
        rlog = (ctypes.c_double * t)()
        res = (ctypes.c_double * t)()
        info = Info()
        st = self.lib.eda_solve(self._h, t, float(tol), ctypes.byref(o), ritz, rlog,
                                X.data_ptr(), _ld(X), res, ctypes.byref(info))
        msg = self.lib.eda_last_error(self._h).decode() if st != EDA_OK else ""
        if st not in (EDA_OK, EDA_ERR_NOCONV) and raise_on_error:
            raise EDAError(st, msg)
        return SolveResult(list(ritz), list(rlog), X, list(res), info.as_dict(), st, msg)

    def autotune(self, d: int, N: int, b: int = 8, storage: str = "f64") -> dict:
        """Measure and record the launch shapes of the product passes for a
        d x N matrix in `storage` and b columns (eda_autotune)."""
        tn, nn = ctypes.c_int32(), ctypes.c_int32()
        us = (ctypes.c_double * 2)()
        self._check(self.lib.eda_autotune(self._h, int(d), int(N), int(b), _DTYPES[storage],
                                          ctypes.byref(tn), ctypes.byref(nn), us))
        return {"tn_steps": tn.value, "nn_tile": nn.value, "tn_us": us[0], "nn_us": us[1]}

    def solve_direct(self, t: int, raise_on_error: bool = True, X=None) -> SolveResult:
        """The t leading pairs by the reduced direct solve (eda_solve_direct)."""
        torch = self._torch
        if X is None:
            X = _empty_cm(self.d, t, torch.float64, self.device)
        ritz = (ctypes.c_double * t)()
        rlog = (ctypes.c_double * t)()
        res = (ctypes.c_double * t)()
        info = Info()
        st = self.lib.eda_solve_direct(self._h, t, ritz, rlog, X.data_ptr(), _ld(X), res,
                                       ctypes.byref(info))
        msg = self.lib.eda_last_error(self._h).decode() if st != EDA_OK else ""
        if st != EDA_OK and raise_on_error:
            raise EDAError(st, msg)
        return SolveResult(list(ritz), list(rlog), X, list(res), info.as_dict(), st, msg)

    def solve_batched(self, problems, storage: str = "f64", block: int = 8, max_iter: int = 0,
                      seed: int = 0, check_every: int = 0, resmode: str = "rel",
                      krylov_dtype: str = "f64", max_refine: int = 0):
        """Solve independent problems together (eda_solve_batched).

        problems: list of (H_W, H_B, t, tol) with H_W, H_B float64 CUDA
        tensors.  Returns (list of SolveResult, overall status)."""
        torch = self._torch
        cnt = len(problems)
        arr = (Problem * cnt)()
        keep = []
        outs = []
        for i, (H_W, H_B, t, tol) in enumerate(problems):
            H_W = self._f64(H_W)
            H_B = self._f64(H_B)
            d = int(H_W.shape[0])
            X = _empty_cm(d, t, torch.float64, H_W.device)
            ritz = (ctypes.c_double * t)()
            rlog = (ctypes.c_double * t)()
            res = (ctypes.c_double * t)()
            keep += [H_W, H_B]
            outs.append((X, ritz, rlog, res, t))
            arr[i] = Problem(d, int(H_W.shape[1]), int(H_B.shape[1]), H_W.data_ptr(), _ld(H_W),
                             H_B.data_ptr(), _ld(H_B), t, float(tol), ritz, rlog, X.data_ptr(),
                             _ld(X), res)
        o = SolveOpts()
        o.form = EDA_FORM_LANCZOS_M
        o.block = block
        o.max_iter = max_iter
        o.resmode = EDA_RES_REL_THETA if resmode == "rel" else EDA_RES_NORMWISE
        o.krylov_dtype = _DTYPES[krylov_dtype]
        o.refine_dtype = EDA_F64
        o.max_refine = max_refine
        o.seed = seed
        o.check_every = check_every
        infos = (Info * cnt)()
        stats = (ctypes.c_int * cnt)()
        st = self.lib.eda_solve_batched(self._h, cnt, arr, _DTYPES[storage], ctypes.byref(o),
                                        infos, stats)
        msg = self.lib.eda_last_error(self._h).decode() if st != EDA_OK else ""
        if st not in (EDA_OK, EDA_ERR_NOCONV):
            raise EDAError(st, msg)
        results = []
        for i, (X, ritz, rlog, res, t) in enumerate(outs):
            results.append(SolveResult(list(ritz), list(rlog), X, list(res), infos[i].as_dict(),
                                       int(stats[i]), msg if stats[i] != EDA_OK else ""))
        return results, st

    def gram(self):
        N = self.n + self.k
        G = _empty_cm(N, N, self._torch.float64, self.device)
        self._check(self.lib.eda_gram(self._h, G.data_ptr(), _ld(G)))
        return G

    def factor_codes(self):
        """The stored factor P = [H_W H_B] in its storage encoding: a d x (n+k)
        column-major tensor of float64 / float32 / int16 (bfloat16 codes) /
        uint8 (E4M3 codes), and for E4M3 storage the per-column scales."""
        torch = self._torch
        N = self.n + self.k
        dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.int16,
              "fp8": torch.uint8}[self.storage]
        P = _empty_cm(self.d, N, dt, self.device)
        sc = torch.empty(N, dtype=torch.float64, device=self.device) if self.storage == "fp8" \
            else None
        self._check(self.lib.eda_factor_codes(self._h, P.data_ptr(), _ld(P),
                                              sc.data_ptr() if sc is not None else None))
        return P, sc

    def nn_classify(self, X, train, train_labels, test):
        """1-NN classification in span X (Section 3.3): for every column of
        `test`, the label and index of the training column nearest in the
        distance ||X^T (x_i - y_j)||_2, and that distance (ties: smallest
        index).  X: d x t orthonormal; train: d x n_train; test: d x n_test
        (float64 CUDA); train_labels: int32 CUDA tensor of n_train entries."""
        torch = self._torch
        X, train, test = self._f64(X), self._f64(train), self._f64(test)
        if train_labels.dtype != torch.int32 or train_labels.device.type != "cuda":
            raise TypeError("train_labels: expected an int32 CUDA tensor")
        train_labels = train_labels.contiguous()
        d, t = X.shape
        n_tr, n_te = train.shape[1], test.shape[1]
        if train.shape[0] != d or test.shape[0] != d or train_labels.numel() != n_tr:
            raise ValueError("shapes of X, train, train_labels and test do not agree")
        pred = torch.empty(n_te, dtype=torch.int32, device=X.device)
        idx = torch.empty(n_te, dtype=torch.int64, device=X.device)
        dist = torch.empty(n_te, dtype=torch.float64, device=X.device)
        self._check(self.lib.eda_nn_classify(self._h, d, t, X.data_ptr(), _ld(X), n_tr,
                                             train.data_ptr(), _ld(train),
                                             train_labels.data_ptr(), n_te, test.data_ptr(),
                                             _ld(test), pred.data_ptr(), idx.data_ptr(),
                                             dist.data_ptr()))
        return pred, idx, dist

    def syev(self, A):
        A = self._f64(A)
        n = A.shape[0]
        w = self._torch.empty(n, dtype=self._torch.float64, device=A.device)
        Z = _empty_cm(n, n, self._torch.float64, A.device)
        self._check(self.lib.eda_syev(self._h, n, A.data_ptr(), _ld(A), w.data_ptr(),
                                      Z.data_ptr(), _ld(Z)))
        return w, Z
