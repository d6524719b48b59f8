"""Python binding of libfds (ctypes): argument marshalling only.

Each function carries the name of the C entry point it calls (include/fds.h).
PyTorch provides the device memory (the library allocates through torch's
caching allocator) and the stream; every computation runs in the HIP kernels
of libfds.so. There is no fallback: if the library is missing, or no GPU is
visible, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import re
import sys
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfds.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fds.h")

FDS_EFIE, FDS_MFIE, FDS_CFIE, FDS_YCFIE = 0, 1, 2, 3
FORMS = {"efie": FDS_EFIE, "mfie": FDS_MFIE, "cfie": FDS_CFIE, "ycfie": FDS_YCFIE}
FDS_FP64, FDS_FP32 = 0, 1
FDS_QR_AUTO, FDS_QR_HOUSEHOLDER = 0, 1
STATUS = {0: "FDS_OK", 1: "FDS_ERR_ARG", 2: "FDS_ERR_ALLOC", 3: "FDS_ERR_HIP",
          4: "FDS_ERR_STATE", 5: "FDS_ERR_SINGULAR", 6: "FDS_ERR_NOCONV", 7: "FDS_ERR_NOTIMPL"}


class FdsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


# ----------------------------------------------------------------- C structs
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class fds_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("user", C.c_void_p)]


class fds_asm_opts(C.Structure):
    _fields_ = [("nquad", C.c_int32), ("precision", C.c_int32), ("band_width", C.c_int32),
                ("filter_modes", C.c_int32), ("reserved", C.c_int32 * 4)]


class fds_filter_opts(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("keep_nullspace", C.c_int32), ("cluster_rtol", C.c_double)]


class fds_compress_opts(C.Structure):
    _fields_ = [("rank_cap", C.c_int32), ("oversample", C.c_int32), ("power_iters", C.c_int32),
                ("precision", C.c_int32), ("tol", C.c_double), ("seed", C.c_uint64), ("qr", C.c_int32),
                ("reserved", C.c_int32)]


class fds_solve_opts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("precision", C.c_int32), ("tol", C.c_double),
                ("unfiltered", C.c_int32), ("reserved", C.c_int32)]


class fds_problem(C.Structure):
    _fields_ = [("nodes", C.c_void_p), ("n", C.c_int64), ("k", C.c_double), ("n_modes", C.c_int32),
                ("nrhs", C.c_int32), ("angles", C.c_void_p), ("amps", C.c_void_p), ("j_out", C.c_void_p)]


class fds_batch_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("form", C.c_int32), ("alpha", C.c_double), ("rank_cap", C.c_int32),
                ("oversample", C.c_int32), ("power_iters", C.c_int32), ("sweeps", C.c_int32), ("tol", C.c_double),
                ("seed", C.c_uint64), ("reserved", C.c_int32 * 4)]


class fds_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("history", C.c_double * 32)]


_SIGS = {
    "fds_last_error": (C.c_char_p, []),
    "fds_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(fds_allocator), C.POINTER(C.c_void_p)]),
    "fds_ctx_destroy": (C.c_int, [C.c_void_p]),
    "fds_sync": (C.c_int, [C.c_void_p]),
    "fds_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "fds_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "fds_autotune": (C.c_int, [C.c_void_p, C.c_int32]),
    "fds_autotune_read": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "fds_hankel_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "fds_hankel_eval_f32": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "fds_cgemm": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_int64,
                            C.POINTER(C.c_float), C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                            C.POINTER(C.c_float), C.c_void_p, C.c_int64]),
    "fds_op_precision": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "fds_op_nband": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    "fds_op_yukawa": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "fds_farfield": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "fds_farfield_objective_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                              C.c_int64, C.c_void_p, C.POINTER(fds_solve_opts),
                                              C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.POINTER(fds_solve_stats)]),
    "fds_kernel_eval": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_int64, C.c_void_p]),
    "fds_yukawa_eval": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_int64, C.c_void_p]),
    "fds_compress_aca": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_int32)]),
    "fds_equal_chord_nodes": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_void_p, C.c_void_p]),
    "fds_zinv": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "fds_zgemm": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_int64,
                            C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                            C.POINTER(C.c_double), C.c_void_p, C.c_int64]),
    "fds_assemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                               C.POINTER(fds_asm_opts), C.POINTER(C.c_void_p)]),
    "fds_op_destroy": (C.c_int, [C.c_void_p]),
    "fds_assemble_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double), C.POINTER(C.c_void_p)]),
    "fds_op_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32)]),
    "fds_op_matrices": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p)]),
    "fds_op_sparse": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_void_p)] * 4),
    "fds_apply_gram": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "fds_filter": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.POINTER(fds_filter_opts),
                             C.POINTER(C.c_int32)]),
    "fds_filter_batch": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.c_int, C.c_double,
                                   C.POINTER(fds_filter_opts), C.POINTER(C.c_int32)]),
    "fds_op_filter_basis": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "fds_op_filter_eigenvalues": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                            C.POINTER(C.c_int32)]),
    "fds_compress": (C.c_int, [C.c_void_p, C.POINTER(fds_compress_opts), C.POINTER(C.c_int32)]),
    "fds_zqr": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                          C.POINTER(C.c_int32)]),
    "fds_op_singular_values": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                         C.POINTER(C.c_int32)]),
    "fds_op_factors": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_int32)]),
    "fds_factor": (C.c_int, [C.c_void_p]),
    "fds_rhs_planewave": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_void_p]),
    "fds_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                            C.POINTER(fds_solve_opts), C.POINTER(fds_solve_stats)]),
    "fds_rhs_system": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.c_void_p]),
    "fds_solve_system": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.POINTER(fds_solve_opts), C.POINTER(fds_solve_stats)]),
    "fds_solve_system_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32]),
    "fds_batch_create": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(fds_problem), C.POINTER(fds_batch_opts),
                                   C.POINTER(C.c_void_p)]),
    "fds_batch_replay": (C.c_int, [C.c_void_p]),
    "fds_batch_op": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    "fds_batch_destroy": (C.c_int, [C.c_void_p]),
    "fds_batch_run": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(fds_problem), C.POINTER(fds_batch_opts)]),
    "fds_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                    C.POINTER(fds_solve_opts), C.POINTER(fds_solve_stats)]),
}

_lib = None
_live = weakref.WeakSet()


def _close_all():
    # close operators, then batches (which own operators), then contexts, while
    # torch is still alive
    for o in [o for o in list(_live) if isinstance(o, Op)]:
        o.close()
    for o in [o for o in list(_live) if type(o).__name__ == "Batch"]:
        o.close()
    for o in list(_live):
        o.close()


atexit.register(_close_all)


def header_symbols() -> list[str]:
    """Entry points declared in include/fds.h."""
    with open(HEADER) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"^\s*(?:fds_status|const char\*|void)\s+(fds_\w+)\s*\(", txt, re.M)))


def lib() -> C.CDLL:
    """Load libfds.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise FdsError(st, lib().fds_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


class _DevView:
    """__cuda_array_interface__ over library-owned memory (kept alive by owner)."""

    def __init__(self, ptr, shape, typestr, owner):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2, "strides": None}
        self._owner = owner


def _view(ptr, shape, dtype, owner):
    ts = {torch.float64: "<f8", torch.complex128: "<c16", torch.complex64: "<c8", torch.float32: "<f4"}[dtype]
    v = torch.as_tensor(_DevView(ptr, shape, ts, owner), device="cuda")
    return v


# ----------------------------------------------------------------- context
class Ctx:
    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libfds runs on the device only")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._keep = []
        alloc_p = None
        if use_torch_allocator:
            dev = device

            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
                except Exception:
                    return None

            def _release(ptr, stream, user):
                torch.cuda.caching_allocator_delete(ptr)

            a = fds_allocator(_ALLOC_FN(_alloc), _RELEASE_FN(_release), None)
            self._keep += [a, a.alloc, a.release]
            alloc_p = C.byref(a)
        h = C.c_void_p()
        _check(lib().fds_ctx_create(device, C.c_void_p(self.stream.cuda_stream), alloc_p, C.byref(h)))
        self.handle = h
        _live.add(self)

    def close(self):
        if getattr(self, "handle", None):
            lib().fds_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self, _fin=sys.is_finalizing):
        # the default argument outlives the module globals at interpreter exit
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass


def fds_ctx_create(device: int = 0, stream=None) -> Ctx:
    return Ctx(device, stream)


def fds_sync(ctx: Ctx):
    _check(lib().fds_sync(ctx.handle))


def fds_profile_enable(ctx: Ctx, on: bool = True):
    _check(lib().fds_profile_enable(ctx.handle, int(bool(on))))


def fds_profile_read(ctx: Ctx, cap: int = 128) -> dict:
    """{kernel name: (total ms, launches)} accumulated since the last read."""
    names = C.create_string_buffer(32 * cap)
    tot = (C.c_double * cap)()
    cnt = (C.c_int64 * cap)()
    n = C.c_int32()
    _check(lib().fds_profile_read(ctx.handle, cap, names, tot, cnt, C.byref(n)))
    raw = names.raw
    out = {}
    for i in range(n.value):
        nm = raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
        out[nm] = (tot[i], cnt[i])
    return out


def fds_autotune(ctx: Ctx, on: bool = True):
    _check(lib().fds_autotune(ctx.handle, int(bool(on))))


def fds_autotune_read(ctx: Ctx, cap: int = 256) -> dict:
    keys = C.create_string_buffer(160 * cap)
    vals = (C.c_int32 * cap)()
    cnt = C.c_int32()
    _check(lib().fds_autotune_read(ctx.handle, cap, keys, vals, C.byref(cnt)))
    raw = keys.raw
    return {raw[160 * i:160 * (i + 1)].split(b"\0")[0].decode(): vals[i] for i in range(min(cnt.value, cap))}


def fds_hankel_eval(ctx: Ctx, x: torch.Tensor) -> torch.Tensor:
    out = torch.empty((x.numel(), 4), dtype=torch.float64, device=x.device)
    _check(lib().fds_hankel_eval(ctx.handle, _ptr(x), x.numel(), _ptr(out)))
    return out


def fds_hankel_eval_f32(ctx: Ctx, x: torch.Tensor) -> torch.Tensor:
    out = torch.empty((x.numel(), 4), dtype=torch.float32, device=x.device)
    _check(lib().fds_hankel_eval_f32(ctx.handle, _ptr(x), x.numel(), _ptr(out)))
    return out


def fds_yukawa_eval(ctx: Ctx, kappa: float, R: torch.Tensor) -> torch.Tensor:
    """(n, 2): (1/2pi) K0(kappa R) and (1/2pi)(K0(kappa R) + log R)."""
    R = R.to(device="cuda", dtype=torch.float64).contiguous()
    out = torch.empty((R.numel(), 2), dtype=torch.float64, device="cuda")
    _check(lib().fds_yukawa_eval(ctx.handle, float(kappa), _ptr(R), R.numel(), _ptr(out)))
    return out


def fds_equal_chord_nodes(trig, n: int):
    """Equal-chord mesh of the trigonometric-polynomial curve trig = (ax, bx, ay, by)
    (host call, no GPU needed): returns (nodes (n, 2) numpy array, chord length)."""
    import numpy as np
    ax, bx, ay, by = (np.ascontiguousarray(v, dtype=np.float64) for v in trig)
    d = ax.size - 1
    if not (bx.size == ay.size == by.size == d + 1):
        raise ValueError("coefficient arrays of different lengths")
    nodes = np.empty((int(n), 2), dtype=np.float64)
    chord = C.c_double(0.0)
    _check(lib().fds_equal_chord_nodes(d, ax.ctypes.data, bx.ctypes.data, ay.ctypes.data, by.ctypes.data,
                                       int(n), nodes.ctypes.data, C.addressof(chord)))
    return nodes, chord.value


def fds_kernel_eval(ctx: Ctx, k: float, R: torch.Tensor) -> torch.Tensor:
    out = torch.empty((R.numel(), 8), dtype=torch.float64, device=R.device)
    _check(lib().fds_kernel_eval(ctx.handle, float(k), _ptr(R), R.numel(), _ptr(out)))
    return out


def fds_zinv(ctx: Ctx, A: torch.Tensor):
    """Inverse of the square complex128 column-major matrix held by A (shape (r, r),
    the matrix is A.T); returns (Ainv in the same layout, (min |pivot|, max |A|))."""
    r = A.shape[0]
    assert A.dtype == torch.complex128 and A.is_contiguous() and A.shape == (r, r)
    out = torch.empty_like(A)
    st = (C.c_double * 2)()
    _check(lib().fds_zinv(ctx.handle, r, _ptr(A), _ptr(out), st))
    return out, (st[0], st[1])


def fds_zqr(ctx: Ctx, A: torch.Tensor, method: int = FDS_QR_AUTO):
    """QR of the M x m complex128 column-major matrix held by A (shape (m, M), the
    matrix is A.T). A is overwritten (R in its upper triangle); returns (Q in the
    same layout, whether the Householder factorisation produced it)."""
    m, M = A.shape
    assert A.dtype == torch.complex128 and A.is_contiguous()
    Q = torch.empty_like(A)
    used = C.c_int32()
    _check(lib().fds_zqr(ctx.handle, M, m, _ptr(A), _ptr(Q), int(method), C.byref(used)))
    return Q, bool(used.value)


def fds_zgemm(ctx: Ctx, opa: int, opb: int, A: torch.Tensor, Bm: torch.Tensor, Cm: torch.Tensor,
              alpha: complex = 1.0, beta: complex = 0.0):
    """Cm = alpha op(A) op(Bm) + beta Cm on column-major views.

    The tensors hold column-major matrices, i.e. C-contiguous tensors of shape
    (cols, rows): the matrix is t.T. Returns Cm."""
    ra, ca = A.shape[1], A.shape[0]
    rb, cb = Bm.shape[1], Bm.shape[0]
    m = ra if opa == 0 else ca
    k = ca if opa == 0 else ra
    n = cb if opb == 0 else rb
    al = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (C.c_double * 2)(complex(beta).real, complex(beta).imag)
    _check(lib().fds_zgemm(ctx.handle, opa, opb, m, n, k, al, _ptr(A), ra, _ptr(Bm), rb, be,
                           _ptr(Cm), Cm.shape[1]))
    return Cm


def fds_cgemm(ctx: Ctx, opa: int, opb: int, A: torch.Tensor, Bm: torch.Tensor, Cm: torch.Tensor,
              alpha: complex = 1.0, beta: complex = 0.0):
    """fds_zgemm for complex64 tensors (FP32 matrix cores)."""
    ra, ca = A.shape[1], A.shape[0]
    rb, cb = Bm.shape[1], Bm.shape[0]
    m = ra if opa == 0 else ca
    k = ca if opa == 0 else ra
    n = cb if opb == 0 else rb
    al = (C.c_float * 2)(complex(alpha).real, complex(alpha).imag)
    be = (C.c_float * 2)(complex(beta).real, complex(beta).imag)
    _check(lib().fds_cgemm(ctx.handle, opa, opb, m, n, k, al, _ptr(A), ra, _ptr(Bm), rb, be,
                           _ptr(Cm), Cm.shape[1]))
    return Cm


# ----------------------------------------------------------------- operator
class Op:
    def __init__(self, ctx: Ctx, handle):
        self.ctx = ctx
        self.handle = handle
        _live.add(self)

    def close(self):
        if getattr(self, "handle", None):
            lib().fds_op_destroy(self.handle)
            self.handle = None

    def __del__(self, _fin=sys.is_finalizing):
        # the default argument outlives the module globals at interpreter exit
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n = C.c_int64()
        ne = C.c_int32()
        r = C.c_int32()
        _check(lib().fds_op_info(self.handle, C.byref(n), C.byref(ne), C.byref(r)))
        return n.value, ne.value, r.value

    @property
    def n(self) -> int:
        return self.info()[0]


def fds_assemble(ctx: Ctx, nodes: torch.Tensor, k: float, opts: fds_asm_opts | None = None,
                 precision: str | None = None, band_width: int = 0, filter_modes: int = 0) -> Op:
    """precision: "fp64" (default) or "fp32" (complex64 operators, mixed precision);
    band_width: FP32 only, half-width of the FP64 band of N (0: the library's default);
    filter_modes: the filtering point of a coming fds_filter (null mode kept), whose
    eigensolver then starts here, beside the dense assembly (0: none)."""
    nodes = nodes.to(device="cuda", dtype=torch.float64).contiguous()
    if precision is not None or filter_modes:
        opts = fds_asm_opts()
        opts.nquad = 8
        opts.precision = {"fp64": FDS_FP64, "fp32": FDS_FP32}[precision or "fp64"]
        opts.band_width = int(band_width)
        opts.filter_modes = int(filter_modes)
    h = C.c_void_p()
    _check(lib().fds_assemble(ctx.handle, _ptr(nodes), nodes.shape[0], float(k),
                              C.byref(opts) if opts is not None else None, C.byref(h)))
    return Op(ctx, h)


def fds_assemble_batch(ctx: Ctx, nodes_list, ks) -> list:
    """Assemble several FP64 operators with one persistent far-field launch."""
    nodes_list = [x.to(device="cuda", dtype=torch.float64).contiguous() for x in nodes_list]
    cnt = len(nodes_list)
    ptrs = (C.c_void_p * cnt)(*[_ptr(x) for x in nodes_list])
    ns = (C.c_int64 * cnt)(*[x.shape[0] for x in nodes_list])
    kk = (C.c_double * cnt)(*[float(v) for v in ks])
    hs = (C.c_void_p * cnt)()
    _check(lib().fds_assemble_batch(ctx.handle, cnt, ptrs, ns, kk, hs))
    return [Op(ctx, C.c_void_p(h)) for h in hs]


def fds_op_matrices(op: Op):
    s, n_, d = C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(lib().fds_op_matrices(op.handle, C.byref(s), C.byref(n_), C.byref(d)))
    N = op.n
    dt = torch.complex64 if fds_op_precision(op) == FDS_FP32 else torch.complex128
    return tuple(_view(p.value, (N, N), dt, op) for p in (s, n_, d))


def fds_op_nband(op: Op):
    """FP32 operators: (band, w) with the complex128 band of N as an (n, 2w + 1)
    tensor (N[i][(i + d) mod n] at [i][d + w]); (None, 0) otherwise."""
    p = C.c_void_p()
    w = C.c_int32()
    _check(lib().fds_op_nband(op.handle, C.byref(p), C.byref(w)))
    if not p.value:
        return None, 0
    return _view(p.value, (op.n, 2 * w.value + 1), torch.complex128, op), w.value


def fds_op_yukawa(op: Op):
    """The Yukawa single layer (n, n) complex128 view, or None before it is built."""
    p = C.c_void_p()
    _check(lib().fds_op_yukawa(op.handle, C.byref(p)))
    if not p.value:
        return None
    return _view(p.value, (op.n, op.n), torch.complex128, op)


def fds_op_precision(op: Op) -> int:
    p = C.c_int32()
    _check(lib().fds_op_precision(op.handle, C.byref(p)))
    return p.value


def fds_op_sparse(op: Op):
    ps = [C.c_void_p() for _ in range(4)]
    _check(lib().fds_op_sparse(op.handle, *[C.byref(p) for p in ps]))
    N = op.n
    return tuple(_view(p.value, (N,), torch.float64, op) for p in ps)


def fds_apply_gram(op: Op, p: int, X: torch.Tensor):
    _check(lib().fds_apply_gram(op.handle, int(p), _ptr(X), X.numel() // op.n))
    return X


def fds_filter(op: Op, form: str = "efie", alpha: float = 1.0, n_modes: int = 21,
               keep_nullspace: bool = True, cluster_rtol: float = 1e-6) -> int:
    o = fds_filter_opts(int(n_modes), int(bool(keep_nullspace)), float(cluster_rtol))
    ne = C.c_int32()
    _check(lib().fds_filter(op.handle, FORMS[form], float(alpha), C.byref(o), C.byref(ne)))
    return ne.value


def fds_filter_batch(ops: list, form: str = "efie", alpha: float = 1.0, n_modes=21,
                     keep_nullspace: bool = True, cluster_rtol: float = 1e-6) -> list:
    """fds_filter on several operators (grouped GEMMs); returns the kept mode counts."""
    cnt = len(ops)
    nms = list(n_modes) if hasattr(n_modes, "__len__") else [n_modes] * cnt
    opts = (fds_filter_opts * cnt)(*[fds_filter_opts(int(m), int(bool(keep_nullspace)), float(cluster_rtol))
                                     for m in nms])
    hs = (C.c_void_p * cnt)(*[o.handle.value if isinstance(o.handle, C.c_void_p) else o.handle for o in ops])
    ne = (C.c_int32 * cnt)()
    _check(lib().fds_filter_batch(cnt, hs, FORMS[form], float(alpha), opts, ne))
    return list(ne)


def fds_op_filter_basis(op: Op) -> torch.Tensor:
    p = C.c_void_p()
    _check(lib().fds_op_filter_basis(op.handle, C.byref(p)))
    n, ne, _ = op.info()
    return _view(p.value, (ne, n), torch.float64, op)


def fds_op_filter_eigenvalues(op: Op, cap: int = 4096):
    buf = (C.c_double * cap)()
    cnt = C.c_int32()
    _check(lib().fds_op_filter_eigenvalues(op.handle, buf, cap, C.byref(cnt)))
    return [buf[i] for i in range(cnt.value)]


def fds_compress(op: Op, rank_cap: int, oversample: int = 10, power_iters: int = 2,
                 tol: float = 0.0, seed: int = 0, precision: int = FDS_FP64, qr: int = 0) -> int:
    """qr: FDS_QR_AUTO (0) or FDS_QR_HOUSEHOLDER (1)."""
    o = fds_compress_opts(int(rank_cap), int(oversample), int(power_iters), int(precision),
                          float(tol), C.c_uint64(seed & ((1 << 64) - 1)), int(qr), 0)
    r = C.c_int32()
    _check(lib().fds_compress(op.handle, C.byref(o), C.byref(r)))
    return r.value


def fds_compress_aca(op: Op, rank_cap: int, tol: float = 0.0) -> int:
    """Skeleton by adaptive cross approximation (partial pivoting); returns the rank."""
    r = C.c_int32()
    _check(lib().fds_compress_aca(op.handle, int(rank_cap), float(tol), C.byref(r)))
    return r.value


def fds_op_singular_values(op: Op, cap: int = 4096):
    buf = (C.c_double * cap)()
    cnt = C.c_int32()
    _check(lib().fds_op_singular_values(op.handle, buf, cap, C.byref(cnt)))
    return [buf[i] for i in range(cnt.value)]


def fds_op_factors(op: Op):
    u, w, r = C.c_void_p(), C.c_void_p(), C.c_int32()
    _check(lib().fds_op_factors(op.handle, C.byref(u), C.byref(w), C.byref(r)))
    n = op.n
    return (_view(u.value, (r.value, n), torch.complex128, op),
            _view(w.value, (r.value, n), torch.complex128, op))


def fds_factor(op: Op):
    _check(lib().fds_factor(op.handle))


def fds_rhs_planewave(op: Op, angles: torch.Tensor, amps: torch.Tensor):
    n = op.n
    nrhs = angles.numel()
    angles = angles.to(device="cuda", dtype=torch.float64).contiguous()
    amps = amps.to(device="cuda", dtype=torch.complex128).contiguous()
    f = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
    h = torch.empty_like(f)
    _check(lib().fds_rhs_planewave(op.handle, _ptr(angles), _ptr(amps), nrhs, _ptr(f), _ptr(h)))
    return f, h


def fds_solve(op: Op, f: torch.Tensor | None, h: torch.Tensor | None, max_iters: int = 4,
              tol: float = 1e-12, want_y: bool = False, stats: bool = True, unfiltered: bool = False):
    ref = f if f is not None else h
    nrhs = ref.shape[0]
    j = torch.empty((nrhs, op.n), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(j) if want_y else None
    o = fds_solve_opts(int(max_iters), FDS_FP64, float(tol), int(bool(unfiltered)), 0)
    st = fds_solve_stats()
    _check(lib().fds_solve(op.handle, _ptr(f), _ptr(h), nrhs, _ptr(j), _ptr(y), C.byref(o),
                           C.byref(st) if stats else None))
    hist = list(st.history[: st.iters + 1]) if stats else []
    return j, y, {"iters": st.iters, "converged": bool(st.converged), "relres": st.relres,
                  "history": hist}


def fds_rhs_system(op: Op, form: str, alpha: float, f: torch.Tensor | None,
                   h: torch.Tensor | None) -> torch.Tensor:
    """w (nrhs, n): the right-hand side in current coefficients for `form` (valid
    from the assembled stage on; asynchronous)."""
    ref = f if f is not None else h
    w = torch.empty((ref.shape[0], op.n), dtype=torch.complex128, device="cuda")
    _check(lib().fds_rhs_system(op.handle, FORMS[form], float(alpha), _ptr(f), _ptr(h), ref.shape[0], _ptr(w)))
    return w


def fds_solve_system(op: Op, w: torch.Tensor, max_iters: int = 4, tol: float = 1e-12, want_y: bool = False,
                     stats: bool = True, unfiltered: bool = False):
    """fds_solve from w = fds_rhs_system(...); same outputs as fds_solve."""
    nrhs = w.shape[0]
    j = torch.empty((nrhs, op.n), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(j) if want_y else None
    o = fds_solve_opts(int(max_iters), FDS_FP64, float(tol), int(bool(unfiltered)), 0)
    st = fds_solve_stats()
    _check(lib().fds_solve_system(op.handle, _ptr(w), nrhs, _ptr(j), _ptr(y), C.byref(o),
                                  C.byref(st) if stats else None))
    hist = list(st.history[: st.iters + 1]) if stats else []
    return j, y, {"iters": st.iters, "converged": bool(st.converged), "relres": st.relres,
                  "history": hist}


def fds_solve_adjoint(op: Op, v: torch.Tensor, max_iters: int = 4, tol: float = 1e-12, want_u: bool = False,
                      stats: bool = True, unfiltered: bool = False):
    """Solves (beta I + P C)^H y = v (unfiltered: (beta I + C)^H y = v) for the rows of
    v (nrhs, n); returns (y, u = G^{-1/2} y or None, stats)."""
    v = v.to(device="cuda", dtype=torch.complex128).contiguous()
    y = torch.empty_like(v)
    u = torch.empty_like(v) if want_u else None
    o = fds_solve_opts(int(max_iters), FDS_FP64, float(tol), int(bool(unfiltered)), 0)
    st = fds_solve_stats()
    _check(lib().fds_solve_adjoint(op.handle, _ptr(v), v.shape[0], _ptr(y), _ptr(u), C.byref(o),
                                   C.byref(st) if stats else None))
    hist = list(st.history[: st.iters + 1]) if stats else []
    return y, u, {"iters": st.iters, "converged": bool(st.converged), "relres": st.relres, "history": hist}


def fds_solve_system_noalloc(op: Op, w: torch.Tensor, j_out: torch.Tensor, sweeps: int = 2) -> torch.Tensor:
    """Allocation-free Woodbury solve with `sweeps` filtered refinement sweeps into the
    caller's j_out (nrhs, n); asynchronous on the context's stream."""
    if w.shape != j_out.shape or w.dtype != torch.complex128 or j_out.dtype != torch.complex128:
        raise ValueError("w and j_out must be complex128 tensors of the same shape")
    _check(lib().fds_solve_system_noalloc(op.handle, _ptr(w), w.shape[0], _ptr(j_out), int(sweeps)))
    return j_out


# ----------------------------------------------------------------- batches
class _BorrowedOp(Op):
    """An operator owned by a batch (never destroyed through this handle)."""

    def close(self):
        self.handle = None


def _batch_args(problems, precision, form, alpha, rank_cap, oversample, power_iters, sweeps, tol, seed):
    keep = []
    arr = (fds_problem * len(problems))()
    for i, p in enumerate(problems):
        nodes = p["nodes"].to(device="cuda", dtype=torch.float64).contiguous()
        ang, amp, jo = p["angles"], p["amps"], p["j_out"]
        if ang.dtype != torch.float64 or not ang.is_cuda or not ang.is_contiguous():
            raise ValueError("angles must be contiguous float64 CUDA tensors")
        if amp.dtype != torch.complex128 or not amp.is_cuda or not amp.is_contiguous() or amp.numel() != ang.numel():
            raise ValueError("amps must be contiguous complex128 CUDA tensors, one per angle")
        if jo.dtype != torch.complex128 or not jo.is_cuda or tuple(jo.shape) != (ang.numel(), nodes.shape[0]):
            raise ValueError("j_out must be a complex128 CUDA tensor of shape (nrhs, n)")
        keep += [nodes, ang, amp, jo]
        arr[i] = fds_problem(_ptr(nodes), nodes.shape[0], float(p["k"]), int(p["n_modes"]), ang.numel(),
                             _ptr(ang), _ptr(amp), _ptr(jo))
    o = fds_batch_opts()
    o.precision = {"fp64": FDS_FP64, "fp32": FDS_FP32}[precision]
    o.form = FORMS[form]
    o.alpha = float(alpha)
    o.rank_cap, o.oversample, o.power_iters = int(rank_cap), int(oversample), int(power_iters)
    o.sweeps, o.tol, o.seed = int(sweeps), float(tol), int(seed)
    return arr, o, keep


class Batch:
    """fds_batch_create: operators of every problem built and factored, the solves
    of all problems recorded in one graph. problems: list of dicts with nodes
    (n, 2), k, n_modes and the caller-owned CUDA tensors angles (nrhs,) float64,
    amps (nrhs,) complex128 and j_out (nrhs, n) complex128, which every replay()
    reads (angles, amps) and writes (j_out)."""

    def __init__(self, ctx: Ctx, problems, precision="fp64", form="cfie", alpha=1.0, rank_cap=0, oversample=10,
                 power_iters=2, sweeps=0, tol=0.0, seed=1):
        self.ctx = ctx
        arr, o, self._keep = _batch_args(problems, precision, form, alpha, rank_cap, oversample, power_iters,
                                         sweeps, tol, seed)
        h = C.c_void_p()
        _check(lib().fds_batch_create(ctx.handle, len(problems), arr, C.byref(o), C.byref(h)))
        self.handle = h
        self.outputs = [p["j_out"] for p in problems]
        _live.add(self)

    def replay(self):
        _check(lib().fds_batch_replay(self.handle))
        return self.outputs

    def op(self, i: int) -> Op:
        h = C.c_void_p()
        _check(lib().fds_batch_op(self.handle, int(i), C.byref(h)))
        return _BorrowedOp(self.ctx, h)

    def close(self):
        if getattr(self, "handle", None):
            lib().fds_batch_destroy(self.handle)
            self.handle = None

    def __del__(self, _fin=sys.is_finalizing):
        # the default argument outlives the module globals at interpreter exit
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass


def fds_batch_run(ctx: Ctx, problems, precision="fp64", form="cfie", alpha=1.0, rank_cap=0, oversample=10,
                  power_iters=2, sweeps=0, tol=0.0, seed=1):
    """All problems solved end to end by one call (set-up, one graph launch); the
    solutions are in each problem's j_out when it returns."""
    arr, o, keep = _batch_args(problems, precision, form, alpha, rank_cap, oversample, power_iters, sweeps, tol,
                               seed)
    _check(lib().fds_batch_run(ctx.handle, len(problems), arr, C.byref(o)))
    return [p["j_out"] for p in problems]


# ----------------------------------------------------------------- inverse problem
def fds_farfield(op: Op, j: torch.Tensor, thetas: torch.Tensor) -> torch.Tensor:
    """Far fields (nrhs, nang) of currents j (nrhs, n)."""
    j = j.to(device="cuda", dtype=torch.complex128).contiguous()
    thetas = thetas.to(device="cuda", dtype=torch.float64).contiguous()
    out = torch.empty((j.shape[0], thetas.numel()), dtype=torch.complex128, device="cuda")
    _check(lib().fds_farfield(op.handle, _ptr(j), j.shape[0], _ptr(thetas), thetas.numel(), _ptr(out)))
    return out


def fds_farfield_objective_grad(op: Op, angles: torch.Tensor, amps: torch.Tensor, thetas: torch.Tensor,
                                target: torch.Tensor, max_iters: int = 8, tol: float = 1e-12):
    """(J, dJ/dnodes (n, 2), dJ/dRe A + i dJ/dIm A (nrhs,), far fields (nrhs, nang), stats)."""
    angles = angles.to(device="cuda", dtype=torch.float64).contiguous()
    amps = amps.to(device="cuda", dtype=torch.complex128).contiguous()
    thetas = thetas.to(device="cuda", dtype=torch.float64).contiguous()
    target = target.to(device="cuda", dtype=torch.complex128).contiguous()
    nrhs, nang = angles.numel(), thetas.numel()
    assert target.shape == (nrhs, nang)
    gn = torch.empty((op.n, 2), dtype=torch.float64, device="cuda")
    ga = torch.empty((nrhs,), dtype=torch.complex128, device="cuda")
    ff = torch.empty((nrhs, nang), dtype=torch.complex128, device="cuda")
    o = fds_solve_opts(int(max_iters), FDS_FP64, float(tol), 1, 0)
    st = fds_solve_stats()
    J = C.c_double()
    _check(lib().fds_farfield_objective_grad(op.handle, _ptr(angles), _ptr(amps), nrhs, _ptr(thetas), nang,
                                             _ptr(target), C.byref(o), C.byref(J), _ptr(gn), _ptr(ga),
                                             _ptr(ff), C.byref(st)))
    stats = {"iters": st.iters, "converged": bool(st.converged), "relres": st.relres}
    return J.value, gn, ga, ff, stats

