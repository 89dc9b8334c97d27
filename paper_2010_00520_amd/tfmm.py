"""ctypes binding of libtfmm (include/tfmm.h): argument marshalling only.

Every computation runs inside libtfmm's HIP kernels.  torch supplies device
buffers (complex64 tensors) and streams.  There is no CPU fallback: if the
library is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtfmm.so")

FORMATS = {"full": 0, "tucker3d": 1, "tt3d": 2, "tucker4d": 3, "tt4d": 4, "htucker4d": 5}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}
PRECISIONS = {"fp32": 0, "bf16x3": 1}
NEAR = {"cheb": 0, "kappa": 1}

STATUS = {
    0: "ok", 1: "invalid argument", 2: "unsupported", 3: "device-memory budget exhausted",
    4: "out of memory", 5: "HIP error", 6: "operator busy", 7: "unknown ticket", 8: "queue full",
    9: "internal error", 10: "no HIP device", 11: "iterative solve did not converge",
}


class TfmmError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


class Problem(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32 * 3),
        ("box_size", ctypes.c_double),
        ("k_re", ctypes.c_double),
        ("k_im", ctypes.c_double),
        ("L", ctypes.c_int32),
        ("digits", ctypes.c_double),
        ("n_theta", ctypes.c_int32),
        ("n_phi", ctypes.c_int32),
        ("dirs", ctypes.POINTER(ctypes.c_double)),
        ("n_dir", ctypes.c_int32),
        ("near_rule", ctypes.c_int),
        ("near_param", ctypes.c_double),
        ("scale_re", ctypes.c_double),
        ("scale_im", ctypes.c_double),
        ("fmt", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("prec", ctypes.c_int),
    ]


class OpInfo(ctypes.Structure):
    _fields_ = [
        ("fmt", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("K", ctypes.c_int32 * 3),
        ("n", ctypes.c_int32 * 3),
        ("n_dir", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("bytes_full", ctypes.c_size_t),
        ("bytes_stored", ctypes.c_size_t),
        ("elems_stored", ctypes.c_size_t),
        ("bytes_scratch", ctypes.c_size_t),
        ("rel_err_fro", ctypes.c_double),
        ("max_dir_rel_err", ctypes.c_double),
        ("ranks", ctypes.c_int32 * 8),
        ("setup_seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {
            "fmt": FORMAT_NAMES.get(self.fmt, self.fmt), "prec": self.prec, "K": tuple(self.K), "n": tuple(self.n),
            "n_dir": self.n_dir, "L": self.L, "bytes_full": self.bytes_full, "bytes_stored": self.bytes_stored,
            "elems_stored": self.elems_stored, "bytes_scratch": self.bytes_scratch, "rel_err_fro": self.rel_err_fro,
            "max_dir_rel_err": self.max_dir_rel_err, "ranks": tuple(self.ranks),
            "setup_seconds": self.setup_seconds,
        }


_VP = ctypes.c_void_p
_ST = ctypes.c_int

# (name, restype, argtypes) for every entry point declared in include/tfmm.h
SIGNATURES = [
    ("tfmm_ctx_create", _ST, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_VP)]),
    ("tfmm_ctx_destroy", _ST, [_VP]),
    ("tfmm_ctx_memory", _ST, [_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    ("tfmm_setup_compressed", _ST, [_VP, ctypes.POINTER(Problem), ctypes.POINTER(_VP)]),
    ("tfmm_op_import", _ST, [_VP, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t,
                             ctypes.POINTER(ctypes.c_double), ctypes.c_size_t, ctypes.POINTER(_VP)]),
    ("tfmm_op_info_get", _ST, [_VP, ctypes.POINTER(OpInfo)]),
    ("tfmm_op_ranks", _ST, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    ("tfmm_op_export", _ST, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    ("tfmm_op_release", _ST, [_VP, _VP]),
    ("tfmm_translate", _ST, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("tfmm_translate_noalloc", _ST, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("tfmm_submit", _ST, [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    ("tfmm_poll", _ST, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int),
                        ctypes.POINTER(ctypes.c_double)]),
    ("tfmm_wait", _ST, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    ("tfmm_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("tfmm_last_error", ctypes.c_char_p, []),
    ("tfmm_set_profiling", _ST, [_VP, ctypes.c_int32]),
    ("tfmm_kernel_times", _ST, [_VP, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("tfmm_autotune", _ST, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_double)]),
    ("tfmm_op_plan", _ST, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t]),
    ("tfmm_sched_stats", _ST, [_VP, ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t]),
    ("tfmm_basis_setup", _ST, [_VP, _VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_VP)]),
    ("tfmm_basis_release", _ST, [_VP, _VP]),
    ("tfmm_aggregate", _ST, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("tfmm_disaggregate", _ST, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("tfmm_farfield_matvec", _ST, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("tfmm_near_setup", _ST, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_VP)]),
    ("tfmm_near_release", _ST, [_VP, _VP]),
    ("tfmm_near_matvec", _ST, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("tfmm_solve_tfqmr", _ST, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtfmm and declare its signatures.  Raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtfmm not built ({path} missing); run paper_2010_00520_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise TfmmError(status, load().tfmm_last_error().decode())


def make_problem(K, box=0.5, k=2 * np.pi, L=0, digits=0.0, fmt="full", tol=1e-4, prec="fp32", near="cheb",
                 near_param=0.0, n_theta=0, n_phi=0, scale=1.0 + 0j, dirs=None, n_dir=0) -> Problem:
    """tfmm_problem from keyword arguments.  `k` may be complex (lossy medium,
    Im k < 0); `dirs` an (n_dir, 3) array of unit vectors replacing the direction
    grid (the returned Problem keeps a reference to its buffer)."""
    p = Problem()
    p.K[:] = [int(x) for x in K]
    p.box_size = float(box)
    p.k_re, p.k_im = float(np.real(k)), float(np.imag(k))
    p.L = int(L)
    p.digits = float(digits)
    p.n_theta, p.n_phi = int(n_theta), int(n_phi)
    if dirs is not None:
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        p._dirs_keep = d
        p.dirs = d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.n_dir = d.shape[0]
    else:
        p.n_dir = int(n_dir)
    p.near_rule = NEAR[near]
    p.near_param = float(near_param)
    p.scale_re, p.scale_im = float(np.real(scale)), float(np.imag(scale))
    p.fmt = FORMATS[fmt]
    p.tol = float(tol)
    p.prec = PRECISIONS[prec]
    return p


def _dev_ptr(t) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if t.dtype != torch.complex64 or not t.is_contiguous():
        raise TypeError("expected a contiguous complex64 tensor")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Operator:
    def __init__(self, ctx: "Context", handle: int):
        self.ctx = ctx
        self.handle = ctypes.c_void_p(handle)
        inf = self.info()
        # per-RHS block shape of A and B: (n_dir, Kx, Ky, Kz)
        self.block = (inf["n_dir"],) + tuple(inf["K"])

    def check_io(self, A, B) -> int:
        """Raise unless A and B are [nrhs, n_dir, Kx, Ky, Kz] complex64 device tensors
        of this operator with the same nrhs; returns nrhs."""
        for name, t in (("A", A), ("B", B)):
            if tuple(t.shape[1:]) != self.block or t.dim() != 5:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, operator needs [nrhs, {', '.join(map(str, self.block))}]")
        if A.shape[0] != B.shape[0] or A.shape[0] < 1:
            raise ValueError("A and B must hold the same number (>= 1) of right-hand sides")
        return int(A.shape[0])

    def info(self) -> dict:
        inf = OpInfo()
        _check(load().tfmm_op_info_get(self.handle, ctypes.byref(inf)))
        return inf.as_dict()

    def plan(self) -> dict:
        """Current tile plan: fused path, three-pass cb, register-chained restoration, tuned,
        x-mode product formed ahead of the z-stage (4-D formats)."""
        v = (ctypes.c_int32 * 5)()
        _check(load().tfmm_op_plan(self.handle, v, 5))
        return {"fused": bool(v[0]), "cb": int(v[1]), "register_chained": bool(v[2]), "tuned": bool(v[3]),
                "w1_formed": bool(v[4])}

    def ranks(self) -> np.ndarray:
        need = ctypes.c_size_t()
        _check(load().tfmm_op_ranks(self.handle, None, 0, ctypes.byref(need)))
        buf = (ctypes.c_int32 * max(1, need.value))()
        _check(load().tfmm_op_ranks(self.handle, buf, need.value, ctypes.byref(need)))
        return np.array(buf[: need.value], dtype=np.int32)

    def export(self) -> np.ndarray:
        need = ctypes.c_size_t()
        _check(load().tfmm_op_export(self.handle, None, 0, ctypes.byref(need)))
        arr = np.empty(need.value, dtype=np.float64)
        _check(load().tfmm_op_export(self.handle, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), need.value,
                                     ctypes.byref(need)))
        return arr.view(np.complex128)

    def release(self):
        if self.handle:
            _check(load().tfmm_op_release(self.ctx.handle, self.handle))
            self.handle = ctypes.c_void_p(0)


class Basis:
    """Point-dipole basis functions of the far-field product (tfmm_basis_setup)."""

    def __init__(self, ctx: "Context", op: "Operator", handle: int, n: int):
        self.ctx, self.op, self.handle, self.n = ctx, op, ctypes.c_void_p(handle), n

    def release(self):
        if self.handle:
            _check(load().tfmm_basis_release(self.ctx.handle, self.handle))
            self.handle = ctypes.c_void_p(0)


class NearField:
    """Near-field matrix of the system (CSR, tfmm_near_setup)."""

    def __init__(self, ctx: "Context", handle: int, n: int):
        self.ctx, self.handle, self.n = ctx, ctypes.c_void_p(handle), n

    def release(self):
        if self.handle:
            _check(load().tfmm_near_release(self.ctx.handle, self.handle))
            self.handle = ctypes.c_void_p(0)


def _check_vec(t, shape, name):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _dev_ptr(t)


class Context:
    """One GPU, one device-memory budget, one scheduler."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.tfmm_ctx_create(int(device), int(budget_bytes), ctypes.byref(h)))
        self.handle = h
        self._live = {}  # ticket -> (A, B) of submitted jobs not yet reported done

    def close(self):
        if self.handle:
            _check(load().tfmm_ctx_destroy(self.handle))
            self.handle = ctypes.c_void_p(0)
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def memory(self) -> Tuple[int, int]:
        u, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().tfmm_ctx_memory(self.handle, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    def setup(self, **kw) -> Operator:
        prob = make_problem(**kw)
        h = ctypes.c_void_p()
        _check(load().tfmm_setup_compressed(self.handle, ctypes.byref(prob), ctypes.byref(h)))
        return Operator(self, h.value)

    def import_factors(self, K, L, fmt: str, ranks: Sequence[int], data: np.ndarray, prec="fp32", n_theta=0,
                       n_phi=0, n_dir=0, tol=0.0) -> Operator:
        """tfmm_op_import; `tol`: the tolerance the factors were compressed at (0: unknown)."""
        prob = make_problem(K, L=L, fmt=fmt, prec=prec, n_theta=n_theta, n_phi=n_phi, n_dir=n_dir, tol=tol)
        r = np.ascontiguousarray(np.asarray(ranks, dtype=np.int32).ravel())
        d = np.ascontiguousarray(np.asarray(data, dtype=np.complex128).ravel()).view(np.float64)
        h = ctypes.c_void_p()
        _check(load().tfmm_op_import(self.handle, ctypes.byref(prob),
                                     r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), r.size,
                                     d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d.size, ctypes.byref(h)))
        return Operator(self, h.value)

    def translate(self, op: Operator, A, B, stream=None):
        """Enqueue B = translate(A) on `stream` (torch stream; default: current)."""
        nrhs = op.check_io(A, B)
        _check(load().tfmm_translate(self.handle, op.handle, ctypes.c_void_p(_dev_ptr(A)),
                                     ctypes.c_void_p(_dev_ptr(B)), nrhs, ctypes.c_void_p(_stream_handle(stream))))

    def translate_noalloc(self, op: Operator, A, B, stream=None):
        """tfmm_translate_noalloc: the same translation with the library's fixed
        device scratch (no device allocation; calls on one device must not overlap)."""
        nrhs = op.check_io(A, B)
        _check(load().tfmm_translate_noalloc(self.handle, op.handle, ctypes.c_void_p(_dev_ptr(A)),
                                             ctypes.c_void_p(_dev_ptr(B)), nrhs,
                                             ctypes.c_void_p(_stream_handle(stream))))

    def submit(self, op: Operator, A, B) -> int:
        """Queue a job for the scheduler.  The scheduler's streams do not wait for
        torch's, so the current stream is synchronised first (A must be complete
        when the job is submitted); A and B are kept alive until poll or wait
        reports the job done."""
        import torch

        nrhs = op.check_io(A, B)
        a, b = _dev_ptr(A), _dev_ptr(B)
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check(load().tfmm_submit(self.handle, op.handle, ctypes.c_void_p(a), ctypes.c_void_p(b), nrhs,
                                  ctypes.byref(t)))
        self._live[t.value] = (A, B)
        return t.value

    def poll(self, ticket: int):
        done, st, lat = ctypes.c_int32(), ctypes.c_int(), ctypes.c_double()
        _check(load().tfmm_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(lat)))
        if done.value:
            self._live.pop(ticket, None)
        return bool(done.value), st.value, lat.value

    def wait(self, ticket: int):
        st, lat = ctypes.c_int(), ctypes.c_double()
        _check(load().tfmm_wait(self.handle, ticket, ctypes.byref(st), ctypes.byref(lat)))
        self._live.pop(ticket, None)
        return st.value, lat.value

    def autotune(self, op: "Operator", nrhs: int = 1, reps: int = 20):
        """Time the admissible tile configurations for `nrhs` RHS and adopt the fastest.
        Returns (plan dict, best median ms)."""
        ch = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double()
        _check(load().tfmm_autotune(self.handle, op.handle, int(nrhs), int(reps), ch, ctypes.byref(ms)))
        return {"fused": bool(ch[0]), "cb": int(ch[1]), "register_chained": bool(ch[2])}, ms.value

    def sched_stats(self) -> dict:
        """Scheduler counters: launches, memory waits, jobs done, jobs failed, queued."""
        v = (ctypes.c_uint64 * 5)()
        _check(load().tfmm_sched_stats(self.handle, v, 5))
        return dict(zip(("launches", "memory_waits", "done", "failed", "queued"), (int(x) for x in v)))

    def basis(self, op: Operator, pos, orient) -> Basis:
        """Point dipoles at pos (n, 3) with unit orientations orient (n, 3)."""
        p = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        u = np.ascontiguousarray(np.asarray(orient, dtype=np.float64).reshape(-1, 3))
        if p.shape != u.shape:
            raise ValueError("pos and orient must have the same shape")
        h = ctypes.c_void_p()
        _check(load().tfmm_basis_setup(self.handle, op.handle, p.shape[0],
                                       p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)))
        return Basis(self, op, h.value, p.shape[0])

    def aggregate(self, basis: Basis, I, A, stream=None):
        """Eq. (4): I [nrhs, n_basis] -> A [2 nrhs, n_dir, Kx, Ky, Kz]."""
        nrhs = int(I.shape[0])
        a = _check_vec(A, (2 * nrhs,) + basis.op.block, "A")
        _check(load().tfmm_aggregate(self.handle, basis.handle, ctypes.c_void_p(_check_vec(I, (nrhs, basis.n), "I")),
                                     ctypes.c_void_p(a), nrhs, ctypes.c_void_p(_stream_handle(stream))))

    def disaggregate(self, basis: Basis, B, y, stream=None):
        """Eq. (6): B [2 nrhs, n_dir, Kx, Ky, Kz] -> y [nrhs, n_basis]."""
        nrhs = int(y.shape[0])
        b = _check_vec(B, (2 * nrhs,) + basis.op.block, "B")
        _check(load().tfmm_disaggregate(self.handle, basis.handle, ctypes.c_void_p(b),
                                        ctypes.c_void_p(_check_vec(y, (nrhs, basis.n), "y")), nrhs,
                                        ctypes.c_void_p(_stream_handle(stream))))

    def farfield_matvec(self, op: Operator, basis: Basis, I, y, stream=None):
        """Far-field product y = Zfar I (aggregate, translate, project)."""
        nrhs = int(I.shape[0])
        _check(load().tfmm_farfield_matvec(self.handle, op.handle, basis.handle,
                                           ctypes.c_void_p(_check_vec(I, (nrhs, basis.n), "I")),
                                           ctypes.c_void_p(_check_vec(y, (nrhs, basis.n), "y")), nrhs,
                                           ctypes.c_void_p(_stream_handle(stream))))

    def near(self, n, row_ptr, cols, vals) -> NearField:
        """Near-field matrix from host CSR arrays (vals complex)."""
        rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
        ci = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        v = np.ascontiguousarray(np.asarray(vals, dtype=np.complex128)).view(np.float64)
        h = ctypes.c_void_p()
        _check(load().tfmm_near_setup(self.handle, int(n), rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)))
        return NearField(self, h.value, int(n))

    def near_matvec(self, near: NearField, x, y, stream=None):
        nrhs = int(x.shape[0])
        _check(load().tfmm_near_matvec(self.handle, near.handle, ctypes.c_void_p(_check_vec(x, (nrhs, near.n), "x")),
                                       ctypes.c_void_p(_check_vec(y, (nrhs, near.n), "y")), nrhs,
                                       ctypes.c_void_p(_stream_handle(stream))))

    def solve_tfqmr(self, op: Operator, basis: Basis, near: NearField, V, I, tol=1e-6, maxit=500):
        """Solve (Zn + Zfar) I = V; returns (iterations, relative residual).  Waits
        for torch's current stream first (the solve runs on its own stream)."""
        import torch

        v = _check_vec(V, (basis.n,), "V")
        i = _check_vec(I, (basis.n,), "I")
        torch.cuda.current_stream().synchronize()
        it, rr = ctypes.c_int32(), ctypes.c_double()
        _check(load().tfmm_solve_tfqmr(self.handle, op.handle, basis.handle, near.handle, ctypes.c_void_p(v),
                                       ctypes.c_void_p(i), float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rr)))
        return it.value, rr.value

    def set_profiling(self, on: bool):
        _check(load().tfmm_set_profiling(self.handle, 1 if on else 0))

    def kernel_times(self, reset: bool = False) -> dict:
        cap = 64
        names = ctypes.create_string_buffer(8192)
        avg = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        _check(load().tfmm_kernel_times(self.handle, names, 8192, avg, cnt, -cap if reset else cap, ctypes.byref(n)))
        keys = [k for k in names.value.decode().split("\n") if k]
        return {k: {"avg_ms": avg[i], "launches": cnt[i]} for i, k in enumerate(keys[: min(n.value, cap)])}
