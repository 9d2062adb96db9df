"""Adaptive multigrid for the 2D U(1) Wilson-Dirac normal equations on MI355X.

Thin Python binding of ``libsmg.so`` (declared in ``include/smg.h``).  Every
numerical step runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory and streams: vectors are complex128
CUDA tensors whose data pointers are handed to the C ABI.

Method: Brannick, Brower, Clark, Osborn and Rebbi, "Adaptive Multigrid Algorithm
for the QCD Dirac-Wilson Operator", arXiv:0710.3612 (Multigrid and Adaptive
Multigrid sections; Results for the smoother, the 4x4 blocks and MG-CG).
"""

from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from pathlib import Path
from typing import Optional, Sequence

__all__ = [
    "load_library",
    "Params",
    "Stats",
    "Solver",
    "Batch",
    "SmgError",
    "FP64",
    "MIXED",
    "COARSEST_DIRECT",
    "COARSEST_CG",
    "STORE_F32",
    "STORE_BF16",
    "STORE_F16",
    "library_path",
    "query_bytes",
    "use_torch_allocator",
]

MAXLEV = 6
FP64 = 0
MIXED = 1
COARSEST_DIRECT = 0
COARSEST_CG = 1
STORE_F32 = 0
STORE_BF16 = 1
STORE_F16 = 2

OK = 0
NOTCONV = 1
EBREAKDOWN = -5
EBUSY = -7

_HERE = Path(__file__).resolve().parent


def library_path() -> Path:
    return Path(os.environ.get("SMG_LIBRARY", _HERE / "libsmg.so"))


class Params(ctypes.Structure):
    """Mirror of smg_params."""

    _fields_ = [
        ("lx", ctypes.c_int32),
        ("lt", ctypes.c_int32),
        ("mass", ctypes.c_double),
        ("levels", ctypes.c_int32),
        ("block", (ctypes.c_int32 * 2) * MAXLEV),
        ("nv", ctypes.c_int32 * MAXLEV),
        ("setup_iters", ctypes.c_int32),
        ("smoother_steps", ctypes.c_int32),
        ("smoother_omega", ctypes.c_double),
        ("t_antiperiodic", ctypes.c_int32),
        ("coarsest", ctypes.c_int32),
        ("coarsest_tol", ctypes.c_double),
        ("coarsest_maxiter", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("sa_scale", ctypes.c_double),
        ("smoother_storage", ctypes.c_int32),
        ("stop_recursive", ctypes.c_int32),
        ("mfma_min_rhs", ctypes.c_int32),
        ("operator_storage", ctypes.c_int32),
        ("split_chirality", ctypes.c_int32),
        ("coarsest_fp64", ctypes.c_int32),
        ("remass_affine", ctypes.c_int32),
        ("nv_stop_rho", ctypes.c_double),
        ("nv_stop_iters", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    """Mirror of smg_stats."""

    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("vcycles", ctypes.c_int32),
        ("fine_applies", ctypes.c_int64),
        ("true_relres", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class SmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"smg error {code}: {msg}")
        self.code = code


_lib = None

# smg_alloc_fn / smg_release_fn
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_allocator = None  # the installed callbacks (kept alive while the library may call them)
# smg_progress_fn
_PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_double, ctypes.c_void_p)
_progress = None  # every installed callback (kept alive while the library may call them)


# Handles and batches still open, closed at interpreter exit while the allocator
# callbacks and torch are still alive (a handle freed during module teardown would
# call a release callback that may already be gone).
_live_solvers = weakref.WeakSet()
_live_batches = weakref.WeakSet()
_live_groups = weakref.WeakSet()


def _close_all():
    for b in list(_live_batches):
        b.close()
    for g in list(_live_groups):
        g.close()
    for s in list(_live_solvers):
        s.close()


def load_library():
    """Load libsmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not path.exists():
        raise RuntimeError(
            f"{path} not found: build it with `python -m paper_0710_3612_amd.build` "
            "(or __graft_entry__.build())"
        )
    lib = ctypes.CDLL(str(path))
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    h = ctypes.c_void_p
    sig = {
        "smg_default_params": (None, [ctypes.POINTER(Params)]),
        "smg_setup": (i32, [P, ctypes.POINTER(Params), P, P, ctypes.POINTER(h)]),
        "smg_setup_from_vectors": (i32, [P, ctypes.POINTER(Params), P, P, P, ctypes.POINTER(h)]),
        "smg_set_mass": (i32, [h, ctypes.c_double, P]),
        "smg_derive": (i32, [h, ctypes.c_double, P, ctypes.POINTER(h)]),
        "smg_apply_D": (i32, [h, P, P, i32, i32, P]),
        "smg_apply_A": (i32, [h, P, P, i32, P]),
        "smg_apply_level": (i32, [h, i32, P, P, i32, P]),
        "smg_apply_level_f32": (i32, [h, i32, P, P, i32, P]),
        "smg_level_op": (i32, [h, i32, i32, ctypes.c_double, P, P, P, P, i32, P]),
        "smg_level_op_f32": (i32, [h, i32, i32, ctypes.c_double, P, P, P, P, i32, P]),
        "smg_restrict": (i32, [h, i32, P, P, i32, P]),
        "smg_prolong": (i32, [h, i32, P, P, i32, P]),
        "smg_smooth": (i32, [h, i32, P, P, i32, P]),
        "smg_vcycle": (i32, [h, P, P, i32, P]),
        "smg_vcycle_f32": (i32, [h, P, P, i32, P]),
        "smg_vcycle_noalloc": (i32, [h, P, P, i32, P]),
        "smg_solve": (i32, [h, P, P, i32, ctypes.c_double, i32, i32, P, ctypes.POINTER(Stats)]),
        "smg_cg": (i32, [h, P, P, i32, ctypes.c_double, i32, P, ctypes.POINTER(Stats)]),
        "smg_level_info": (i32, [h, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "smg_get_prolongator": (i32, [h, i32, i32, P, P]),
        "smg_transfer_info": (i32, [h, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
        "smg_get_coarse_links": (i32, [h, i32, P, P]),
        "smg_get_smoother_coefs": (i32, [h, i32, ctypes.POINTER(ctypes.c_double)]),
        "smg_get_setup_factors": (i32, [h, i32, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]),
        "smg_memory_bytes": (i32, [h, ctypes.POINTER(ctypes.c_size_t)]),
        "smg_query_bytes": (i32, [ctypes.POINTER(Params), i32, i32, ctypes.POINTER(ctypes.c_size_t),
                                  ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "smg_set_allocator": (i32, [_ALLOC_FN, _RELEASE_FN, P]),
        "smg_set_progress": (i32, [_PROGRESS_FN, P]),
        "smg_batch_create": (i32, [h, i32, ctypes.c_double, i32, i32, P, ctypes.POINTER(h)]),
        "smg_batch_admit": (i32, [h, P, ctypes.POINTER(i32), P]),
        "smg_batch_step": (i32, [h, i32, P]),
        "smg_batch_poll": (i32, [h, P, ctypes.POINTER(Stats)]),
        "smg_batch_active": (i32, [h, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "smg_batch_harvest": (i32, [h, i32, P, P]),
        "smg_batch_cancel": (i32, [h, i32, P]),
        "smg_batch_memory_bytes": (i32, [h, ctypes.POINTER(ctypes.c_size_t)]),
        "smg_batch_use_graphs": (i32, [h, i32]),
        "smg_batch_destroy": (None, [h]),
        "smg_group_create": (i32, [ctypes.POINTER(h), i32, P, ctypes.POINTER(h)]),
        "smg_group_solve": (i32, [h, P, P, ctypes.c_double, i32, P, ctypes.POINTER(Stats)]),
        "smg_group_destroy": (None, [h]),
        "smg_group_level_op_f32": (i32, [h, i32, i32, P, P, P, P]),
        "smg_destroy": (None, [h]),
        "smg_strerror": (ctypes.c_char_p, [i32]),
        "smg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    use_torch_allocator(True)
    atexit.register(_close_all)  # runs before torch's own exit handlers, registered earlier
    return lib


def _torch_alloc(nbytes, stream, _ctx):
    import torch

    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # the library reports SMG_ENOMEM
        return None


def _torch_release(ptr, _nbytes, _stream, _ctx, _finalizing=sys.is_finalizing):
    if _finalizing():  # torch may already be gone; the process is ending
        return
    import torch

    torch.cuda.caching_allocator_delete(int(ptr))


def use_torch_allocator(enable: bool = True):
    """Route the library's device memory through PyTorch's caching allocator
    (smg_set_allocator), so that torch accounts for it and can reuse it; with
    enable=False the library returns to hipMalloc for handles created later.
    Installed when the library is loaded."""
    global _allocator
    lib = _lib
    if enable:
        cbs = (_ALLOC_FN(_torch_alloc), _RELEASE_FN(_torch_release))
        _check(lib.smg_set_allocator(cbs[0], cbs[1], None))
        # handles created before keep the callbacks they captured: keep every pair alive
        _allocator = (cbs, _allocator)
    else:
        _check(lib.smg_set_allocator(_ALLOC_FN(), _RELEASE_FN(), None))


def set_progress(fn=None):
    """Install fn(stage, level, step, total, value) as the library's progress
    callback (smg_set_progress: setup levels and vectors, outer iterations,
    defect-correction passes), or turn reporting off with None.  fn runs on the
    thread that made the library call and must not call the library."""
    global _progress
    lib = load_library()
    if fn is None:
        _check(lib.smg_set_progress(_PROGRESS_FN(), None))
        return

    def cb(stage, level, step, total, value, _ctx):
        fn(stage.decode(), level, step, total, value)

    c = _PROGRESS_FN(cb)
    _check(lib.smg_set_progress(c, None))
    # a call on another thread may still be inside an earlier callback: keep every one alive
    _progress = (c, _progress)


def query_bytes(params: "Params", nrhs: int = 1, precision: int = FP64):
    """(setup, solve, batch) device bytes that smg_query_bytes plans for these
    parameters: a handle after setup, what its first solve of nrhs columns adds,
    and what a batch of nrhs slots adds (None when nrhs > 256)."""
    lib = load_library()
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    pc = ctypes.byref(c) if nrhs <= 256 else None
    _check(lib.smg_query_bytes(ctypes.byref(params), int(nrhs), int(precision), ctypes.byref(a), ctypes.byref(b), pc))
    return a.value, b.value, (c.value if nrhs <= 256 else None)


def _check(code: int, allow_notconv: bool = False) -> int:
    if code == OK or (allow_notconv and code == NOTCONV):
        return code
    lib = load_library()
    raise SmgError(code, f"{lib.smg_strerror(code).decode()}: {lib.smg_last_error().decode()}")


def make_params(lx: int, lt: int, mass: float, levels: int = 2, blocks: Sequence = ((4, 4),),
                nv: Sequence[int] = (8,), setup_iters: int = 5, smoother_steps: int = 4,
                smoother_omega: float = 0.8, t_antiperiodic: bool = True, coarsest: int = COARSEST_DIRECT,
                coarsest_tol: float = 1e-12, coarsest_maxiter: int = 10000, inner_tol: float = 1e-5,
                seed: int = 1, sa_scale: float = 4.0 / 3.0, mfma_min_rhs: int = 16,
                smoother_storage: int = STORE_F32, stop_recursive: bool = False,
                operator_storage: int = STORE_F32, split_chirality: bool = False,
                coarsest_fp64: bool = True, remass_affine: bool = False, nv_stop_rho: float = 0.0,
                nv_stop_iters: int = 3) -> Params:
    lib = load_library()
    p = Params()
    lib.smg_default_params(ctypes.byref(p))
    p.lx, p.lt, p.mass, p.levels = lx, lt, mass, levels
    for l in range(levels - 1):
        p.block[l][0], p.block[l][1] = blocks[l]
        p.nv[l] = nv[l]
    p.setup_iters = setup_iters
    p.smoother_steps = smoother_steps
    p.smoother_omega = smoother_omega
    p.t_antiperiodic = int(bool(t_antiperiodic))
    p.coarsest = coarsest
    p.coarsest_tol = coarsest_tol
    p.coarsest_maxiter = coarsest_maxiter
    p.inner_tol = inner_tol
    p.seed = seed
    p.sa_scale = sa_scale
    p.mfma_min_rhs = mfma_min_rhs
    p.smoother_storage = smoother_storage
    p.stop_recursive = int(bool(stop_recursive))
    p.operator_storage = operator_storage
    p.split_chirality = int(bool(split_chirality))
    p.coarsest_fp64 = int(bool(coarsest_fp64))
    p.remass_affine = int(bool(remass_affine))
    p.nv_stop_rho = float(nv_stop_rho)
    p.nv_stop_iters = int(nv_stop_iters)
    return p


def _stream(stream) -> ctypes.c_void_p:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError("expected a contiguous complex128 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Adaptive-MG hierarchy for one gauge field (handle of the C library).

    gauge: complex128 CUDA tensor [2, lt, lx].  Either run the adaptive setup
    (optionally from given random starts, a complex128 CUDA tensor holding the
    per-level blocks [1 + nv_l, n_l] concatenated) or build the hierarchy from
    given near-null vectors (`vectors` and `calib`, see smg_setup_from_vectors).
    """

    def __init__(self, gauge, params: Params, randoms=None, vectors=None, calib=None, stream=None):
        import torch

        self.lib = load_library()
        self.params = params
        self.handle = ctypes.c_void_p()
        g = gauge.contiguous()
        if tuple(g.shape) != (2, params.lt, params.lx):
            raise ValueError(f"gauge must have shape (2, {params.lt}, {params.lx})")
        st = _stream(stream)
        if vectors is not None:
            code = self.lib.smg_setup_from_vectors(_ptr(g), ctypes.byref(params), _ptr(vectors.contiguous()),
                                                   _ptr(calib.contiguous()), st, ctypes.byref(self.handle))
        else:
            rp = _ptr(randoms.contiguous()) if randoms is not None else ctypes.c_void_p()
            code = self.lib.smg_setup(_ptr(g), ctypes.byref(params), rp, st, ctypes.byref(self.handle))
        _check(code)
        self._torch = torch
        _live_solvers.add(self)

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.smg_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # closed at exit already, or the process is ending
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- shapes -----------------------------------------------------------------
    def level_info(self, level: int):
        lx, lt, dof = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.smg_level_info(self.handle, level, ctypes.byref(lx), ctypes.byref(lt), ctypes.byref(dof)))
        return lx.value, lt.value, dof.value

    def level_size(self, level: int) -> int:
        lx, lt, dof = self.level_info(level)
        return lx * lt * dof

    def _new(self, n, like):
        return self._torch.empty(n, dtype=self._torch.complex128, device=like.device)

    @staticmethod
    def _nrhs(x, n):
        if x.numel() % n:
            raise ValueError(f"vector length {x.numel()} is not a multiple of {n}")
        return x.numel() // n

    # -- operators ----------------------------------------------------------------
    def set_mass(self, mass: float, stream=None):
        _check(self.lib.smg_set_mass(self.handle, float(mass), _stream(stream)))
        self.params.mass = mass

    def derive(self, mass: float, stream=None) -> "Solver":
        """New Solver at another mass sharing this setup's near-null vectors."""
        import copy

        other = Solver.__new__(Solver)
        other.lib = self.lib
        other.params = copy.copy(self.params)
        other.params.mass = mass
        other.handle = ctypes.c_void_p()
        other._torch = self._torch
        _check(self.lib.smg_derive(self.handle, float(mass), _stream(stream), ctypes.byref(other.handle)))
        _live_solvers.add(other)
        return other

    def apply_D(self, x, dagger: bool = False, stream=None):
        x = x.contiguous()
        nr = self._nrhs(x, self.level_size(0))
        y = self._new(x.shape, x)
        _check(self.lib.smg_apply_D(self.handle, _ptr(x), _ptr(y), nr, int(dagger), _stream(stream)))
        return y

    def apply_A(self, x, stream=None):
        return self.apply_level(0, x, stream)

    def apply_level(self, level: int, x, stream=None):
        x = x.contiguous()
        nr = self._nrhs(x, self.level_size(level))
        y = self._new(x.shape, x)
        _check(self.lib.smg_apply_level(self.handle, level, _ptr(x), _ptr(y), nr, _stream(stream)))
        return y

    def apply_level_f32(self, level: int, x, stream=None):
        """A^(l) x with the FP32 operator of the mixed-precision solver (complex64 in/out)."""
        import torch

        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex64):
            raise TypeError("expected a complex64 CUDA tensor")
        x = x.contiguous()
        nr = self._nrhs(x, self.level_size(level))
        y = torch.empty_like(x)
        _check(self.lib.smg_apply_level_f32(self.handle, level, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()), nr, _stream(stream)))
        return y

    def level_op(self, level: int, x, mode: int = 0, coef: float = 0.0, xacc=None, aux=None, stream=None):
        """FP64 level operator with the V-cycle's epilogues (smg_level_op);
        complex128 tensors; returns y (xacc is updated in place for modes 1 and 3)."""
        def p64(t):
            if t is None:
                return ctypes.c_void_p()
            if not t.is_cuda or t.dtype != self._torch.complex128 or not t.is_contiguous():
                raise TypeError("expected a contiguous complex128 CUDA tensor")
            return ctypes.c_void_p(t.data_ptr())

        nr = self._nrhs(x, self.level_size(level))
        y = self._torch.empty_like(x)
        _check(self.lib.smg_level_op(self.handle, level, int(mode), float(coef), p64(x), p64(y), p64(xacc),
                                     p64(aux), nr, _stream(stream)))
        return y

    def level_op_f32(self, level: int, x, mode: int = 0, coef: float = 0.0, xacc=None, aux=None, stream=None):
        """FP32 level operator with the V-cycle's epilogues (smg_level_op_f32);
        complex64 tensors; returns y (xacc is updated in place for modes 1 and 3)."""
        def p32(t):
            if t is None:
                return ctypes.c_void_p()
            if not t.is_cuda or t.dtype != self._torch.complex64 or not t.is_contiguous():
                raise TypeError("expected a contiguous complex64 CUDA tensor")
            return ctypes.c_void_p(t.data_ptr())

        nr = self._nrhs(x, self.level_size(level))
        y = self._torch.empty_like(x)
        _check(self.lib.smg_level_op_f32(self.handle, level, int(mode), float(coef), p32(x), p32(y), p32(xacc),
                                         p32(aux), nr, _stream(stream)))
        return y

    def restrict(self, level: int, x, stream=None):
        x = x.contiguous()
        nr = self._nrhs(x, self.level_size(level))
        y = self._new(nr * self.level_size(level + 1), x)
        _check(self.lib.smg_restrict(self.handle, level, _ptr(x), _ptr(y), nr, _stream(stream)))
        return y

    def prolong(self, level: int, e, stream=None):
        e = e.contiguous()
        nr = self._nrhs(e, self.level_size(level + 1))
        y = self._new(nr * self.level_size(level), e)
        _check(self.lib.smg_prolong(self.handle, level, _ptr(e), _ptr(y), nr, _stream(stream)))
        return y

    def smooth(self, level: int, b, stream=None):
        b = b.contiguous()
        nr = self._nrhs(b, self.level_size(level))
        x = self._new(b.shape, b)
        _check(self.lib.smg_smooth(self.handle, level, _ptr(b), _ptr(x), nr, _stream(stream)))
        return x

    def vcycle(self, b, stream=None):
        b = b.contiguous()
        nr = self._nrhs(b, self.level_size(0))
        x = self._new(b.shape, b)
        _check(self.lib.smg_vcycle(self.handle, _ptr(b), _ptr(x), nr, _stream(stream)))
        return x

    def vcycle_noalloc(self, b, out, stream=None):
        """x = V b into `out` without any allocation in the library (smg_vcycle_noalloc)."""
        b = b.contiguous()
        nr = self._nrhs(b, self.level_size(0))
        if out.numel() != b.numel():
            raise ValueError("out must have as many entries as b")
        _check(self.lib.smg_vcycle_noalloc(self.handle, _ptr(b), _ptr(out), nr, _stream(stream)))
        return out

    def vcycle_f32(self, b, stream=None):
        """The mixed solve's FP32 V-cycle (complex64 in/out)."""
        if not (b.is_cuda and b.dtype == self._torch.complex64):
            raise TypeError("expected a complex64 CUDA tensor")
        b = b.contiguous()
        nr = self._nrhs(b, self.level_size(0))
        x = self._torch.empty_like(b)
        _check(self.lib.smg_vcycle_f32(self.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                       nr, _stream(stream)))
        return x

    # -- solvers ------------------------------------------------------------------
    def solve(self, rhs, tol: float = 1e-10, maxiter: int = 10000, precision: int = FP64, out=None, stream=None):
        """Solve A x = rhs; returns (x, [per-column stats dicts], status)."""
        rhs = rhs.contiguous()
        nr = self._nrhs(rhs, self.level_size(0))
        x = out if out is not None else self._new(rhs.shape, rhs)
        st = (Stats * nr)()
        code = self.lib.smg_solve(self.handle, _ptr(rhs), _ptr(x), nr, float(tol), int(maxiter), int(precision),
                                  _stream(stream), st)
        _check(code, allow_notconv=True)
        return x, [s.as_dict() for s in st], code

    def cg(self, rhs, tol: float = 1e-10, maxiter: int = 100000, stream=None):
        rhs = rhs.contiguous()
        nr = self._nrhs(rhs, self.level_size(0))
        x = self._new(rhs.shape, rhs)
        st = (Stats * nr)()
        code = self.lib.smg_cg(self.handle, _ptr(rhs), _ptr(x), nr, float(tol), int(maxiter), _stream(stream), st)
        _check(code, allow_notconv=True)
        return x, [s.as_dict() for s in st], code

    # -- introspection -------------------------------------------------------------
    def transfer_info(self, level: int):
        """(halo, smoothed-aggregation weight) of the prolongator of coarsening `level`."""
        h, w = ctypes.c_int32(), ctypes.c_double()
        _check(self.lib.smg_transfer_info(self.handle, level, ctypes.byref(h), ctypes.byref(w)))
        return h.value, w.value

    def prolongator(self, level: int, smoothed: bool = False, stream=None):
        """P of coarsening `level` as [J, nc, nw] complex128: the tentative one
        (smoothed=False, nw = bx*bt*dof) or the one the V-cycle uses (windows of
        (bx+2h)(bt+2h) sites)."""
        lx, lt, dof = self.level_info(level)
        cx, ct, nc = self.level_info(level + 1)
        bx, bt = lx // cx, lt // ct
        hh = self.transfer_info(level)[0] if smoothed else 0
        nw = (bx + 2 * hh) * (bt + 2 * hh) * dof
        out = self._torch.empty((cx * ct, nc, nw), dtype=self._torch.complex128, device="cuda")
        _check(self.lib.smg_get_prolongator(self.handle, level, int(bool(smoothed)), _ptr(out), _stream(stream)))
        return out

    def coarse_links(self, level: int, stream=None):
        """Links of level >= 1 as [K, 9, nc, nc] complex128 (block (dt+1)*3+(dx+1))."""
        cx, ct, nc = self.level_info(level)
        out = self._torch.empty((cx * ct, 9, nc, nc), dtype=self._torch.complex128, device="cuda")
        _check(self.lib.smg_get_coarse_links(self.handle, level, _ptr(out), _stream(stream)))
        return out

    def smoother_coefs(self, level: int):
        buf = (ctypes.c_double * 64)()
        _check(self.lib.smg_get_smoother_coefs(self.handle, level, buf))
        return [buf[i] for i in range(self.params.smoother_steps)]

    def memory_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(self.lib.smg_memory_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def setup_factors(self, level: int):
        """Two-level factors the adaptive stop measured on coarsening `level`."""
        buf = (ctypes.c_double * 64)()
        cnt = ctypes.c_int32()
        _check(self.lib.smg_get_setup_factors(self.handle, level, buf, 64, ctypes.byref(cnt)))
        return [buf[i] for i in range(cnt.value)]


class Group:
    """Several independent systems of one hierarchy shape solved together
    (smg_group_*): system j is column j of every launch of the mixed-precision
    solve, so one launch per step serves all of them, and x_j equals Solver j's own
    one-column solve bit for bit.  The first solver runs the group: no other call
    may use it while the group is in use."""

    def __init__(self, solvers, stream=None):
        self.lib = solvers[0].lib
        self.solvers = list(solvers)
        self.n = solvers[0].level_size(0)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.handle.value for s in self.solvers])
        self.handle = ctypes.c_void_p()
        _check(self.lib.smg_group_create(arr, len(self.solvers), _stream(stream), ctypes.byref(self.handle)))
        self._torch = solvers[0]._torch
        _live_groups.add(self)

    def solve(self, rhs, tol: float = 1e-10, maxiter: int = 10000, out=None, stream=None):
        """rhs: [nsys, n] complex128 CUDA tensor; returns (x, [per-system stats], status)."""
        rhs = rhs.contiguous()
        G = len(self.solvers)
        if tuple(rhs.shape) != (G, self.n) or rhs.dtype != self._torch.complex128 or not rhs.is_cuda:
            raise ValueError(f"rhs must be a complex128 CUDA tensor of shape ({G}, {self.n})")
        x = out if out is not None else self._torch.empty_like(rhs)
        st = (Stats * G)()
        code = self.lib.smg_group_solve(self.handle, _ptr(rhs), _ptr(x), float(tol), int(maxiter), _stream(stream),
                                        st)
        _check(code, allow_notconv=True)
        return x, [q.as_dict() for q in st], code

    def level_op_f32(self, level: int, x, mode: int = 0, aux=None, out=None, stream=None):
        """Every system's FP32 level operator on its own column (smg_group_level_op_f32):
        x: [nsys, n_level] complex64 CUDA tensor; mode 0: y_j = A_j x_j, mode 2:
        y_j = aux_j - A_j x_j.  Returns y."""
        G = len(self.solvers)
        shape = (G, self.solvers[0].level_size(level))

        def p32(t):
            if t is None:
                return ctypes.c_void_p()
            if (tuple(t.shape) != shape or t.dtype != self._torch.complex64 or not t.is_cuda
                    or not t.is_contiguous()):
                raise ValueError(f"expected a contiguous complex64 CUDA tensor of shape {shape}")
            return ctypes.c_void_p(t.data_ptr())

        y = out if out is not None else self._torch.empty(shape, dtype=self._torch.complex64, device=x.device)
        _check(self.lib.smg_group_level_op_f32(self.handle, int(level), int(mode), p32(x), p32(y), p32(aux),
                                               _stream(stream)))
        return y

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.smg_group_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Continuous batch of MG-CG solves on one Solver (smg_batch_* of the C ABI).

    `capacity` column slots; right-hand sides are admitted into free slots at any
    time, `step(k)` advances every running slot by k iterations, finished slots
    are harvested and reused.  A slot's result does not depend on what else runs
    in the batch.  While the batch exists its Solver must not run other solves.
    """

    def __init__(self, solver: Solver, capacity: int, tol: float = 1e-10, maxiter: int = 10000,
                 precision: int = FP64, stream=None):
        self.lib = solver.lib
        self.solver = solver
        self.capacity = int(capacity)
        self.n = solver.level_size(0)
        self.handle = ctypes.c_void_p()
        _check(self.lib.smg_batch_create(solver.handle, self.capacity, float(tol), int(maxiter), int(precision),
                                         _stream(stream), ctypes.byref(self.handle)))
        self._stats = (Stats * self.capacity)()
        self._done = (ctypes.c_uint8 * self.capacity)()
        _live_batches.add(self)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.smg_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # closed at exit already, or the process is ending
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def admit(self, rhs, stream=None) -> Optional[int]:
        """Start solving A x = rhs (complex128, n entries); returns the slot, or
        None when every slot is occupied."""
        rhs = rhs.contiguous()
        if rhs.numel() != self.n:
            raise ValueError(f"rhs must have {self.n} entries")
        slot = ctypes.c_int32()
        code = self.lib.smg_batch_admit(self.handle, _ptr(rhs), ctypes.byref(slot), _stream(stream))
        if code == EBUSY:
            return None
        _check(code)
        return slot.value

    def step(self, iters: int = 1, stream=None):
        _check(self.lib.smg_batch_step(self.handle, int(iters), _stream(stream)))

    def poll(self):
        """[(slot, stats dict)] of the finished, not yet harvested slots."""
        _check(self.lib.smg_batch_poll(self.handle, self._done, self._stats))
        return [(j, self._stats[j].as_dict()) for j in range(self.capacity) if self._done[j]]

    def stats(self, slot: int) -> dict:
        _check(self.lib.smg_batch_poll(self.handle, None, self._stats))
        return self._stats[slot].as_dict()

    def counts(self):
        """(occupied slots, running slots)."""
        u, r = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.smg_batch_active(self.handle, ctypes.byref(u), ctypes.byref(r)))
        return u.value, r.value

    def harvest(self, slot: int, out=None, stream=None):
        """Solution of a finished slot (a new tensor, or `out`); frees the slot."""
        import torch

        x = out if out is not None else torch.empty(self.n, dtype=torch.complex128, device="cuda")
        _check(self.lib.smg_batch_harvest(self.handle, int(slot), _ptr(x), _stream(stream)))
        return x

    def cancel(self, slot: int, stream=None):
        _check(self.lib.smg_batch_cancel(self.handle, int(slot), _stream(stream)))

    def memory_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(self.lib.smg_batch_memory_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def use_graphs(self, enable: bool):
        """Replay iterations as captured HIP graphs (default with a direct coarsest solve) or not."""
        _check(self.lib.smg_batch_use_graphs(self.handle, int(bool(enable))))
