"""MI355X free-space Poisson solver: thin Python binding of ``libpsn.so``.

Every step of a solve runs in the HIP kernels of the C library; this module
only marshals arguments (plan handles, device pointers, the current HIP
stream).  PyTorch supplies device memory and streams.  There is no fallback:
if the library is missing, importing this module raises ImportError.

    import torch, paper_1612_01799_amd as psn
    plan = psn.Plan(n=128, L=8.0, tol=1e-12, dtype="f32").build()
    u = plan.solve(rho)            # rho: (n, n, n) float32 CUDA tensor

The names follow the C ABI in ``include/psn.h``: ``plan_create``,
``kernel_build``, ``solve``, ``solve_batched``, ``plan_query``.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Plan", "PsnError", "solve_batched", "solve_batched_noalloc", "size_supported", "library_path",
           "F64", "F32", "SPLIT", "CORRECTION_FOLDED", "CORRECTION_FOURIER", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpsn.so")

F64, F32, SPLIT = 0, 1, 2
CORRECTION_FOLDED, CORRECTION_FOURIER = 0, 1
_CORRECTIONS = {"folded": CORRECTION_FOLDED, "fourier": CORRECTION_FOURIER,
                CORRECTION_FOLDED: CORRECTION_FOLDED, CORRECTION_FOURIER: CORRECTION_FOURIER}
_DTYPES = {"f64": F64, "f32": F32, "split": SPLIT, F64: F64, F32: F32, SPLIT: SPLIT}
STATUS = {0: "PSN_OK", -1: "PSN_EINVAL", -2: "PSN_ESIZE", -3: "PSN_ENOMEM", -4: "PSN_EDEVICE",
          -5: "PSN_ESTATE", -6: "PSN_EFIT", -7: "PSN_ELIMIT"}


class PsnError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = _lib.psn_last_error().decode()
        msg = f"{what}: {STATUS.get(status, status)} ({_lib.psn_strerror(status).decode()})"
        super().__init__(msg + (f"; {detail}" if detail else ""))


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("dtype", ctypes.c_int), ("L", ctypes.c_double), ("tol", ctypes.c_double),
        ("h", ctypes.c_double), ("T", ctypes.c_double), ("period", ctypes.c_double),
        ("delta", ctypes.c_double), ("R", ctypes.c_double), ("hs", ctypes.c_double),
        ("terms", ctypes.c_int), ("eps_achieved", ctypes.c_double), ("C0", ctypes.c_double),
        ("C2", ctypes.c_double), ("built", ctypes.c_int), ("device_bytes", ctypes.c_size_t),
        ("algorithmic_bytes", ctypes.c_double), ("a", ctypes.c_double * 3), ("b", ctypes.c_double * 3),
        ("h3", ctypes.c_double * 3), ("T3", ctypes.c_double * 3), ("schedule", ctypes.c_int * 2),
        ("tuned", ctypes.c_int), ("device", ctypes.c_int), ("correction", ctypes.c_int),
        ("n3", ctypes.c_int * 3),
    ]


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 (soname
    # libamdhip64.so.7) and loads it by an unversioned name, so if this library
    # were loaded first the process would end up with two runtimes and the
    # second would see no device.  Loading torch first makes the library bind
    # to torch's runtime through the shared soname.
    import torch  # noqa: F401
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run `python paper_1612_01799_amd/build.py`")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    sig = {
        "psn_plan_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(P)]),
        "psn_plan_create_box": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_int,
                                               ctypes.POINTER(P)]),
        "psn_plan_create_grid": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_int,
                                                ctypes.POINTER(P)]),
        "psn_kernel_build": (ctypes.c_int, [P, P]),
        "psn_solve": (ctypes.c_int, [P, P, P, P]),
        "psn_solve_timed": (ctypes.c_int, [P, P, P, P, ctypes.POINTER(ctypes.c_double)]),
        "psn_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P),
                                             ctypes.POINTER(P), P]),
        "psn_solve_batched_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P),
                                                     ctypes.POINTER(P), P]),
        "psn_plan_query": (ctypes.c_int, [P, ctypes.POINTER(PlanInfo)]),
        "psn_plan_gs_table": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "psn_kernel_download": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double)]),
        "psn_plan_set_schedule": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int]),
        "psn_plan_set_correction": (ctypes.c_int, [P, ctypes.c_int]),
        "psn_plan_destroy": (None, [P]),
        "psn_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "psn_last_error": (ctypes.c_char_p, []),
        "psn_size_supported": (ctypes.c_int, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def library_path() -> str:
    return _LIB_PATH


def size_supported(n: int) -> bool:
    return bool(_lib.psn_size_supported(int(n)))


def _check(st: int, what: str):
    if st != 0:
        raise PsnError(st, what)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """One grid geometry: n^3 points on [-L, L]^3 (or on the box a..b when
    `box=(a, b)` is given, a and b 3-sequences), Gaussian-sum tolerance tol.
    `n` may be a 3-sequence of per-axis point counts (psn_plan_create_grid).
    `correction` is "folded" (the near-zone correction's symbol added to the
    kernel spectrum) or "fourier" (added after the convolution, with the
    Laplacian from the density's size-N Fourier series)."""

    def __init__(self, n, L: float = None, tol: float = 1e-12, dtype="f32", box=None,
                 correction="folded"):
        self._h = ctypes.c_void_p()
        n3 = tuple(int(v) for v in n) if isinstance(n, (tuple, list)) else (int(n),) * 3
        if len(n3) != 3:
            raise ValueError("n must be an int or a 3-sequence")
        self.n = n3[0]
        self.shape = n3
        self.dtype = _DTYPES[dtype]
        if box is None and len(set(n3)) == 1:
            self.L = float(L)
            _check(_lib.psn_plan_create(self.n, self.L, float(tol), self.dtype, ctypes.byref(self._h)),
                   "psn_plan_create")
        else:
            if box is None:
                box = ((-float(L),) * 3, (float(L),) * 3)
            a = (ctypes.c_double * 3)(*[float(v) for v in box[0]])
            b = (ctypes.c_double * 3)(*[float(v) for v in box[1]])
            self.L = max(0.5 * (b[q] - a[q]) for q in range(3))
            nn = (ctypes.c_int * 3)(*n3)
            _check(_lib.psn_plan_create_grid(nn, a, b, float(tol), self.dtype, ctypes.byref(self._h)),
                   "psn_plan_create_grid")
        if _CORRECTIONS[correction] != CORRECTION_FOLDED:
            _check(_lib.psn_plan_set_correction(self._h, _CORRECTIONS[correction]), "psn_plan_set_correction")

    # -- setup
    def build(self, stream=None) -> "Plan":
        _check(_lib.psn_kernel_build(self._h, _stream_handle(stream)), "psn_kernel_build")
        self._dev = self.info()["device"]
        return self

    # -- solve
    def io_dtype(self):
        import torch
        return torch.float32 if self.dtype == F32 else torch.float64

    def device(self) -> int:
        """HIP device the kernel spectrum was built on (-1 before build())."""
        return getattr(self, "_dev", -1)

    def _check_io(self, rho, out, what):
        """Every pointer handed to the kernels must be a contiguous CUDA tensor
        of the plan's shape and I/O dtype on the plan's device: a host pointer
        reaching a kernel is a GPU page fault, a wrong dtype a wrong result."""
        import torch
        for name, t in (("rho", rho), ("out", out)):
            if not isinstance(t, torch.Tensor):
                raise ValueError(f"{what}: {name} must be a torch tensor")
            if not t.is_cuda:
                raise ValueError(f"{what}: {name} must be a CUDA tensor (got device {t.device})")
            if tuple(t.shape) != self.shape or t.dtype != self.io_dtype() or not t.is_contiguous():
                raise ValueError(f"{what}: {name} must be a contiguous {self.shape} {self.io_dtype()} tensor, "
                                 f"got {tuple(t.shape)} {t.dtype} contiguous={t.is_contiguous()}")
        dev = self.device()
        if dev < 0:
            return  # not built: the library reports PSN_ESTATE before any launch
        cur = torch.cuda.current_device()
        for name, t in (("rho", rho), ("out", out)):
            if t.device.index != dev or dev != cur:
                raise ValueError(f"{what}: {name} is on cuda:{t.device.index}, the plan on cuda:{dev}, "
                                 f"the current device is cuda:{cur}")

    def solve(self, rho, out=None, stream=None):
        import torch
        if not isinstance(rho, torch.Tensor) or not rho.is_cuda:
            raise ValueError("psn_solve: rho must be a CUDA tensor")
        if out is None:
            out = torch.empty_like(rho)
        self._check_io(rho, out, "psn_solve")
        _check(_lib.psn_solve(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              _stream_handle(stream)), "psn_solve")
        return out

    def solve_timed(self, rho, out, stream=None):
        """One solve with per-pass HIP events; returns the five pass times in ms."""
        import numpy as np
        self._check_io(rho, out, "psn_solve_timed")
        ms = np.zeros(5)
        _check(_lib.psn_solve_timed(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream_handle(stream), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "psn_solve_timed")
        return ms

    def set_schedule(self, p24: int, p3: int) -> "Plan":
        _check(_lib.psn_plan_set_schedule(self._h, int(p24), int(p3)), "psn_plan_set_schedule")
        return self

    # -- introspection
    def info(self) -> dict:
        inf = PlanInfo()
        _check(_lib.psn_plan_query(self._h, ctypes.byref(inf)), "psn_plan_query")
        out = {}
        for f, _ in PlanInfo._fields_:
            v = getattr(inf, f)
            out[f] = tuple(v) if isinstance(v, ctypes.Array) else v
        return out

    def gs_table(self):
        import numpy as np
        m = ctypes.c_int()
        _check(_lib.psn_plan_gs_table(self._h, None, None, 0, ctypes.byref(m)), "psn_plan_gs_table")
        tau = np.empty(m.value)
        w = np.empty(m.value)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(_lib.psn_plan_gs_table(self._h, tau.ctypes.data_as(dp), w.ctypes.data_as(dp), m.value,
                                      ctypes.byref(m)), "psn_plan_gs_table")
        return tau, w

    def kernel_octant(self):
        import numpy as np
        k = np.empty(tuple(v + 1 for v in self.shape))
        _check(_lib.psn_kernel_download(self._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "psn_kernel_download")
        return k

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.psn_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_args(plans, rhos, outs, what):
    import torch
    count = len(plans)
    if len(rhos) != count or (outs is not None and len(outs) != count):
        raise ValueError("plans, rhos and outs differ in length")
    for r in rhos:
        if not isinstance(r, torch.Tensor) or not r.is_cuda:
            raise ValueError(f"{what}: every rho must be a CUDA tensor")
    if outs is None:
        outs = [torch.empty_like(r) for r in rhos]
    for i, (p, r, o) in enumerate(zip(plans, rhos, outs)):
        p._check_io(r, o, f"{what} entry {i}")
    P = ctypes.c_void_p
    hp = (P * count)(*[p.handle for p in plans])
    hr = (P * count)(*[P(r.data_ptr()) for r in rhos])
    ho = (P * count)(*[P(o.data_ptr()) for o in outs])
    return count, hp, hr, ho, outs


def solve_batched(plans, rhos, outs=None, stream=None):
    """Enqueue one batch of solves (sizes may differ); returns the outputs."""
    count, hp, hr, ho, outs = _batch_args(plans, rhos, outs, "psn_solve_batched")
    _check(_lib.psn_solve_batched(count, hp, hr, ho, _stream_handle(stream)), "psn_solve_batched")
    return outs


def solve_batched_noalloc(plans, rhos, outs, stream=None):
    """As solve_batched, through the entry point that allocates no device
    memory (the workspace is the library's fixed scratch array); `outs` must
    be given, so that the call itself allocates nothing either."""
    count, hp, hr, ho, outs = _batch_args(plans, rhos, outs, "psn_solve_batched_noalloc")
    _check(_lib.psn_solve_batched_noalloc(count, hp, hr, ho, _stream_handle(stream)),
           "psn_solve_batched_noalloc")
    return outs
