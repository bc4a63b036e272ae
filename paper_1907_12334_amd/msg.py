"""ctypes binding of ``libmsg.so`` (C-ABI of include/msg.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory and the stream.  A missing library is an
error; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsg.so")

MSG_OK, MSG_ERR_ARG, MSG_ERR_LAYOUT, MSG_ERR_WORKSPACE, MSG_ERR_HIP, MSG_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SAMPLE_CONVERGED, SAMPLE_MAXITER, SAMPLE_NONFINITE = 0, 1, 2
FIELD_COS_TABLE, FIELD_SEPARABLE_SE = 0, 1
FACE_POINT, FACE_MEAN = 0, 1
FP64, MIXED = 0, 1

EXPORTS = ("msg_default_opts", "msg_create", "msg_destroy", "msg_last_error", "msg_layout",
           "msg_workspace_size", "msg_sample_field", "msg_solve_batch", "msg_quantity", "mimc_delta_q",
           "msg_set_profiling", "msg_get_profile", "msg_cycles_workspace_size", "msg_cycles",
           "msg_matern_workspace_size", "msg_sample_matern", "msg_sample_field_noalloc")
CYCLES_MSG, CYCLES_MG = 0, 1
QOI_MEAN, QOI_POINT, QOI_SUBDOMAIN, QOI_FLUX = range(4)
(KERNEL_SMOOTH, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_TAIL, KERNEL_RESIDUAL_NORM, KERNEL_SMOOTH_STAGE,
 KERNEL_RESTRICT_STAGE) = range(7)
KERNEL_NAMES = ("smooth", "restrict", "prolong", "tail", "residual_norm", "smooth_stage", "restrict_stage")


class MsgError(RuntimeError):
    def __init__(self, code, where, detail):
        super().__init__(f"{where} failed ({code}): {detail}")
        self.code = code


class FieldSpecC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("a", ctypes.POINTER(ctypes.c_int32)), ("b", ctypes.POINTER(ctypes.c_int32)),
                ("amp", ctypes.POINTER(ctypes.c_double)),
                ("mx", ctypes.c_int32), ("my", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("sigma2", ctypes.c_double),
                ("face_rule", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("sample_id", ctypes.POINTER(ctypes.c_int64))]


class BatchDescC(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("c", ctypes.c_int32),
                ("P", ctypes.POINTER(ctypes.c_int32)), ("Q", ctypes.POINTER(ctypes.c_int32))]


class MaternSpecC(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("nu", ctypes.c_double),
                ("eta", ctypes.POINTER(ctypes.c_double)), ("theta", ctypes.POINTER(ctypes.c_double)),
                ("sample_id", ctypes.POINTER(ctypes.c_int64)), ("seed", ctypes.c_uint64),
                ("pad", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class KernelStatsC(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("milliseconds", ctypes.c_double), ("bytes", ctypes.c_double),
                ("model_bytes", ctypes.c_double)]


class SolveOptsC(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_int32), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("max_cycles", ctypes.c_int32), ("tol", ctypes.c_double), ("omega", ctypes.c_double),
                ("precision", ctypes.c_int32), ("tail_levels", ctypes.c_int32), ("handoff", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("tail_budget", ctypes.c_int32), ("tile_width", ctypes.c_int32),
                ("tile_cells", ctypes.c_int32), ("tile_lds", ctypes.c_int32), ("graphs", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        # torch carries its own HIP runtime; loading it first lets the library
        # bind to that same runtime, so the process holds one device context
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
        L.msg_default_opts.argtypes = [ctypes.POINTER(SolveOptsC)]
        L.msg_default_opts.restype = None
        L.msg_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.msg_destroy.argtypes = [vp]
        L.msg_destroy.restype = None
        L.msg_last_error.restype = ctypes.c_char_p
        L.msg_layout.argtypes = [ctypes.POINTER(BatchDescC), i64p, i64p, i64p, i64p]
        L.msg_workspace_size.argtypes = [vp, ctypes.POINTER(BatchDescC), ctypes.POINTER(SolveOptsC),
                                         ctypes.POINTER(ctypes.c_size_t)]
        L.msg_sample_field.argtypes = [vp, ctypes.POINTER(FieldSpecC), ctypes.POINTER(BatchDescC),
                                       vp, vp, vp, vp, vp, vp]
        L.msg_sample_field_noalloc.argtypes = L.msg_sample_field.argtypes
        L.msg_solve_batch.argtypes = [vp, ctypes.POINTER(BatchDescC), ctypes.POINTER(SolveOptsC),
                                      vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.mimc_delta_q.argtypes = [ctypes.POINTER(BatchDescC), vp, vp, vp]
        L.msg_quantity.argtypes = [ctypes.POINTER(BatchDescC), ctypes.c_int, vp, vp, vp, vp]
        L.msg_set_profiling.argtypes = [vp, ctypes.c_int]
        L.msg_get_profile.argtypes = [vp, ctypes.c_int, ctypes.POINTER(KernelStatsC)]
        L.msg_cycles_workspace_size.argtypes = [vp, ctypes.POINTER(BatchDescC), ctypes.POINTER(SolveOptsC),
                                                ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.msg_cycles.argtypes = [vp, ctypes.POINTER(BatchDescC), ctypes.POINTER(SolveOptsC), ctypes.c_int,
                                 ctypes.c_int, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.msg_matern_workspace_size.argtypes = [ctypes.POINTER(BatchDescC), ctypes.POINTER(MaternSpecC),
                                                ctypes.POINTER(ctypes.c_size_t)]
        L.msg_sample_matern.argtypes = [vp, ctypes.POINTER(MaternSpecC), ctypes.POINTER(BatchDescC),
                                        vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        for n in ("msg_create", "msg_layout", "msg_workspace_size", "msg_sample_field", "msg_sample_field_noalloc",
                  "msg_solve_batch",
                  "msg_quantity", "mimc_delta_q", "msg_set_profiling", "msg_get_profile",
                  "msg_cycles_workspace_size", "msg_cycles", "msg_matern_workspace_size", "msg_sample_matern"):
            getattr(L, n).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().msg_last_error().decode()


def _check(code, where):
    if code != MSG_OK:
        raise MsgError(code, where, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- descriptors
class Batch:
    """A batch descriptor: coarsest cells c and per-sample finest (P, Q)."""

    def __init__(self, c: int, P: Sequence[int], Q: Sequence[int]):
        self.c = int(c)
        self.P = np.ascontiguousarray(P, dtype=np.int32)
        self.Q = np.ascontiguousarray(Q, dtype=np.int32)
        if self.P.shape != self.Q.shape or self.P.ndim != 1:
            raise ValueError("P and Q must be 1-D and of equal length")
        self.c_struct = BatchDescC(len(self.P), self.c,
                                   self.P.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   self.Q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))

    @property
    def n(self):
        return len(self.P)

    def layout(self):
        n = self.n + 1
        cell, xf, yf, grid = (np.zeros(n, dtype=np.int64) for _ in range(4))
        p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _check(lib().msg_layout(ctypes.byref(self.c_struct), p(cell), p(xf), p(yf), p(grid)), "msg_layout")
        return {"cell": cell, "xface": xf, "yface": yf, "grid": grid}


@dataclasses.dataclass
class SolveOpts:
    mu: int = 2
    nu1: int = 2
    nu2: int = 2
    max_cycles: int = 50
    tol: float = 1e-10
    omega: float = 1.0
    precision: int = FP64
    tail_levels: int = -1
    handoff: int = -1
    overlap: int = -1
    tail_budget: int = 0
    tile_width: int = 0
    tile_cells: int = 0
    tile_lds: int = 0
    graphs: int = 0

    def c_struct(self):
        return SolveOptsC(self.mu, self.nu1, self.nu2, self.max_cycles, self.tol, self.omega, self.precision,
                          self.tail_levels, self.handoff, self.overlap, self.tail_budget, self.tile_width,
                          self.tile_cells, self.tile_lds, self.graphs)


def default_opts() -> SolveOpts:
    o = SolveOptsC()
    lib().msg_default_opts(ctypes.byref(o))
    return SolveOpts(o.mu, o.nu1, o.nu2, o.max_cycles, o.tol, o.omega, o.precision, o.tail_levels, o.handoff,
                     o.overlap, o.tail_budget, o.tile_width, o.tile_cells, o.tile_lds, o.graphs)


class FieldSpec:
    """msg_field_spec from an inputs.FieldSpec-like object.  seed and
    sample_id (host int64 [n_samples] or None for 0..n-1) name the random
    streams of the normals when msg_sample_field draws them on the device."""

    def __init__(self, spec, seed: int = 0, sample_id=None):
        self._keep = []
        face_rule = int(getattr(spec, "face_rule", 0))
        ids = None if sample_id is None else np.ascontiguousarray(sample_id, dtype=np.int64)
        pid = ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if ids is not None else None
        if spec.kind == "cos":
            a = np.ascontiguousarray(spec.a, dtype=np.int32)
            b = np.ascontiguousarray(spec.b, dtype=np.int32)
            amp = np.ascontiguousarray(spec.amp, dtype=np.float64)
            self._keep = [a, b, amp, ids]
            self.c_struct = FieldSpecC(FIELD_COS_TABLE, len(a), a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       amp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, 0, 0.0, 0.0, 0.0,
                                       face_rule, 0, int(seed) & ((1 << 64) - 1), pid)
        else:
            self._keep = [ids]
            self.c_struct = FieldSpecC(FIELD_SEPARABLE_SE, spec.mx * spec.my, None, None, None, spec.mx, spec.my,
                                       spec.lx, spec.ly, spec.sigma2, face_rule, 0, int(seed) & ((1 << 64) - 1), pid)


def workspace_size(batch: Batch, opts: SolveOpts, handle=None) -> int:
    n = ctypes.c_size_t(0)
    o = opts.c_struct()
    _check(lib().msg_workspace_size(handle, ctypes.byref(batch.c_struct), ctypes.byref(o), ctypes.byref(n)),
           "msg_workspace_size")
    return n.value


class Handle:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().msg_create(ctypes.byref(h), device), "msg_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().msg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on: bool, every: int = 1):
        """Event timing of kernel launches; with every = n > 1, of one launch in n."""
        _check(lib().msg_set_profiling(self.h, int(every) if on else 0), "msg_set_profiling")

    def profile(self):
        """{kernel name: (launches, milliseconds, algorithmic bytes, per-step model bytes)}"""
        out = {}
        for k, name in enumerate(KERNEL_NAMES):
            st = KernelStatsC()
            _check(lib().msg_get_profile(self.h, k, ctypes.byref(st)), "msg_get_profile")
            out[name] = (st.launches, st.milliseconds, st.bytes, st.model_bytes)
        return out

    def sample_matern(self, spec: MaternSpec, batch: Batch, kx, ky, kx32=None, ky32=None, ratio=None, ws=None,
                      stream=None):
        """Matern fields of every sample (k at every face of every grid)."""
        if ws is None:
            import torch
            n = matern_workspace_size(batch, spec)
            ws = torch.empty((n + 7) // 8, dtype=torch.float64, device=kx.device)
        _check(lib().msg_sample_matern(self.h, ctypes.byref(spec.c_struct), ctypes.byref(batch.c_struct), _ptr(kx),
                                       _ptr(ky), _ptr(kx32), _ptr(ky32), _ptr(ratio), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(stream)),
               "msg_sample_matern")

    def cycles(self, batch: Batch, opts: SolveOpts, kind: int, ncycles: int, kx, ky, rhs, u_top, ratios, ws,
               stream=None):
        """Plain cycles from zero (CYCLES_MSG or CYCLES_MG) on every sample's finest grid."""
        o = opts.c_struct()
        _check(lib().msg_cycles(self.h, ctypes.byref(batch.c_struct), ctypes.byref(o), int(kind), int(ncycles),
                                _ptr(kx), _ptr(ky), _ptr(rhs), _ptr(u_top), _ptr(ratios), _ptr(ws),
                                ws.numel() * ws.element_size() if ws is not None else 0, _stream(stream)),
               "msg_cycles")

    # ---- raw entry points (device tensors in, device tensors out)
    def sample_field(self, spec: FieldSpec, batch: Batch, xi, kx, ky, kx32=None, ky32=None, stream=None):
        _check(lib().msg_sample_field(self.h, ctypes.byref(spec.c_struct), ctypes.byref(batch.c_struct), _ptr(xi),
                                      _ptr(kx), _ptr(ky), _ptr(kx32), _ptr(ky32), _stream(stream)),
               "msg_sample_field")

    def solve_batch(self, batch: Batch, opts: SolveOpts, kx, ky, kx32, ky32, rhs, u, q, status, cycles, ws,
                    stream=None):
        o = opts.c_struct()
        _check(lib().msg_solve_batch(self.h, ctypes.byref(batch.c_struct), ctypes.byref(o), _ptr(kx), _ptr(ky),
                                     _ptr(kx32), _ptr(ky32), _ptr(rhs), _ptr(u), _ptr(q), _ptr(status),
                                     _ptr(cycles), _ptr(ws), ws.numel() * ws.element_size() if ws is not None else 0,
                                     _stream(stream)),
               "msg_solve_batch")


class MaternSpec:
    """Matern field parameters: length scale lam, smoothness nu, per-sample
    anisotropic ratio eta and rotation theta (radians), random streams
    (sample ids, seed) and the embedding factor pad (0: the paper's)."""

    def __init__(self, lam: float, nu: float, eta, theta, sample_id=None, seed: int = 0, pad: int = 0):
        self.eta = np.ascontiguousarray(eta, dtype=np.float64)
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.ids = None if sample_id is None else np.ascontiguousarray(sample_id, dtype=np.int64)
        self.c_struct = MaternSpecC(float(lam), float(nu),
                                    self.eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    self.theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    self.ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if self.ids is not None
                                    else None, int(seed), int(pad), 0)


def matern_workspace_size(batch: Batch, spec: MaternSpec) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().msg_matern_workspace_size(ctypes.byref(batch.c_struct), ctypes.byref(spec.c_struct),
                                           ctypes.byref(n)), "msg_matern_workspace_size")
    return n.value


def cycles_workspace_size(batch: Batch, opts: SolveOpts, kind: int, handle=None) -> int:
    n = ctypes.c_size_t(0)
    o = opts.c_struct()
    _check(lib().msg_cycles_workspace_size(handle, ctypes.byref(batch.c_struct), ctypes.byref(o), int(kind),
                                           ctypes.byref(n)), "msg_cycles_workspace_size")
    return n.value


def quantity(batch: Batch, kind: int, kx, u, q, stream=None):
    """Per-grid quantity of interest `kind` (QOI_*) of solutions u into q."""
    _check(lib().msg_quantity(ctypes.byref(batch.c_struct), int(kind), _ptr(kx), _ptr(u), _ptr(q), _stream(stream)),
           "msg_quantity")


def delta_q(batch: Batch, q, dq, stream=None):
    _check(lib().mimc_delta_q(ctypes.byref(batch.c_struct), _ptr(q), _ptr(dq), _stream(stream)), "mimc_delta_q")


# ---------------------------------------------------------------- convenience
class Buffers:
    """Device buffers of one batch: fields, outputs and workspace (torch).
    With `arena` (a uint8 device tensor), every buffer is a 256-byte aligned
    view into it instead of an allocation of its own (Buffers.bytes_needed
    says how much it must hold)."""

    def __init__(self, batch: Batch, opts: SolveOpts, device="cuda:0", mixed_fields=None, arena=None):
        import torch
        lay = batch.layout()
        self.layout = lay
        dev = torch.device(device) if arena is None else arena.device
        mixed = opts.precision == MIXED if mixed_fields is None else mixed_fields
        nbytes = workspace_size(batch, opts)
        plan = self._plan(lay, batch.n, mixed, nbytes)
        if arena is not None:
            arena = arena[(-arena.data_ptr()) % 256:]            # views start on 256-byte boundaries
            if plan[-1][1] > arena.numel():
                raise ValueError(f"arena of {arena.numel()} bytes cannot hold the batch ({plan[-1][1]} bytes)")
        for name, end, dtype, n in plan[:-1]:
            if dtype is None:
                setattr(self, name, None)
            elif arena is None:
                setattr(self, name, torch.empty(n, dtype=dtype, device=dev))
            else:
                size = n * torch.empty((), dtype=dtype).element_size()
                setattr(self, name, arena[end - size:end].view(dtype))

    @staticmethod
    def _plan(lay, S, mixed, ws_bytes):
        """[(name, end byte in the arena, dtype or None, elements)] plus the total."""
        import torch
        items = [("kx", torch.float64, int(lay["xface"][-1])), ("ky", torch.float64, int(lay["yface"][-1])),
                 ("kx32", torch.float32 if mixed else None, int(lay["xface"][-1])),
                 ("ky32", torch.float32 if mixed else None, int(lay["yface"][-1])),
                 ("u", torch.float64, int(lay["cell"][-1])), ("q", torch.float64, int(lay["grid"][-1])),
                 ("dq", torch.float64, int(lay["grid"][-1])), ("cycles", torch.int32, int(lay["grid"][-1])),
                 ("status", torch.int32, S), ("ws", torch.float64, (ws_bytes + 7) // 8)]
        out, off = [], 0
        for name, dt, n in items:
            if dt is None:
                out.append((name, off, None, 0))
                continue
            size = n * torch.empty((), dtype=dt).element_size()
            off = (off + 255) // 256 * 256 + size
            out.append((name, off, dt, n))
        out.append(("total", (off + 255) // 256 * 256, None, 0))
        return out

    @staticmethod
    def bytes_needed(batch: Batch, opts: SolveOpts, mixed_fields=None) -> int:
        """Arena bytes that hold every buffer of the batch."""
        mixed = opts.precision == MIXED if mixed_fields is None else mixed_fields
        return Buffers._plan(batch.layout(), batch.n, mixed, workspace_size(batch, opts))[-1][1] + 256


def run(handle: Handle, spec, batch: Batch, opts: SolveOpts, xi, bufs: Optional[Buffers] = None, rhs=None,
        stream=None, field=True, seed: int = 0, sample_id=None):
    """Field synthesis, full-MSG solve of every sample, multi-index differences.
    xi: device normals [S][n_terms], or None to draw them on the device from
    the streams (seed, sample_id)."""
    bufs = bufs or Buffers(batch, opts)
    if field:
        handle.sample_field(FieldSpec(spec, seed, sample_id), batch, xi, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32,
                            stream)
    handle.solve_batch(batch, opts, bufs.kx, bufs.ky, bufs.kx32, bufs.ky32, rhs, bufs.u, bufs.q, bufs.status,
                       bufs.cycles, bufs.ws, stream)
    delta_q(batch, bufs.q, bufs.dq, stream)
    return bufs
