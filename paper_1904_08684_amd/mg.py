"""Python binding of libmg.so (ctypes; argument marshalling only).

Every numerical step runs inside the HIP library.  The module-level
functions carry the C names of include/mg.h; ``Solver`` bundles a context
with the PyTorch device workspace it lives in.  PyTorch provides device
memory and the stream only.

Importing this module loads the built library and raises ImportError when it
is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmg.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_1904_08684_amd.build` "
                      "or __graft_entry__.build()")
# torch's HIP libraries name the runtime libamdhip64.so, this library
# libamdhip64.so.7: loaded first, this library would pull in the system's
# runtime and torch then a second copy of its own, whose late start finds no
# device.  With torch loaded first the dynamic linker resolves this
# library's dependency to torch's runtime, one runtime for both.
try:
    import torch  # noqa: F401
except ImportError:          # the C-ABI alone, without torch
    pass
lib = C.CDLL(_LIB_PATH)

# ------------------------------------------------------------------ constants
MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE = 0, -1, -2, -3
MG_ENOTCONV, MG_ENONFINITE, MG_EDIVERGED, MG_EBUSY = -4, -5, -6, -7
MG_ECANCELED, MG_ETIMEDOUT = -8, -9
MG_NODE, MG_CELL = 0, 1
MG_LAPLACE, MG_VARCOEF = 0, 1
MG_DIRICHLET0, MG_NEUMANN0 = 0, 1
MG_COARSE_REDISCRETISE, MG_COARSE_GALERKIN = 0, 1
MG_JACOBI, MG_RBGS = 0, 1
MG_FP64, MG_MIXED = 0, 1
MG_CYCLE_V, MG_CYCLE_W, MG_CYCLE_F = 0, 1, 2
MG_PREC_FP64, MG_PREC_FP32 = 0, 1
MG_FIELD_U, MG_FIELD_F, MG_FIELD_R = 0, 1, 2
(MG_OP_GS_RED, MG_OP_GS_BLACK, MG_OP_JACOBI, MG_OP_RESIDUAL, MG_OP_RESTRICT,
 MG_OP_PROLONG, MG_OP_COARSE, MG_OP_VCYCLE, MG_OP_RESIDUAL_RESTRICT, MG_OP_PRESMOOTH,
 MG_OP_POSTSMOOTH, MG_OP_PRESMOOTH_RESTRICT) = range(12)
(MG_K_SMOOTH, MG_K_RESIDUAL, MG_K_RESTRICT, MG_K_PROLONG, MG_K_COARSE, MG_K_REDUCE,
 MG_K_CAST, MG_K_UPDATE, MG_K_COPY, MG_K_COUNT) = range(10)


class mg_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("centering", C.c_int), ("coarsest_n", C.c_int)]


class mg_stencil(C.Structure):
    _fields_ = [("kind", C.c_int), ("k", C.POINTER(C.c_double)), ("k_on_device", C.c_int)]


class mg_bc(C.Structure):
    _fields_ = [("kind", C.c_int)]


class mg_opts(C.Structure):
    _fields_ = [("smoother", C.c_int), ("omega", C.c_double), ("nu1", C.c_int), ("nu2", C.c_int),
                ("precision", C.c_int), ("max_cycles", C.c_int), ("post_order", C.c_int), ("cycle", C.c_int),
                ("krylov", C.c_int), ("coarse_op", C.c_int)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_sigs = {
    "mg_version": (C.c_char_p, []),
    "mg_default_opts": (None, [C.POINTER(mg_opts)]),
    "mg_workspace_bytes": (C.c_int, [C.POINTER(mg_grid), C.POINTER(mg_stencil), C.POINTER(mg_opts),
                                     C.POINTER(C.c_size_t)]),
    "mg_setup": (C.c_int, [C.POINTER(mg_grid), C.POINTER(mg_stencil), C.POINTER(mg_bc), C.POINTER(mg_opts),
                           _P, C.c_size_t, _P, C.POINTER(_P)]),
    "mg_destroy": (None, [_P]),
    "mg_set_rhs": (C.c_int, [_P, _P, C.c_int]),
    "mg_set_initial": (C.c_int, [_P, _P, C.c_int]),
    "mg_get_solution": (C.c_int, [_P, _P, C.c_int]),
    "mg_vcycle": (C.c_int, [_P, C.c_int]),
    "mg_solve": (C.c_int, [_P, C.c_double, C.POINTER(C.c_int), _D]),
    "mg_fmg": (C.c_int, [_P, C.c_int]),
    "mg_pcg": (C.c_int, [_P, C.c_double, C.c_int, C.POINTER(C.c_int), _D]),
    "mg_residual_norm": (C.c_int, [_P, _D]),
    "mg_history": (C.c_int, [_P, _D, C.c_int, C.POINTER(C.c_int)]),
    "mg_levels": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "mg_level_size": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int)]),
    "mg_level_set": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, C.c_int]),
    "mg_level_get": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, C.c_int]),
    "mg_apply": (C.c_int, [_P, C.c_int, C.c_int, C.c_int]),
    "mg_profile": (C.c_int, [_P, C.c_int]),
    "mg_profile_read": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_int), _D]),
    "mg_graph_launches": (C.c_int, [_P, C.POINTER(C.c_longlong)]),
    "mg_strerror": (C.c_char_p, [C.c_int]),
    "mg_last_error": (C.c_char_p, [_P]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


class MGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{mg_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code: int, ctx=None):
    if code != MG_OK:
        raise MGError(code, mg_last_error(ctx).decode())
    return code


def make_grid(dim: int, n: int, centering: int = MG_NODE, coarsest: int | None = None) -> mg_grid:
    if coarsest is None:
        coarsest = 5 if centering == MG_NODE else 4
    g = mg_grid()
    g.dim = dim
    g.n[0] = g.n[1] = n
    g.n[2] = n if dim == 3 else 1
    g.centering = centering
    g.coarsest_n = coarsest
    return g


def make_opts(smoother=MG_RBGS, omega=0.8, nu1=2, nu2=2, precision=MG_FP64, max_cycles=100,
              post_order=0, cycle=0, krylov=0, coarse_op=0) -> mg_opts:
    o = mg_opts()
    o.smoother, o.omega, o.nu1, o.nu2 = smoother, omega, nu1, nu2
    o.precision, o.max_cycles, o.post_order, o.cycle, o.krylov = precision, max_cycles, post_order, cycle, krylov
    o.coarse_op = coarse_op
    return o


def workspace_bytes(grid: mg_grid, opts: mg_opts, stencil: mg_stencil | None = None) -> int:
    b = C.c_size_t()
    _check(mg_workspace_bytes(C.byref(grid), C.byref(stencil) if stencil else None, C.byref(opts),
                              C.byref(b)))
    return b.value


def _ptr(a):
    """(pointer, on_device, keepalive) for a NumPy array or a torch tensor of float64."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.dtype != torch.float64 or not a.is_contiguous():
                raise ValueError("tensors crossing the ABI must be contiguous float64")
            return C.c_void_p(a.data_ptr()), int(a.is_cuda), a
    except ImportError:
        pass
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return C.c_void_p(arr.ctypes.data), 0, arr


class Solver:
    """One multigrid context and the device workspace it lives in."""

    def __init__(self, dim: int, n: int, centering: int = MG_NODE, coarsest: int | None = None,
                 smoother: int = MG_RBGS, omega: float = 0.8, nu1: int = 2, nu2: int = 2,
                 precision: int = MG_FP64, max_cycles: int = 100, post_order: int = 0, cycle: int = 0,
                 krylov: int = 0, bc: int = 0, coarse_op: int = 0,
                 k=None, stream=None, device: str = "cuda"):
        import torch
        self.dim, self.n, self.centering = dim, n, centering
        self.grid = make_grid(dim, n, centering, coarsest)
        self.opts = make_opts(smoother, omega, nu1, nu2, precision, max_cycles, post_order, cycle, krylov,
                              coarse_op)
        self.stencil = mg_stencil()
        self._k = None
        if k is not None:
            kp, kd, self._k = _ptr(k)
            self.stencil.kind = MG_VARCOEF
            self.stencil.k = C.cast(kp, _D)
            self.stencil.k_on_device = kd
        else:
            self.stencil.kind = MG_LAPLACE
        self.bytes = workspace_bytes(self.grid, self.opts, self.stencil)
        self.workspace = torch.empty(max(self.bytes, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        bc = mg_bc(bc)
        h = C.c_void_p()
        _check(mg_setup(C.byref(self.grid), C.byref(self.stencil), C.byref(bc), C.byref(self.opts),
                        C.c_void_p(self.workspace.data_ptr()), self.bytes,
                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.ctx = h
        self._k = None

    # -------------------------------------------------------------- sizes
    @property
    def shape(self):
        return (self.n,) * self.dim

    def levels(self) -> int:
        v = C.c_int()
        _check(mg_levels(self.ctx, C.byref(v)), self.ctx)
        return v.value

    def level_size(self, level: int) -> int:
        v = C.c_int()
        _check(mg_level_size(self.ctx, level, C.byref(v)), self.ctx)
        return v.value

    # ------------------------------------------------------------ data
    def set_rhs(self, f):
        p, dev, keep = _ptr(f)
        _check(mg_set_rhs(self.ctx, p, dev), self.ctx)
        del keep

    def set_initial(self, u0=None):
        if u0 is None:
            _check(mg_set_initial(self.ctx, None, 0), self.ctx)
            return
        p, dev, keep = _ptr(u0)
        _check(mg_set_initial(self.ctx, p, dev), self.ctx)
        del keep

    def solution(self, out=None):
        if out is None:
            out = np.empty(self.shape, dtype=np.float64)
        p, dev, keep = _ptr(out)
        _check(mg_get_solution(self.ctx, p, dev), self.ctx)
        return out

    def level_set(self, level: int, field: int, a, prec: int = MG_PREC_FP64):
        p, dev, keep = _ptr(a)
        _check(mg_level_set(self.ctx, level, field, prec, p, dev), self.ctx)
        del keep

    def level_get(self, level: int, field: int, prec: int = MG_PREC_FP64):
        n = self.level_size(level)
        out = np.empty((n,) * self.dim, dtype=np.float64)
        _check(mg_level_get(self.ctx, level, field, prec, C.c_void_p(out.ctypes.data), 0), self.ctx)
        return out

    # --------------------------------------------------------- compute
    def apply(self, op: int, level: int = 0, prec: int = MG_PREC_FP64):
        _check(mg_apply(self.ctx, op, level, prec), self.ctx)

    def vcycle(self, k: int = 1):
        _check(mg_vcycle(self.ctx, k), self.ctx)

    def solve(self, tol: float):
        """Returns (status, cycles, relres); status is MG_OK or a convergence code."""
        cyc = C.c_int()
        rel = C.c_double()
        code = mg_solve(self.ctx, tol, C.byref(cyc), C.byref(rel))
        if code not in (MG_OK, MG_ENOTCONV, MG_ENONFINITE, MG_EDIVERGED):
            _check(code, self.ctx)
        return code, cyc.value, rel.value

    def residual_norm(self) -> float:
        v = C.c_double()
        _check(mg_residual_norm(self.ctx, C.byref(v)), self.ctx)
        return v.value

    def history(self) -> list:
        n = C.c_int()
        _check(mg_history(self.ctx, None, 0, C.byref(n)), self.ctx)
        buf = (C.c_double * max(n.value, 1))()
        _check(mg_history(self.ctx, buf, n.value, C.byref(n)), self.ctx)
        return list(buf[: n.value])

    # -------------------------------------------------------- profiling
    def profile(self, enable: bool = True):
        _check(mg_profile(self.ctx, int(enable)), self.ctx)

    def profile_read(self, kclass: int, level: int = -1):
        n = C.c_int()
        ms = C.c_double()
        _check(mg_profile_read(self.ctx, kclass, level, C.byref(n), C.byref(ms)), self.ctx)
        return n.value, ms.value

    def fmg(self, cycles_per_level: int = 1):
        """Full multigrid from the right-hand side; the result becomes the iterate."""
        _check(mg_fmg(self.ctx, cycles_per_level), self.ctx)

    def pcg(self, tol: float, max_it: int = 100):
        """Multigrid-preconditioned CG from the current iterate; returns (code, iterations, relres)."""
        its = C.c_int()
        rel = C.c_double()
        code = mg_pcg(self.ctx, tol, max_it, C.byref(its), C.byref(rel))
        if code not in (MG_OK, MG_ENOTCONV, MG_ENONFINITE):
            _check(code, self.ctx)
        return code, its.value, rel.value

    def graph_launches(self) -> int:
        n = C.c_longlong()
        _check(mg_graph_launches(self.ctx, C.byref(n)), self.ctx)
        return n.value

    def close(self):
        if getattr(self, "ctx", None):
            mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ===================================================================== serving
class mg_server_opts(C.Structure):
    _fields_ = [("d_arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_slots", C.c_int),
                ("max_queue", C.c_int), ("hip_stream", C.c_void_p)]


class mg_request(C.Structure):
    _fields_ = [("id", C.c_uint64), ("grid", mg_grid), ("opts", mg_opts), ("tol", C.c_double),
                ("f", C.c_void_p), ("u_out", C.c_void_p), ("t_arrive", C.c_double), ("deadline", C.c_double)]


class mg_result(C.Structure):
    _fields_ = [("id", C.c_uint64), ("ticket", C.c_uint64), ("status", C.c_int), ("steps", C.c_int),
                ("relres", C.c_double), ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class mg_server_stats(C.Structure):
    _fields_ = [("rounds", C.c_longlong), ("launches", C.c_longlong), ("admitted", C.c_longlong),
                ("completed", C.c_longlong), ("hierarchies_built", C.c_longlong), ("evictions", C.c_longlong),
                ("arena_peak_bytes", C.c_size_t), ("arena_used_bytes", C.c_size_t),
                ("in_flight", C.c_int), ("queued", C.c_int), ("resident", C.c_int),
                ("algorithmic_bytes", C.c_double)]


_EX_BUILD = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(mg_request))
_EX_STEP = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(mg_request),
                       C.POINTER(C.c_double))
_EX_FINISH = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(mg_request))
_EX_RELEASE = C.CFUNCTYPE(None, C.c_void_p, C.c_int)


class mg_server_executor(C.Structure):
    _fields_ = [("user", C.c_void_p), ("build", _EX_BUILD), ("step", _EX_STEP), ("finish", _EX_FINISH),
                ("release", _EX_RELEASE)]


_ssigs = {
    "mg_server_footprint": (C.c_int, [C.POINTER(mg_grid), C.POINTER(mg_opts), C.POINTER(C.c_size_t)]),
    "mg_server_create": (C.c_int, [C.POINTER(mg_server_opts), C.POINTER(_P)]),
    "mg_server_create_hosted": (C.c_int, [C.POINTER(mg_server_opts), C.POINTER(mg_server_executor), C.POINTER(_P)]),
    "mg_server_destroy": (None, [_P]),
    "mg_server_clock": (C.c_double, [_P]),
    "mg_server_submit": (C.c_int, [_P, C.POINTER(mg_request), C.POINTER(C.c_uint64)]),
    "mg_server_step": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "mg_server_cancel": (C.c_int, [_P, C.c_uint64]),
    "mg_server_poll": (C.c_int, [_P, C.POINTER(mg_result), C.c_int, C.POINTER(C.c_int)]),
    "mg_server_get_stats": (C.c_int, [_P, C.POINTER(mg_server_stats)]),
    "mg_server_last_error": (C.c_char_p, [_P]),
}
for _name, (_res, _args) in _ssigs.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


def server_footprint(dim: int, n: int, smoother: int, nu1: int, nu2: int, omega: float = 0.8) -> int:
    b = C.c_size_t()
    g = make_grid(dim, n)
    o = make_opts(smoother, omega, nu1, nu2, MG_MIXED)
    _check(mg_server_footprint(C.byref(g), C.byref(o), C.byref(b)))
    return b.value


class Server:
    """A solve server on a PyTorch-allocated device arena."""

    def __init__(self, arena_bytes: int, max_slots: int = 256, max_queue: int = 1 << 20, stream=None,
                 device: str = "cuda"):
        import torch
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        o = mg_server_opts()
        o.d_arena = self.arena.data_ptr()
        o.arena_bytes = arena_bytes
        o.max_slots = max_slots
        o.max_queue = max_queue
        o.hip_stream = self.stream.cuda_stream
        h = C.c_void_p()
        code = mg_server_create(C.byref(o), C.byref(h))
        if code != MG_OK:
            raise MGError(code, "server create")
        self.h = h
        self._keep = {}

    def _err(self, code):
        raise MGError(code, mg_server_last_error(self.h).decode())

    def clock(self) -> float:
        return mg_server_clock(self.h)

    def submit(self, rid: int, dim: int, n: int, f, u_out, tol: float, smoother: int = MG_RBGS,
               nu1: int = 2, nu2: int = 2, omega: float = 0.8, max_steps: int = 50, t_arrive=None,
               deadline: float = 0.0) -> int:
        """f and u_out: contiguous float64 CUDA tensors of shape (n,)*dim, kept
        alive here until the result is polled; deadline on the server clock
        (0: none).  Returns the status code; the ticket is in last_ticket."""
        r = mg_request()
        r.id = rid
        r.grid = make_grid(dim, n)
        r.opts = make_opts(smoother, omega, nu1, nu2, MG_MIXED, max_steps)
        r.tol = tol
        r.f = _address(f)
        r.u_out = _address(u_out)
        r.t_arrive = self.clock() if t_arrive is None else t_arrive
        r.deadline = deadline
        t = C.c_uint64()
        code = mg_server_submit(self.h, C.byref(r), C.byref(t))
        if code == MG_OK:
            self._keep[rid] = (f, u_out)
            self.last_ticket = t.value
        return code

    def cancel(self, ticket: int) -> int:
        """Cancel a queued or running request; returns the status code."""
        return mg_server_cancel(self.h, ticket)

    def step(self):
        a = C.c_int()
        q = C.c_int()
        code = mg_server_step(self.h, C.byref(a), C.byref(q))
        if code != MG_OK:
            self._err(code)
        return a.value, q.value

    def poll(self, cap: int = 4096) -> list:
        buf = (mg_result * cap)()
        n = C.c_int()
        _check(mg_server_poll(self.h, buf, cap, C.byref(n)))
        out = []
        for i in range(n.value):
            r = buf[i]
            out.append({"id": r.id, "ticket": r.ticket, "status": r.status, "steps": r.steps, "relres": r.relres,
                        "t_arrive": r.t_arrive, "t_admit": r.t_admit, "t_done": r.t_done})
            self._keep.pop(r.id, None)
        return out

    def stats(self) -> dict:
        st = mg_server_stats()
        _check(mg_server_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in mg_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            mg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _address(a) -> int:
    """Data address of a torch tensor or a NumPy array."""
    return a.data_ptr() if hasattr(a, "data_ptr") else a.ctypes.data


class HostedServer(Server):
    """The server's scheduler with its rounds run by a host executor instead
    of the batched device kernels (mg_server_create_hosted): no device work.
    The executor object provides build(slot, request),
    step(slots, first, requests) -> [(initial sum r^2, sum r^2), ...],
    finish(slot, request) and release(slot); requests are mg_request
    structures whose f and u_out hold the addresses of the arrays passed to
    submit.  An exception in a callback aborts the round with MG_EDEVICE."""

    def __init__(self, executor, arena_bytes: int, max_slots: int = 256, max_queue: int = 1 << 20):
        o = mg_server_opts()
        o.arena_bytes = arena_bytes
        o.max_slots = max_slots
        o.max_queue = max_queue
        self.executor = executor
        self.callback_error = None

        def guard(fn):
            def run(*a):
                try:
                    return fn(*a)
                except Exception as e:   # reported through the round's status
                    self.callback_error = e
                    return MG_EDEVICE
            return run

        @guard
        def build(_user, slot, req):
            executor.build(slot, req.contents)
            return MG_OK

        @guard
        def step(_user, count, slots, first, reqs, norms):
            out = executor.step([slots[i] for i in range(count)], [first[i] for i in range(count)],
                                [reqs[i] for i in range(count)])
            for i, (a, b) in enumerate(out):
                norms[2 * i] = a
                norms[2 * i + 1] = b
            return MG_OK

        @guard
        def finish(_user, slot, req):
            executor.finish(slot, req.contents)
            return MG_OK

        def release(_user, slot):
            try:
                executor.release(slot)
            except Exception as e:
                self.callback_error = e

        self._callbacks = (_EX_BUILD(build), _EX_STEP(step), _EX_FINISH(finish), _EX_RELEASE(release))
        ex = mg_server_executor(None, *self._callbacks)
        h = C.c_void_p()
        code = mg_server_create_hosted(C.byref(o), C.byref(ex), C.byref(h))
        if code != MG_OK:
            raise MGError(code, "hosted server create")
        self.h = h
        self._keep = {}


# ------------------------------------------- DG volume terms (include/dg.h)
_dsigs = {
    "dg_last_error": (C.c_char_p, []),
    "dg_basis_values": (C.c_int, [C.c_int, C.c_longlong, _D, _D, _D]),
    "dg_reference_size": (C.c_longlong, [C.c_int]),
    "dg_reference_integrals": (C.c_int, [C.c_int, _D]),
    "dg_volume_integrals": (C.c_int, [C.c_int, C.c_longlong, _P, _P, _P, _P, C.c_double, _P, _P, _P]),
    "dg_product_size": (C.c_longlong, [C.c_int]),
    "dg_product_integrals": (C.c_int, [C.c_int, _D]),
    "dg_velocity_projection": (C.c_int, [C.c_int, C.c_longlong, _P, _P, _P, _P, _P, _P]),
    "dg_edge_table_size": (C.c_longlong, [C.c_int]),
    "dg_edge_integrals": (C.c_int, [C.c_int, _D]),
    "dg_edge_terms": (C.c_int, [C.c_int, C.c_longlong, _P, _P, _P, _P, _P, _P, C.c_longlong, _P, _P,
                                C.c_double, _P, _P, _P]),
    "dg_rhs": (C.c_int, [C.c_int, C.c_longlong, _P, _P, _P, _P, _P, _P, C.c_longlong, _P, _P, C.c_double,
                         C.c_double, C.c_double, _P, _P, _P, _P, _P]),
    "dg_ssp_rk3_step": (C.c_int, [C.c_int, C.c_longlong, _P, _P, _P, _P, _P, _P, _P, C.c_longlong, _P, _P,
                                  C.c_double, C.c_double, C.c_double, _P, _P, _P, _P, C.c_double, _P]),
    "dg_ssp_rk3_step_noalloc": (C.c_int, [C.c_int, C.c_longlong, _P, _P, _P, _P, _P, _P, C.c_longlong, _P, _P,
                                          C.c_double, C.c_double, C.c_double, _P, _P, _P, _P, C.c_double, _P]),
}
for _name, (_res, _args) in _dsigs.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn

DG_K = {0: 1, 1: 3, 2: 6, 3: 10}
DG_KB = {0: 3, 1: 3, 2: 6, 3: 10}     # bathymetry coefficients; table order max(k, 1)


def _dgc(code: int):
    """Raise MGError for a failed dg_ entry point, with the library's reason."""
    if code != MG_OK:
        raise MGError(code, dg_last_error().decode())


def dg_basis(k: int, x, y) -> np.ndarray:
    """Values (K, n) of the reference basis of order k at the points (x, y) (host)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.ascontiguousarray(y, dtype=np.float64).ravel()
    if x.shape != y.shape:
        raise ValueError("x and y must have the same size")
    out = np.empty((DG_K[k], x.size), dtype=np.float64)
    _dgc(dg_basis_values(k, x.size, x.ctypes.data_as(_D), y.ctypes.data_as(_D), out.ctypes.data_as(_D)))
    return out


def dg_reference(k: int) -> np.ndarray:
    """The exact reference integrals for order k (host), over the first
    KB = DG_KB[k] basis functions: G (2, KB, KB), H (2, KB, KB, KB)."""
    K = DG_KB[k]
    ref = np.empty(int(dg_reference_size(k)), dtype=np.float64)
    _dgc(dg_reference_integrals(k, ref.ctypes.data_as(_D)))
    return ref[:2 * K * K].reshape(2, K, K), ref[2 * K * K:].reshape(2, K, K, K)


def dg_products(k: int) -> np.ndarray:
    """The exact triple-product integrals of order k (host): T (K, K, K)."""
    K = DG_K[k]
    T = np.empty(int(dg_product_size(k)), dtype=np.float64)
    _dgc(dg_product_integrals(k, T.ctypes.data_as(_D)))
    return T.reshape(K, K, K)


def _dg_check(tensors, ne):
    import torch
    for t, rows in tensors:
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (rows, ne):
            raise ValueError("expected contiguous FP64 device tensors of shape (rows, ne)")


def _dg_index(ne, *tensors):
    import torch
    for t in tensors:
        if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (3, ne):
            raise ValueError("nbr and nq must be contiguous int32 device tensors of shape (3, ne)")


def _dg_ghosts(K, nb, cb, ub, stages=1):
    """Pointers of the prescribed exterior states (NULL when nb = 0)."""
    import torch
    if nb == 0:
        return C.c_void_p(None), C.c_void_p(None)
    want = ((stages, 3 * K, nb), (stages, 2 * K, nb)) if stages > 1 else ((3 * K, nb), (2 * K, nb))
    for t, shape in zip((cb, ub), want):
        if t is None or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"expected contiguous FP64 device tensors of shapes {want}")
    return C.c_void_p(cb.data_ptr()), C.c_void_p(ub.data_ptr())


def _dptr(t):
    return C.c_void_p(None if t is None else t.data_ptr())


def _stream(st, dev):
    import torch
    return C.c_void_p((st if st is not None else torch.cuda.current_stream(dev)).cuda_stream)


class DGProjection:
    """Velocity projection of order k on the GPU; the product table lives on the device."""

    def __init__(self, k: int, device: str = "cuda"):
        import torch
        self.k, self.K, self.KB = k, DG_K[k], DG_KB[k]
        self.T = torch.from_numpy(dg_products(k).ravel().copy()).to(device)

    def __call__(self, c, B, hb, u, stream=None):
        """c (3K, ne), B (4, ne), hb (KB, ne) in; u (2K, ne) out."""
        ne = B.shape[1]
        _dg_check(((c, 3 * self.K), (B, 4), (hb, self.KB), (u, 2 * self.K)), ne)
        _dgc(dg_velocity_projection(self.k, ne, _dptr(c), _dptr(B), _dptr(hb), _dptr(self.T), _dptr(u),
                                      _stream(stream, B.device)))


DG_NB = {0: 2, 1: 2, 2: 3, 3: 4}     # Legendre coefficients of an edge trace, max(k, 1) + 1


def dg_edge_table(k: int) -> dict:
    """The exact edge-trace table for order k (host): C (3, KB, NB), the
    coefficients of the first KB = DG_KB[k] reference basis functions on
    each local edge in the shifted Legendre polynomials P_0 .. P_(NB-1) of
    the edge parameter."""
    t = np.empty(int(dg_edge_table_size(k)), dtype=np.float64)
    _dgc(dg_edge_integrals(k, t.ctypes.data_as(_D)))
    return {"raw": t, "C": t.reshape(3, DG_KB[k], DG_NB[k])}


class DGEdges:
    """Edge (Lax-Friedrichs) terms of order k on the GPU: interior edges and
    edges with a prescribed exterior state (nbr = -2 - b)."""

    def __init__(self, k: int, device: str = "cuda"):
        import torch
        self.k, self.K, self.KB = k, DG_K[k], DG_KB[k]
        self.tab = torch.from_numpy(dg_edge_table(k)["raw"].copy()).to(device)

    def __call__(self, c, u, B, hb, nbr, nq, g: float, out, cb=None, ub=None, stream=None):
        """c (3K, ne), u (2K, ne), B (4, ne), hb (KB, ne) FP64; nbr, nq (3, ne)
        int32; out (3K, ne); cb (3K, nb), ub (2K, nb) the prescribed states
        (None: nb = 0): contiguous device tensors."""
        ne = B.shape[1]
        _dg_check(((c, 3 * self.K), (u, 2 * self.K), (B, 4), (hb, self.KB), (out, 3 * self.K)), ne)
        _dg_index(ne, nbr, nq)
        nb = 0 if cb is None else cb.shape[1]
        pcb, pub = _dg_ghosts(self.K, nb, cb, ub)
        _dgc(dg_edge_terms(self.k, ne, _dptr(c), _dptr(u), _dptr(B), _dptr(hb), _dptr(nbr), _dptr(nq), nb, pcb, pub,
                             g, _dptr(self.tab), _dptr(out), _stream(stream, B.device)))


class DGVolume:
    """Volume terms of order k on the GPU; the reference table lives on the device."""

    def __init__(self, k: int, device: str = "cuda"):
        import torch
        self.k, self.K, self.KB = k, DG_K[k], DG_KB[k]
        G, H = dg_reference(k)
        self.ref = torch.from_numpy(np.concatenate([G.ravel(), H.ravel()])).to(device)

    def __call__(self, c, u, B, hb, g: float, out, stream=None):
        """c (3K, ne), u (2K, ne), B (4, ne), hb (KB, ne), out (3K, ne): contiguous
        FP64 device tensors, element index fastest."""
        ne = B.shape[1]
        _dg_check(((c, 3 * self.K), (u, 2 * self.K), (B, 4), (hb, self.KB), (out, 3 * self.K)), ne)
        _dgc(dg_volume_integrals(self.k, ne, _dptr(c), _dptr(u), _dptr(B), _dptr(hb), g, _dptr(self.ref), _dptr(out),
                                   _stream(stream, B.device)))


class DGSystem:
    """The semi-discrete shallow-water system of order k on a fixed mesh, on
    the GPU: dc/dt = E - S + R + F (dg_rhs) and the SSP-RK3 step
    (dg_ssp_rk3_step).  B (4, ne), hb (KB, ne) FP64 and nbr, nq (3, ne) int32
    device tensors; nb prescribed exterior states (nbr = -2 - b)."""

    def __init__(self, k: int, B, hb, nbr, nq, nb: int = 0, g: float = 9.81, tau: float = 0.0,
                 fc: float = 0.0):
        import torch
        self.k, self.K, self.KB = k, DG_K[k], DG_KB[k]
        self.ne, self.nb = B.shape[1], nb
        _dg_check(((B, 4), (hb, self.KB)), self.ne)
        _dg_index(self.ne, nbr, nq)
        self.B, self.hb, self.nbr, self.nq = B, hb, nbr, nq
        self.g, self.tau, self.fc = g, tau, fc
        dev = B.device
        G, H = dg_reference(k)
        self.ref = torch.from_numpy(np.concatenate([G.ravel(), H.ravel()])).to(dev)
        self.T = torch.from_numpy(dg_products(k).ravel().copy()).to(dev)
        self.tab = torch.from_numpy(dg_edge_table(k)["raw"].copy()).to(dev)
        self.work = torch.empty(6 * self.K * self.ne, dtype=torch.float64, device=dev)

    def project(self, c, u, stream=None):
        _dg_check(((c, 3 * self.K), (u, 2 * self.K)), self.ne)
        _dgc(dg_velocity_projection(self.k, self.ne, _dptr(c), _dptr(self.B), _dptr(self.hb), _dptr(self.T), _dptr(u),
                                      _stream(stream, c.device)))

    def rhs(self, c, u, out, cb=None, ub=None, F=None, stream=None):
        """out = dc/dt for the state c with velocity u; cb (3K, nb), ub (2K, nb)
        the prescribed states, F (3K, ne) the body force (None: none)."""
        _dg_check(((c, 3 * self.K), (u, 2 * self.K), (out, 3 * self.K)), self.ne)
        if F is not None:
            _dg_check(((F, 3 * self.K),), self.ne)
        pcb, pub = _dg_ghosts(self.K, self.nb, cb, ub)
        _dgc(dg_rhs(self.k, self.ne, _dptr(c), _dptr(u), _dptr(self.B), _dptr(self.hb), _dptr(self.nbr), _dptr(self.nq),
                      self.nb, pcb, pub, self.g, self.tau, self.fc, _dptr(F), _dptr(self.ref), _dptr(self.tab), _dptr(out),
                      _stream(stream, c.device)))

    def step(self, c, u, dt: float, cb3=None, ub3=None, F3=None, stream=None):
        """Advance c (3K, ne) in place by one SSP-RK3 step; u (2K, ne) is
        scratch for the stage velocities; cb3 (3, 3K, nb), ub3 (3, 2K, nb),
        F3 (3, 3K, ne) the data of the stages at t, t + dt, t + dt / 2."""
        import torch
        _dg_check(((c, 3 * self.K), (u, 2 * self.K)), self.ne)
        if F3 is not None:
            if (F3.dtype != torch.float64 or not F3.is_cuda or not F3.is_contiguous()
                    or tuple(F3.shape) != (3, 3 * self.K, self.ne)):
                raise ValueError("F3 must be a contiguous FP64 device tensor (3, 3K, ne)")
        pcb, pub = _dg_ghosts(self.K, self.nb, cb3, ub3, stages=3)
        _dgc(dg_ssp_rk3_step(self.k, self.ne, _dptr(c), _dptr(u), _dptr(self.work), _dptr(self.B), _dptr(self.hb),
                               _dptr(self.nbr), _dptr(self.nq), self.nb, pcb, pub, self.g, self.tau, self.fc, _dptr(F3),
                               _dptr(self.ref), _dptr(self.T), _dptr(self.tab), dt, _stream(stream, c.device)))

    def step_noalloc(self, c, u, dt: float, cb3=None, ub3=None, F3=None, stream=None):
        """As step, through dg_ssp_rk3_step_noalloc: the stage scratch is the
        library's fixed device array (6 K ne <= 2^23 doubles) instead of
        self.work."""
        import torch
        _dg_check(((c, 3 * self.K), (u, 2 * self.K)), self.ne)
        if F3 is not None:
            if (F3.dtype != torch.float64 or not F3.is_cuda or not F3.is_contiguous()
                    or tuple(F3.shape) != (3, 3 * self.K, self.ne)):
                raise ValueError("F3 must be a contiguous FP64 device tensor (3, 3K, ne)")
        pcb, pub = _dg_ghosts(self.K, self.nb, cb3, ub3, stages=3)
        _dgc(dg_ssp_rk3_step_noalloc(self.k, self.ne, _dptr(c), _dptr(u), _dptr(self.B), _dptr(self.hb),
                                       _dptr(self.nbr), _dptr(self.nq), self.nb, pcb, pub, self.g, self.tau, self.fc,
                                       _dptr(F3), _dptr(self.ref), _dptr(self.T), _dptr(self.tab), dt,
                                       _stream(stream, c.device)))
