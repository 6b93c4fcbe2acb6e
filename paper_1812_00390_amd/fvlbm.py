"""Python binding of the C ABI in include/fvlbm.h (libfvlbm.so, gfx950).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch provides the device memory of the solver state and the
stream.  There is no CPU fallback: without the built library every entry
point raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfvlbm.so")

EULER, RK4, AB2 = 0, 1, 2
FP32, FP32_DEV, FP16_DEV, I16_DEV = 0, 1, 2, 3
REORDER_NONE, REORDER_RCM, REORDER_HILBERT, REORDER_BISECT = 0, 1, 2, 3
SCHEMES = {"euler": EULER, "rk4": RK4, "ab2": AB2}
STORAGES = {"fp32": FP32, "fp32dev": FP32_DEV, "fp16dev": FP16_DEV, "i16dev": I16_DEV}
FLAG_FORCE_DT = 1

STATUS = {0: "OK", -1: "E_ARG", -2: "E_MESH", -3: "E_PARAM", -4: "E_NOMEM", -5: "E_DEVICE",
          -6: "E_DIVERGED", -7: "E_STATE"}


class FvlbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fvlbm {STATUS.get(status, status)}: {msg}")
        self.status = status


class BC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("internal", C.c_int32), ("u", C.c_double * 2), ("rho", C.c_double)]


class Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("dt", C.c_double), ("cfl", C.c_double), ("u_ref", C.c_double),
                ("scheme", C.c_int32), ("storage", C.c_int32), ("rho0", C.c_double),
                ("fp16_scale", C.c_double), ("residual_lag", C.c_int32), ("flags", C.c_int32),
                ("u_dev", C.c_double * 2)]


_lib = None

# every function the header declares, with (restype, argtypes)
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
SIGNATURES = {
    "fvlbm_create_mesh": (C.c_int, [C.c_int32, _dp, C.c_int32, _ip, _ip, C.c_int32, _ip, _ip, C.c_int32,
                                    C.POINTER(BC), C.c_int32, _ip, _dp, C.c_int32, _vp, C.POINTER(_vp)]),
    "fvlbm_mesh_info": (C.c_int, [_vp, C.POINTER(C.c_int64)]),
    "fvlbm_mesh_cfl_length": (C.c_double, [_vp]),
    "fvlbm_state_bytes": (C.c_size_t, [_vp, C.POINTER(Params)]),
    "fvlbm_init": (C.c_int, [_vp, C.POINTER(Params), _dp, _dp, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "fvlbm_solver_dt": (C.c_double, [_vp]),
    "fvlbm_step": (C.c_int, [_vp, C.c_int64]),
    "fvlbm_prepare": (C.c_int, [_vp, C.c_int64]),
    "fvlbm_macros": (C.c_int, [_vp, _dp, _dp, _dp]),
    "fvlbm_macros_noalloc": (C.c_int, [_vp, _vp, _vp, _vp]),
    "fvlbm_get_f": (C.c_int, [_vp, _dp]),
    "fvlbm_set_f": (C.c_int, [_vp, _dp]),
    "fvlbm_rhs": (C.c_int, [_vp, _dp]),
    "fvlbm_wall_force": (C.c_int, [_vp, C.c_int32, _dp, C.POINTER(C.c_int32), _dp]),
    "fvlbm_checkpoint_bytes": (C.c_size_t, [_vp]),
    "fvlbm_checkpoint": (C.c_int, [_vp, _vp, C.c_size_t]),
    "fvlbm_restore": (C.c_int, [_vp, _vp, C.c_size_t]),
    "fvlbm_solver_destroy": (None, [_vp]),
    "fvlbm_mesh_destroy": (None, [_vp]),
    "fvlbm_batch_create": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(_vp)]),
    "fvlbm_batch_step": (C.c_int, [_vp, C.c_int64]),
    "fvlbm_batch_destroy": (None, [_vp]),
    "fvlbm_set_schedule": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32]),
    "fvlbm_get_schedule": (C.c_int, [_vp, _ip, _ip, _ip]),
    "fvlbm_batch_set_schedule": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32]),
    "fvlbm_batch_get_schedule": (C.c_int, [_vp, _ip, _ip, _ip]),
    "fvlbm_batch_residuals": (C.c_int, [_vp, _dp]),
    "fvlbm_batch_set_members": (C.c_int, [_vp, C.POINTER(_vp), C.c_int32]),
    "fvlbm_batch_remove": (C.c_int, [_vp, _vp]),
    "fvlbm_batch_graph_counts": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "fvlbm_set_stream": (C.c_int, [_vp, _vp]),
    "fvlbm_autotune": (C.c_int, [_vp, C.c_int32, _dp]),
    "fvlbm_batch_autotune": (C.c_int, [_vp, C.c_int32, _dp]),
    "fvlbm_last_error": (C.c_char_p, []),
}


def lib():
    """Load libfvlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1812_00390_amd/build.py "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise FvlbmError(st, lib().fvlbm_last_error().decode())


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(_ip)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("fvlbm needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_handle(stream=None):
    if isinstance(stream, int) and stream == 0:
        return C.c_void_p(None)          # the null stream, without touching torch
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Mesh:
    """A mesh resident on the device (fvlbm_create_mesh)."""

    def __init__(self, raw, reorder: int = REORDER_BISECT, stream=None):
        L = lib()
        self.raw = raw
        self.n_cells = raw.n_cells
        xy = np.ascontiguousarray(raw.nodes, dtype=np.float64).reshape(-1)
        ptr = np.ascontiguousarray(raw.cell_ptr, dtype=np.int32)
        cn = np.ascontiguousarray(raw.cell_nodes, dtype=np.int32)
        bfn = np.ascontiguousarray(raw.bface_nodes, dtype=np.int32).reshape(-1)
        bfg = np.ascontiguousarray(raw.bface_group, dtype=np.int32)
        ng = len(raw.groups)
        groups = (BC * max(ng, 1))()
        for i, g in enumerate(raw.groups):
            groups[i].kind = g.kind
            groups[i].internal = g.internal
            groups[i].u[0], groups[i].u[1] = g.u
            groups[i].rho = g.rho
        per = np.ascontiguousarray(raw.periodic, dtype=np.int32).reshape(-1)
        sh = np.ascontiguousarray(raw.periodic_shift, dtype=np.float64).reshape(-1)
        if per.size == 0:
            per = np.zeros(2, np.int32); sh = np.zeros(2)
        if bfn.size == 0:
            bfn = np.zeros(2, np.int32); bfg = np.zeros(1, np.int32)
        h = C.c_void_p()
        _check(L.fvlbm_create_mesh(raw.n_nodes, _dptr(xy), raw.n_cells, _iptr(ptr), _iptr(cn),
                                   int(raw.bface_nodes.shape[0]), _iptr(bfn), _iptr(bfg), ng, groups,
                                   int(raw.periodic.shape[0]), _iptr(per), _dptr(sh), int(reorder),
                                   _stream_handle(stream), C.byref(h)))
        self.h = h
        self._solvers = weakref.WeakSet()     # solvers on this mesh, closed before it

    def info(self) -> dict:
        out = (C.c_int64 * 4)()
        _check(lib().fvlbm_mesh_info(self.h, out))
        return dict(n_cells=out[0], nf=out[1], bytes=out[2], boundary_cells=out[3])

    @property
    def cfl_length(self) -> float:
        return lib().fvlbm_mesh_cfl_length(self.h)

    def close(self):
        """Release the mesh; solvers still open on it are closed first.  (The
        library also keeps a mesh alive while solvers use it, so either order
        of destruction is safe, including under the cycle collector.)"""
        if getattr(self, "h", None):
            for s in list(getattr(self, "_solvers", ())):
                s.close()
            lib().fvlbm_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(tau: float, dt: float = 0.0, cfl: float = 0.5, u_ref: float = 0.1, scheme="euler",
                storage="fp32", rho0: float = 1.0, fp16_scale: float = 0.0, residual_lag: int = 1000,
                flags: int = 0, u_dev=(0.0, 0.0)) -> Params:
    p = Params()
    p.tau, p.dt, p.cfl, p.u_ref = tau, dt, cfl, u_ref
    p.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    p.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
    p.rho0, p.fp16_scale, p.residual_lag, p.flags = rho0, fp16_scale, residual_lag, flags
    p.u_dev[0], p.u_dev[1] = float(u_dev[0]), float(u_dev[1])
    return p


def state_bytes(mesh: Mesh, params: Params) -> int:
    return int(lib().fvlbm_state_bytes(mesh.h, C.byref(params)))


class Solver:
    """One solve: Step 0 at construction, then step()/macros() (fvlbm_init ...)."""

    def __init__(self, mesh: Mesh, params: Params, rho=None, u=None, stream=None):
        torch = _torch()
        L = lib()
        self.mesh = mesh
        self.params = params
        self.n = mesh.n_cells
        nbytes = state_bytes(mesh, params)
        if nbytes == 0:
            raise FvlbmError(-1, "bad parameters")
        # caller-owned state buffer (torch), 256-byte aligned
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._buf.data_ptr()
        off = (-base) % 256
        self.buf_ptr = base + off
        self.nbytes = nbytes
        self.stream = stream
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        h = C.c_void_p()
        _check(L.fvlbm_init(mesh.h, C.byref(params), _dptr(r), _dptr(v), C.c_void_p(self.buf_ptr),
                            nbytes, _stream_handle(stream), C.byref(h)))
        self.h = h
        mesh._solvers.add(self)

    @property
    def dt(self) -> float:
        return lib().fvlbm_solver_dt(self.h)

    def step(self, n: int = 1):
        _check(lib().fvlbm_step(self.h, int(n)))

    def prepare(self, n: int):
        """Instantiate the launch graphs a step(n) call from here would replay (runs nothing)."""
        _check(lib().fvlbm_prepare(self.h, int(n)))

    def macros(self):
        rho = np.zeros(self.n); u = np.zeros((self.n, 2)); st = np.zeros(4)
        _check(lib().fvlbm_macros(self.h, _dptr(rho), _dptr(u), _dptr(st)))
        return rho, u, dict(mass=st[0], residual=st[1], t=st[2], steps=int(st[3]))

    def macros_noalloc(self, rho=None, u=None, stats=None):
        """Step 6 into device tensors (float64; rho [n], u [n, 2], stats [2] = mass, non-finite
        flag), enqueued on the solver's stream without allocating or syncing."""
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        _check(lib().fvlbm_macros_noalloc(self.h, ptr(rho), ptr(u), ptr(stats)))

    def stats(self) -> dict:
        st = np.zeros(4)
        _check(lib().fvlbm_macros(self.h, None, None, _dptr(st)))
        return dict(mass=st[0], residual=st[1], t=st[2], steps=int(st[3]))

    @property
    def f(self) -> np.ndarray:
        out = np.zeros((self.n, 9))
        _check(lib().fvlbm_get_f(self.h, _dptr(out)))
        return out

    @f.setter
    def f(self, value):
        a = np.ascontiguousarray(value, dtype=np.float64).reshape(self.n, 9)
        _check(lib().fvlbm_set_f(self.h, _dptr(a)))

    def rhs(self) -> np.ndarray:
        out = np.zeros((self.n, 9))
        _check(lib().fvlbm_rhs(self.h, _dptr(out)))
        return out

    def wall_force(self, group: int):
        """Force the fluid exerts on wall group `group` (Fx, Fy) and p = rho/3 at each of its faces
        (the order of the mesh's boundary-face arrays)."""
        n = C.c_int32(0)
        _check(lib().fvlbm_wall_force(self.h, int(group), None, C.byref(n), None))
        force = np.zeros(2)
        face_p = np.zeros(max(1, n.value))
        _check(lib().fvlbm_wall_force(self.h, int(group), _dptr(force), C.byref(n), _dptr(face_p)))
        return force, face_p[:n.value]

    def checkpoint(self) -> bytes:
        nb = int(lib().fvlbm_checkpoint_bytes(self.h))
        buf = C.create_string_buffer(nb)
        _check(lib().fvlbm_checkpoint(self.h, buf, nb))
        return buf.raw

    def restore(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(lib().fvlbm_restore(self.h, buf, len(data)))

    def set_schedule(self, block: int, xcd_remap: bool = True, persistent: int = 0):
        """persistent: 0 (or False) one workgroup per tile, 1 (True) a resident
        grid walking the tiles, 2 one workgroup per tile plus a wave for the halo
        slots (tiles of 64 or 128 cells; Euler and RK stages)."""
        _check(lib().fvlbm_set_schedule(self.h, int(block), int(bool(xcd_remap)), int(persistent)))

    def set_stream(self, stream):
        """Move the solver's later work to `stream` (a torch stream, or 0 for the null stream)."""
        _check(lib().fvlbm_set_stream(self.h, _stream_handle(stream)))
        self.stream = stream

    def get_schedule(self):
        b, x, p = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().fvlbm_get_schedule(self.h, C.byref(b), C.byref(x), C.byref(p)))
        return dict(block=b.value, xcd_remap=bool(x.value), persistent=int(p.value))

    def autotune(self, trial_steps: int = 64) -> float:
        """Pick the fastest launch schedule (state restored afterwards); returns ms per step."""
        ms = C.c_double()
        _check(lib().fvlbm_autotune(self.h, int(trial_steps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().fvlbm_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several solvers advanced by shared launches (fvlbm_batch_*)."""

    def __init__(self, solvers: Sequence[Solver]):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = C.c_void_p()
        _check(lib().fvlbm_batch_create(arr, len(self.solvers), C.byref(h)))
        self.h = h

    def step(self, n: int):
        _check(lib().fvlbm_batch_step(self.h, int(n)))

    def set_members(self, solvers: Sequence[Solver]):
        """Replace the members, keeping the schedule and re-pointing the instantiated graphs."""
        solvers = list(solvers)
        arr = (C.c_void_p * len(solvers))(*[s.h.value for s in solvers])
        _check(lib().fvlbm_batch_set_members(self.h, arr, len(solvers)))
        self.solvers = solvers

    def remove(self, solver: Solver):
        """Remove one member (fvlbm_batch_remove); the others keep their order and the graphs."""
        _check(lib().fvlbm_batch_remove(self.h, solver.h))
        self.solvers = [s for s in self.solvers if s is not solver]

    def graph_counts(self) -> dict:
        """Graphs instantiated so far, and graphs re-pointed by membership changes."""
        b, r = C.c_int64(), C.c_int64()
        _check(lib().fvlbm_batch_graph_counts(self.h, C.byref(b), C.byref(r)))
        return dict(built=b.value, repointed=r.value)

    def set_schedule(self, block: int, xcd_remap: bool = True, persistent: bool = False):
        _check(lib().fvlbm_batch_set_schedule(self.h, int(block), int(bool(xcd_remap)), int(bool(persistent))))

    def get_schedule(self) -> dict:
        """The schedule the batch launches with (as the library holds it)."""
        b, x, p = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().fvlbm_batch_get_schedule(self.h, C.byref(b), C.byref(x), C.byref(p)))
        return dict(block=b.value, xcd_remap=bool(x.value), persistent=bool(p.value))

    def residuals(self):
        """(residual, steps) of every member, one sync: residual of Eq. 32 over the lag, -1 if none yet."""
        out = np.zeros(2 * len(self.solvers))
        _check(lib().fvlbm_batch_residuals(self.h, _dptr(out)))
        return out[0::2].copy(), out[1::2].astype(np.int64)

    def autotune(self, trial_steps: int = 64) -> float:
        """Pick the fastest launch schedule for the whole batch (states restored); ms per step."""
        ms = C.c_double()
        _check(lib().fvlbm_batch_autotune(self.h, int(trial_steps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().fvlbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
