"""Python binding of the C-ABI library ``liblbmgls.so`` (include/lbmgls.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides the device workspace (a uint8 tensor) and the HIP
stream; numpy arrays carry host inputs and outputs.  The library must have
been built (``__graft_entry__.build()``); nothing here falls back to any other
implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmgls.so")
DEVICE = "cuda"

STORAGE = {"fp64": 0, "fp32": 1, "fp16dev": 2, "bf16dev": 3}
ERRORS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_ENONFINITE", -5: "LBM_EUNSUPPORTED", -6: "LBM_ESTATE"}
EXPORTED = [
    "lbm_default_params", "lbm_workspace_bytes", "lbm_create", "lbm_step", "lbm_set_check", "lbm_check",
    "lbm_read", "lbm_mass", "lbm_energy", "lbm_steps_done", "lbm_state_bytes",
    "lbm_export_state", "lbm_import_state", "lbm_last_step_ms", "lbm_destroy",
    "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_add", "lbm_batch_remove",
    "lbm_batch_step", "lbm_batch_size", "lbm_batch_destroy", "lbm_last_error",
    "lbm_create_particles", "lbm_particles", "lbm_smooth_workspace_bytes", "lbm_smooth_solid",
    "lbm_smooth_solid_noalloc",
]
NOALLOC_MAX_NODES = 1 << 18  # LBM_NOALLOC_MAX_NODES of include/lbmgls.h
EXPORTED_3D = [  # include/lbmgls3d.h
    "lbm3_last_error", "lbm3_default_params", "lbm3_workspace_bytes", "lbm3_create", "lbm3_step",
    "lbm3_read", "lbm3_mass", "lbm3_energy", "lbm3_last_step_ms", "lbm3_destroy",
]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("d0", ctypes.c_double), ("sigma", ctypes.c_double), ("D", ctypes.c_double),
        ("M", ctypes.c_double), ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
        ("mu1", ctypes.c_double), ("mu2", ctypes.c_double), ("tau_phi", ctypes.c_double),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("s2", ctypes.c_double),
        ("s3", ctypes.c_double), ("s4", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("fbx", ctypes.c_double), ("fby", ctypes.c_double), ("solid_eps", ctypes.c_double),
        ("rep_xi", ctypes.c_double), ("rep_eps", ctypes.c_double),
        ("wall_x0", ctypes.c_double), ("wall_x1", ctypes.c_double),
        ("wall_y0", ctypes.c_double), ("wall_y1", ctypes.c_double),
        ("np", ctypes.c_int32), ("walls", ctypes.c_int32), ("bounce_y", ctypes.c_int32),
        ("bounce_x", ctypes.c_int32), ("h_form", ctypes.c_int32),
    ]


class Lbm3Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("d0", ctypes.c_double), ("sigma", ctypes.c_double), ("D", ctypes.c_double), ("M", ctypes.c_double),
        ("rho1", ctypes.c_double), ("rho2", ctypes.c_double), ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
        ("tau_phi", ctypes.c_double),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("s2", ctypes.c_double), ("s3", ctypes.c_double),
        ("s4", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("fbx", ctypes.c_double), ("fby", ctypes.c_double), ("fbz", ctypes.c_double),
        ("solid_eps", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def lib():
    """Load liblbmgls.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        if DEVICE == "cuda":
            # torch brings its own HIP runtime; load it first so that the
            # library binds to the same runtime (and device context) as the
            # tensors and streams it is handed
            _torch()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(LbmParams)
        P3 = ctypes.POINTER(Lbm3Params)
        sig = {
            "lbm_default_params": (None, [P, ctypes.c_int32, ctypes.c_int32]),
            "lbm_workspace_bytes": (ctypes.c_size_t, [P]),
            "lbm_create": (ctypes.c_int, [P, _VP, ctypes.c_size_t, _VP, _D, _D, _D, _D, _D,
                                          ctypes.POINTER(_VP)]),
            "lbm_step": (ctypes.c_int, [_VP, ctypes.c_int64]),
            "lbm_set_check": (ctypes.c_int, [_VP, ctypes.c_int64]),
            "lbm_check": (ctypes.c_int, [_VP]),
            "lbm_read": (ctypes.c_int, [_VP, _D, _D, _D, _D]),
            "lbm_mass": (ctypes.c_int, [_VP, _D]),
            "lbm_energy": (ctypes.c_int, [_VP, _D, _D]),
            "lbm_steps_done": (ctypes.c_int64, [_VP]),
            "lbm_state_bytes": (ctypes.c_size_t, [_VP]),
            "lbm_export_state": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
            "lbm_import_state": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
            "lbm_last_step_ms": (ctypes.c_double, [_VP]),
            "lbm_destroy": (ctypes.c_int, [_VP]),
            "lbm_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
            "lbm_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int64, _VP, ctypes.c_size_t, _VP,
                                                ctypes.POINTER(_VP)]),
            "lbm_batch_add": (ctypes.c_int, [_VP, _VP]),
            "lbm_batch_remove": (ctypes.c_int, [_VP, _VP]),
            "lbm_batch_step": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
            "lbm_batch_size": (ctypes.c_int, [_VP]),
            "lbm_batch_destroy": (ctypes.c_int, [_VP]),
            "lbm_last_error": (ctypes.c_char_p, []),
            "lbm_create_particles": (ctypes.c_int, [P, _VP, ctypes.c_size_t, _VP, _D, _D, _D, _D, _D, _D,
                                                    ctypes.POINTER(_VP)]),
            "lbm_particles": (ctypes.c_int, [_VP, _D, _D]),
            "lbm_smooth_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
            "lbm_smooth_solid": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_double, _VP, ctypes.c_size_t, _VP,
                                                _D, _D]),
            "lbm_smooth_solid_noalloc": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_double, _VP, _D, _D]),
            "lbm3_last_error": (ctypes.c_char_p, []),
            "lbm3_default_params": (None, [P3, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
            "lbm3_workspace_bytes": (ctypes.c_size_t, [P3]),
            "lbm3_create": (ctypes.c_int, [P3, _VP, ctypes.c_size_t, _VP, _D, _D, _D, _D, _D, _D,
                                           ctypes.POINTER(_VP)]),
            "lbm3_step": (ctypes.c_int, [_VP, ctypes.c_int64]),
            "lbm3_read": (ctypes.c_int, [_VP, _D, _D, _D, _D, _D]),
            "lbm3_mass": (ctypes.c_int, [_VP, _D]),
            "lbm3_energy": (ctypes.c_int, [_VP, _D, _D]),
            "lbm3_last_step_ms": (ctypes.c_double, [_VP]),
            "lbm3_destroy": (ctypes.c_int, [_VP]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise LbmError(rc, lib().lbm_last_error().decode())


def make_params(p: dict, storage: str | int = "fp32", tile: int = 0, np_: int = 0) -> LbmParams:
    lp = LbmParams()
    lib().lbm_default_params(ctypes.byref(lp), int(p["nx"]), int(p["ny"]))
    for name, _ in LbmParams._fields_:
        if name in p and name not in ("storage", "tile", "np"):
            setattr(lp, name, p[name])
    lp.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    lp.tile = int(tile)
    lp.np = int(np_)
    return lp


def _torch():
    import torch
    return torch


def current_stream_handle():
    torch = _torch()
    if DEVICE == "cuda":
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


def new_stream():
    """A new default-priority HIP stream: (torch stream, handle for the ABI)."""
    torch = _torch()
    s = torch.cuda.Stream()
    return s, ctypes.c_void_p(s.cuda_stream)


def alloc_workspace(nbytes: int):
    """A device uint8 tensor with a 256-byte aligned region of nbytes."""
    torch = _torch()
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=DEVICE)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off


def _arr(a, shape):
    if a is None:
        return None, None
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
    return a, a.ctypes.data_as(_D)


def workspace_bytes(params: dict, storage="fp32", tile=0, n_particles=0) -> int:
    lp = make_params(params, storage, tile, n_particles)
    n = lib().lbm_workspace_bytes(ctypes.byref(lp))
    if n == 0:
        raise LbmError(-1, lib().lbm_last_error().decode())
    return int(n)


class Domain:
    """One periodic nx x ny domain resident in GPU memory."""

    def __init__(self, params: dict, phi, phi0, cos_theta=None, ux=None, uy=None,
                 storage: str = "fp32", tile: int = 0, stream=None, particles=None):
        """particles: (np, 8) array, columns x, y, ux, uy, omega, R, rho_p,
        cos_theta (free rigid disks); phi0 and cos_theta are then the
        stationary solid only."""
        self.params = dict(params)
        self.storage = storage
        ny, nx = int(params["ny"]), int(params["nx"])
        self.shape = (ny, nx)
        parts = None if particles is None else np.ascontiguousarray(np.reshape(particles, (-1, 8)),
                                                                    dtype=np.float64)
        self.n_particles = 0 if parts is None else len(parts)
        self._lp = make_params(params, storage, tile, self.n_particles)
        self.nbytes = lib().lbm_workspace_bytes(ctypes.byref(self._lp))
        if self.nbytes == 0:
            raise LbmError(-1, lib().lbm_last_error().decode())
        self._ws, ptr = alloc_workspace(self.nbytes)
        self._stream = stream if stream is not None else current_stream_handle()
        keep = [_arr(a, self.shape) for a in (phi, phi0, cos_theta, ux, uy)]
        h = _VP()
        if self.n_particles:
            _check(lib().lbm_create_particles(ctypes.byref(self._lp), _VP(ptr), self.nbytes, self._stream,
                                              *[k[1] for k in keep], parts.ctypes.data_as(_D), ctypes.byref(h)))
        else:
            _check(lib().lbm_create(ctypes.byref(self._lp), _VP(ptr), self.nbytes, self._stream,
                                    *[k[1] for k in keep], ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            # the workspace may still be in use by work queued on another
            # stream than the allocator's: drain before releasing it
            if DEVICE == "cuda":
                _torch().cuda.synchronize()
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(lib().lbm_step(self._h, int(n)))

    def set_check(self, every: int):
        _check(lib().lbm_set_check(self._h, int(every)))

    def check(self) -> bool:
        """True if phi, u and P are finite; False (and the domain refuses further
        steps) otherwise."""
        rc = lib().lbm_check(self._h)
        if rc == -4:
            return False
        _check(rc)
        return True

    @property
    def steps(self) -> int:
        return int(lib().lbm_steps_done(self._h))

    @property
    def last_step_ms(self) -> float:
        return float(lib().lbm_last_step_ms(self._h))

    def read(self):
        """phi, ux, uy, P as (ny, nx) float64 arrays at the current level."""
        out = [np.empty(self.shape) for _ in range(4)]
        _check(lib().lbm_read(self._h, *[o.ctypes.data_as(_D) for o in out]))
        return tuple(out)

    def mass(self) -> float:
        m = ctypes.c_double()
        _check(lib().lbm_mass(self._h, ctypes.byref(m)))
        return m.value

    def energy(self):
        ef, ek = ctypes.c_double(), ctypes.c_double()
        _check(lib().lbm_energy(self._h, ctypes.byref(ef), ctypes.byref(ek)))
        return ef.value, ek.value

    def particles(self):
        """(state (np, 8), outputs of the last update (np, 7)): x, y, ux, uy,
        omega, R, rho_p, cos_theta; F_f x, y, T_f, F^in x, y, T^in, rho_in."""
        st = np.zeros((self.n_particles, 8))
        out = np.zeros((self.n_particles, 7))
        if self.n_particles:
            _check(lib().lbm_particles(self._h, st.ctypes.data_as(_D), out.ctypes.data_as(_D)))
        return st, out

    def export_state(self) -> bytes:
        n = lib().lbm_state_bytes(self._h)
        buf = ctypes.create_string_buffer(n)
        _check(lib().lbm_export_state(self._h, ctypes.cast(buf, _VP), n))
        return buf.raw

    def import_state(self, state: bytes):
        buf = ctypes.create_string_buffer(state, len(state))
        _check(lib().lbm_import_state(self._h, ctypes.cast(buf, _VP), len(state)))


def smooth_solid(params: dict, solid, iters: int = 20, dtau: float = 0.0):
    """phi0 from a voxel solid by `iters` steps of the smoothing
    Cahn-Hilliard equation on the GPU (lbm_smooth_solid); params supplies
    nx, ny, D and the walls."""
    solid, sp = _arr(solid, (params["ny"], params["nx"]))
    nbytes = lib().lbm_smooth_workspace_bytes(int(params["nx"]), int(params["ny"]))
    if nbytes == 0:
        raise LbmError(-1, "invalid grid size")
    buf, ptr = alloc_workspace(nbytes)
    out = np.zeros_like(solid)
    lp = make_params(params)
    _check(lib().lbm_smooth_solid(ctypes.byref(lp), int(iters), float(dtau), _VP(ptr), nbytes,
                                  current_stream_handle(), sp, out.ctypes.data_as(_D)))
    del buf
    return out


def smooth_solid_noalloc(params: dict, solid, iters: int = 20, dtau: float = 0.0):
    """As smooth_solid, through the allocation-free entry point
    (lbm_smooth_solid_noalloc): no workspace, grids of at most
    NOALLOC_MAX_NODES nodes."""
    solid, sp = _arr(solid, (params["ny"], params["nx"]))
    out = np.zeros_like(solid)
    lp = make_params(params)
    _check(lib().lbm_smooth_solid_noalloc(ctypes.byref(lp), int(iters), float(dtau), current_stream_handle(), sp,
                                          out.ctypes.data_as(_D)))
    return out


class Batch:
    """Several domains advanced by one fused launch per step (HIP graph)."""

    def __init__(self, storage: str = "fp32", tile: int = 0, max_members: int = 64,
                 max_tiles: int = 1 << 20, stream=None):
        """stream: ABI handle of a created stream; a new one by default.
        Members must be created with ``stream=batch.stream``."""
        self.storage = storage
        n = lib().lbm_batch_workspace_bytes(int(max_members), int(max_tiles))
        self._ws, ptr = alloc_workspace(n)
        if stream is None:
            self._torch_stream, stream = new_stream()
        self._stream = stream
        h = _VP()
        _check(lib().lbm_batch_create(STORAGE[storage], int(tile), int(max_members), int(max_tiles),
                                      _VP(ptr), n, self._stream, ctypes.byref(h)))
        self._h = h
        self.members: list[Domain] = []

    @property
    def stream(self):
        return self._stream

    def domain(self, params: dict, *arrays, tile: int = 0) -> "Domain":
        """Create a domain on this batch's stream (not yet a member)."""
        d = Domain(params, *arrays, storage=self.storage, tile=tile, stream=self._stream)
        d._stream_owner = getattr(self, "_torch_stream", None)
        return d

    def add(self, d: Domain):
        _check(lib().lbm_batch_add(self._h, d.handle))
        self.members.append(d)

    def remove(self, d: Domain):
        _check(lib().lbm_batch_remove(self._h, d.handle))
        self.members.remove(d)

    def step(self, n: int, budget=None):
        if budget is None:
            _check(lib().lbm_batch_step(self._h, int(n), None))
        else:
            arr = (ctypes.c_int64 * len(budget))(*[int(b) for b in budget])
            _check(lib().lbm_batch_step(self._h, int(n), arr))

    def __len__(self):
        return int(lib().lbm_batch_size(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- 3-D path
def _check3(rc: int):
    if rc != 0:
        raise LbmError(rc, lib().lbm3_last_error().decode())


def make_params3(p: dict, storage: str | int = "fp64") -> Lbm3Params:
    lp = Lbm3Params()
    lib().lbm3_default_params(ctypes.byref(lp), int(p["nx"]), int(p["ny"]), int(p["nz"]))
    for name, _ in Lbm3Params._fields_:
        if name in p and name != "storage":
            setattr(lp, name, p[name])
    lp.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    return lp


class Domain3:
    """One periodic nx x ny x nz domain (lbmgls3d.h) resident in GPU memory;
    fields are (nz, ny, nx) arrays."""

    def __init__(self, params: dict, phi, phi0, cos_theta=None, ux=None, uy=None, uz=None,
                 storage: str = "fp64", stream=None):
        self.params = dict(params)
        self.storage = storage
        self.shape = (int(params["nz"]), int(params["ny"]), int(params["nx"]))
        self._lp = make_params3(params, storage)
        self.nbytes = lib().lbm3_workspace_bytes(ctypes.byref(self._lp))
        if self.nbytes == 0:
            raise LbmError(-1, lib().lbm3_last_error().decode())
        self._ws, ptr = alloc_workspace(self.nbytes)
        self._stream = stream if stream is not None else current_stream_handle()
        keep = [_arr(a, self.shape) for a in (phi, phi0, cos_theta, ux, uy, uz)]
        h = _VP()
        _check3(lib().lbm3_create(ctypes.byref(self._lp), _VP(ptr), self.nbytes, self._stream,
                                  *[k[1] for k in keep], ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            if DEVICE == "cuda":
                _torch().cuda.synchronize()
            lib().lbm3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check3(lib().lbm3_step(self._h, int(n)))

    @property
    def last_step_ms(self) -> float:
        return float(lib().lbm3_last_step_ms(self._h))

    def read(self):
        """phi, ux, uy, uz, P at the current level."""
        out = [np.empty(self.shape) for _ in range(5)]
        _check3(lib().lbm3_read(self._h, *[o.ctypes.data_as(_D) for o in out]))
        return tuple(out)

    def mass(self) -> float:
        m = ctypes.c_double()
        _check3(lib().lbm3_mass(self._h, ctypes.byref(m)))
        return m.value

    def energy(self):
        ef, ek = ctypes.c_double(), ctypes.c_double()
        _check3(lib().lbm3_energy(self._h, ctypes.byref(ef), ctypes.byref(ek)))
        return ef.value, ek.value
