"""ctypes wrapper around the three-dimensional FP64 CPU oracle
(``lbm3d_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; the GPU library and its binding never
import it.  The oracle's header lists the paper passages it follows and the
readings it takes for three dimensions.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm3d_oracle.c")
LIB = os.path.join(HERE, "liblbm3d_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]
Q = 15


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = "%s.%d.tmp" % (LIB, os.getpid())
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Orc3Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("d0", ctypes.c_double), ("sigma", ctypes.c_double), ("D", ctypes.c_double), ("M", ctypes.c_double),
        ("rho1", ctypes.c_double), ("rho2", ctypes.c_double), ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
        ("tau_phi", ctypes.c_double),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("s2", ctypes.c_double), ("s3", ctypes.c_double),
        ("s4", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("fbx", ctypes.c_double), ("fby", ctypes.c_double), ("fbz", ctypes.c_double),
        ("solid_eps", ctypes.c_double),
    ]


OPTIONAL = {"pad": 0, "gx": 0.0, "gy": 0.0, "gz": 0.0, "rho_ref": 0.0, "fbx": 0.0, "fby": 0.0, "fbz": 0.0}
PLANT_TERMS = {"H": 0, "KDT": 1, "G": 2, "FC": 3, "ISO": 4, "UDR": 5}

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(Orc3Params)
        L.orc3_create.argtypes = [P, _D, _D, _D, _D, _D, _D, ctypes.POINTER(ctypes.c_void_p)]
        L.orc3_create.restype = ctypes.c_int
        L.orc3_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc3_destroy.argtypes = [ctypes.c_void_p]
        L.orc3_steps_done.argtypes = [ctypes.c_void_p]
        L.orc3_steps_done.restype = ctypes.c_long
        L.orc3_nfields.restype = ctypes.c_int
        L.orc3_field_name.argtypes = [ctypes.c_int]
        L.orc3_field_name.restype = ctypes.c_char_p
        L.orc3_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.orc3_get_field.restype = ctypes.c_int
        L.orc3_get_pops.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc3_set_pops.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc3_mass.argtypes = [ctypes.c_void_p]
        L.orc3_mass.restype = ctypes.c_double
        L.orc3_energy.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc3_lattice.argtypes = [ctypes.c_double, _D, _I, _I, _I]
        L.orc3_matrices.argtypes = [ctypes.c_double, _D, _D, _D, _D]
        L.orc3_matrices.restype = ctypes.c_int
        L.orc3_collision_matrix.argtypes = [ctypes.c_double, _D, _D]
        L.orc3_geq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc3_gsrc.argtypes = [ctypes.c_double, _D, _D]
        L.orc3_feq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc3_fsrc.argtypes = [ctypes.c_double, _D, _D, _D, _D, _D, _D]
        L.orc3_macro_node.argtypes = [P, ctypes.c_int, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      _D, _D, _D, ctypes.c_double, _D, _D]
        L.orc3_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        L.orc3_lap.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc3_plant.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc3_plant.restype = ctypes.c_int
        L.orc3_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(p: dict) -> Orc3Params:
    q = dict(OPTIONAL)
    q.update(p)
    return Orc3Params(**{k: q[k] for k, _ in Orc3Params._fields_})


@contextlib.contextmanager
def planted(**factors):
    """Scale terms of the method (keys of PLANT_TERMS) inside the block."""
    L = lib()
    try:
        for k, v in factors.items():
            assert L.orc3_plant(PLANT_TERMS[k], float(v)) == 0
        yield
    finally:
        L.orc3_plant_reset()


def set_threads(n: int):
    lib().orc3_set_threads(int(n))


def lattice(d0: float):
    w = np.zeros(Q)
    c = [np.zeros(Q, dtype=np.int32) for _ in range(3)]
    lib().orc3_lattice(d0, _ptr(w), *[x.ctypes.data_as(_I) for x in c])
    return w, np.stack(c, axis=1).astype(np.int64)


def matrices(d0: float):
    m0, nh, mh, mhi = (np.zeros((Q, Q)) for _ in range(4))
    assert lib().orc3_matrices(d0, _ptr(m0), _ptr(nh), _ptr(mh), _ptr(mhi)) == 0
    return m0, nh, mh, mhi


def collision_matrix(d0: float, s) -> np.ndarray:
    lam = np.zeros((Q, Q))
    lib().orc3_collision_matrix(d0, _ptr(_c64(s)), _ptr(lam))
    return lam


def geq(d0, eta, phi, mu, u):
    out = np.zeros(Q)
    lib().orc3_geq(d0, eta, phi, mu, _ptr(_c64(u)), _ptr(out))
    return out


def gsrc(d0, dtphiu):
    out = np.zeros(Q)
    lib().orc3_gsrc(d0, _ptr(_c64(dtphiu)), _ptr(out))
    return out


def feq(d0, P, rho, u, S):
    out = np.zeros(Q)
    lib().orc3_feq(d0, P, rho, _ptr(_c64(u)), _ptr(_c64(S)), _ptr(out))
    return out


def fsrc(d0, u, drho, F, rf, M2):
    out = np.zeros(Q)
    lib().orc3_fsrc(d0, _ptr(_c64(u)), _ptr(_c64(drho)), _ptr(_c64(F)), _ptr(_c64(rf)), _ptr(_c64(M2)),
                    _ptr(out))
    return out


def macro_node(params: dict, f, rho, muv, phi0, F, S, drho, q_p, u0=(0.0, 0.0, 0.0), init=False):
    """u* (3), f dt (3), u (3), s2a, s2b, H, P at one node."""
    out = np.zeros(13)
    op = make_params(params)
    lib().orc3_macro_node(ctypes.byref(op), int(init), _ptr(_c64(f)), rho, muv, phi0, _ptr(_c64(F)),
                          _ptr(_c64(S)), _ptr(_c64(drho)), q_p, _ptr(_c64(u0)), _ptr(out))
    return out


def grad(chi):
    chi = _c64(chi)
    nz, ny, nx = chi.shape
    g = [np.zeros_like(chi) for _ in range(3)]
    lib().orc3_grad(nx, ny, nz, _ptr(chi), *[_ptr(x) for x in g])
    return g


def lap(chi):
    chi = _c64(chi)
    nz, ny, nx = chi.shape
    out = np.zeros_like(chi)
    lib().orc3_lap(nx, ny, nz, _ptr(chi), _ptr(out))
    return out


class Oracle3:
    """FP64 CPU stepper in three dimensions.  Fields are (nz, ny, nx)."""

    def __init__(self, params: dict, phi, phi0, cos_theta=None, ux=None, uy=None, uz=None):
        phi = _c64(phi)
        nz, ny, nx = phi.shape
        assert (params["nx"], params["ny"], params["nz"]) == (nx, ny, nz)
        self.params = dict(params)
        self.shape = phi.shape

        def b(a):
            return None if a is None else _c64(np.broadcast_to(a, phi.shape))

        self._keep = [phi, _c64(phi0), b(cos_theta), b(ux), b(uy), b(uz)]
        op = make_params(self.params)
        h = ctypes.c_void_p()
        rc = lib().orc3_create(ctypes.byref(op), *[_ptr(a) for a in self._keep], ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"orc3_create failed ({rc})")
        self._h = h
        self._fid = {lib().orc3_field_name(k).decode(): k for k in range(lib().orc3_nfields())}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.orc3_destroy(h)
            self._h = None

    @property
    def steps(self) -> int:
        return lib().orc3_steps_done(self._h)

    def step(self, n: int = 1):
        lib().orc3_step(self._h, int(n))

    def field(self, name: str) -> np.ndarray:
        out = np.zeros(self.shape)
        assert lib().orc3_get_field(self._h, self._fid[name], _ptr(out)) == 0
        return out

    def read(self):
        """phi, ux, uy, uz, P at the current level."""
        return tuple(self.field(k) for k in ("phi", "ux", "uy", "uz", "P"))

    def pops(self):
        g = np.zeros((Q,) + self.shape)
        f = np.zeros((Q,) + self.shape)
        lib().orc3_get_pops(self._h, _ptr(g), _ptr(f))
        return g, f

    def set_pops(self, g=None, f=None):
        lib().orc3_set_pops(self._h, _ptr(None if g is None else _c64(g)), _ptr(None if f is None else _c64(f)))

    def mass(self) -> float:
        return lib().orc3_mass(self._h)

    def energy(self):
        ef, ek = ctypes.c_double(), ctypes.c_double()
        lib().orc3_energy(self._h, ctypes.byref(ef), ctypes.byref(ek))
        return ef.value, ek.value
