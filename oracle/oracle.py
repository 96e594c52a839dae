"""ctypes wrapper around the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: this module is imported by the test suite, by the
smoke check and by the CPU-baseline leg of the benchmark.  The GPU library
and its Python binding never import it.

The oracle itself is plain C (FP64, scalar, literal 9x9 matrix collision); this
file only marshals numpy arrays.  See the header of ``lbm_oracle.c`` for the
paper passages it follows and the readings it takes.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

# -O2 without -march=native: the library built here also runs on the GPU
# host.  -ffp-contract=off keeps every product and sum rounded separately, as
# written.
CFLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``liblbm_oracle.so`` next to its source."""
    if force or not os.path.exists(LIB):
        # a name of its own per process: concurrent test workers may all
        # find the library stale and build it at once; the rename is atomic
        tmp = "%s.%d.tmp" % (LIB, os.getpid())
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
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
        ("walls", ctypes.c_int32), ("bounce_y", ctypes.c_int32),
        ("bounce_x", ctypes.c_int32), ("h_form", ctypes.c_int32),
    ]


# parameters of the free-particle extension; absent keys take these values
OPTIONAL = {"rep_xi": 0.0, "rep_eps": 1.0, "wall_x0": 0.0, "wall_x1": 0.0, "wall_y0": 0.0,
            "wall_y1": 0.0, "walls": 0, "bounce_y": 0,
            "bounce_x": 0, "h_form": 0}
# particle state columns (input) and per-particle outputs of the last update
PARTICLE_IN = ["x", "y", "ux", "uy", "omega", "R", "rho_p", "cos_theta"]
PARTICLE_OUT = ["Fx", "Fy", "T", "Fin_x", "Fin_y", "Tin", "rho_in"]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        L.orc_create.argtypes = [ctypes.POINTER(OrcParams), _D, _D, _D, _D, _D,
                                 ctypes.POINTER(ctypes.c_void_p)]
        L.orc_create.restype = ctypes.c_int
        L.orc_create_particles.argtypes = [ctypes.POINTER(OrcParams), _D, _D, _D, _D, _D,
                                           ctypes.c_int, _D, ctypes.POINTER(ctypes.c_void_p)]
        L.orc_create_particles.restype = ctypes.c_int
        L.orc_nparticles.argtypes = [ctypes.c_void_p]
        L.orc_nparticles.restype = ctypes.c_int
        L.orc_get_particles.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_repulsion.argtypes = [ctypes.c_double] * 5 + [_D]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_steps_done.argtypes = [ctypes.c_void_p]
        L.orc_steps_done.restype = ctypes.c_long
        L.orc_nfields.restype = ctypes.c_int
        L.orc_field_name.argtypes = [ctypes.c_int]
        L.orc_field_name.restype = ctypes.c_char_p
        L.orc_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.orc_get_field.restype = ctypes.c_int
        L.orc_get_pops.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_mass.argtypes = [ctypes.c_void_p]
        L.orc_vox_dtau.argtypes = [ctypes.c_double]
        L.orc_vox_dtau.restype = ctypes.c_double
        L.orc_smooth_solid.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                             _D, _D]
        L.orc_smooth_chi.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                           _D, _D]
        L.orc_mass.restype = ctypes.c_double
        L.orc_energy.argtypes = [ctypes.c_void_p, _D, _D]
        L.orc_lattice.argtypes = [ctypes.c_double, _D, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]
        L.orc_matrices.argtypes = [ctypes.c_double, _D, _D, _D, _D]
        L.orc_collision_matrix.argtypes = [ctypes.c_double, _D, _D]
        L.orc_geq.argtypes = [ctypes.c_double] * 6 + [_D]
        L.orc_gsrc.argtypes = [ctypes.c_double] * 3 + [_D]
        L.orc_feq.argtypes = [ctypes.c_double] * 7 + [_D]
        L.orc_fsrc.argtypes = [ctypes.c_double] * 12 + [_D]
        L.orc_grad.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D]
        L.orc_lap.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_mu.argtypes = [ctypes.POINTER(OrcParams), _D, _D, _D, _D]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_plant.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_plant.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_params(p: dict) -> OrcParams:
    op = OrcParams()
    for name, _ in OrcParams._fields_:
        setattr(op, name, p[name] if name in p else OPTIONAL[name])
    return op


# terms a test may scale to plant a mistake (names of the PL_* factors in
# lbm_oracle.c, in order)
PLANT_TERMS = ["H", "KDT", "G", "FC", "FEQS", "M2FDT", "M2FUF", "M2FD0", "M2FISO", "UDR"]


@contextlib.contextmanager
def planted(**factors):
    """Run the enclosed oracle steps with some terms of the method scaled
    (e.g. ``planted(FC=-1.0)`` flips the sign of F_c), to show that a pin
    fails on that mistake.  Every factor is restored to 1 on exit."""
    L = lib()
    try:
        for name, v in factors.items():
            assert L.orc_plant(PLANT_TERMS.index(name), float(v)) == 0
        yield
    finally:
        L.orc_plant_reset()


def threads() -> int:
    """OpenMP threads the collision loop uses."""
    return int(lib().orc_threads())


def set_threads(n: int):
    """Threads of the collision loop for the following steps."""
    lib().orc_set_threads(int(n))


def build_native(path: str) -> str:
    """The same source built for the host it runs on (-O3 -march=native), into
    `path`: the CPU-baseline timing build.  Arithmetic is still unfused
    (-ffp-contract=off)."""
    flags = ["-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]
    tmp = path + ".tmp"
    subprocess.check_call(["gcc", *flags, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, path)
    return path


def use_library(path: str):
    """Load the oracle from another build of the same source (before the
    first call into it)."""
    global LIB, _lib
    assert _lib is None, "the oracle library is already loaded"
    LIB = path


# ---------------------------------------------------------------- unit level
def lattice(d0: float):
    w = np.zeros(9)
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    lib().orc_lattice(d0, _ptr(w), cx, cy)
    return w, np.array(list(cx)), np.array(list(cy))


def matrices(d0: float):
    out = [np.zeros(81) for _ in range(4)]
    lib().orc_matrices(d0, *[_ptr(a) for a in out])
    return [a.reshape(9, 9) for a in out]  # M0, NH, MH, MHinv


def collision_matrix(d0: float, s) -> np.ndarray:
    s = _c64(s)
    lam = np.zeros(81)
    lib().orc_collision_matrix(d0, _ptr(s), _ptr(lam))
    return lam.reshape(9, 9)


def geq(d0, eta, phi, mu, ux, uy):
    out = np.zeros(9)
    lib().orc_geq(d0, eta, phi, mu, ux, uy, _ptr(out))
    return out


def gsrc(d0, dtphiux, dtphiuy):
    out = np.zeros(9)
    lib().orc_gsrc(d0, dtphiux, dtphiuy, _ptr(out))
    return out


def feq(d0, P, rho, ux, uy, Sx, Sy):
    out = np.zeros(9)
    lib().orc_feq(d0, P, rho, ux, uy, Sx, Sy, _ptr(out))
    return out


def fsrc(d0, ux, uy, drx, dry, Fx, Fy, rfx, rfy, M2xx, M2xy, M2yy):
    out = np.zeros(9)
    lib().orc_fsrc(d0, ux, uy, drx, dry, Fx, Fy, rfx, rfy, M2xx, M2xy, M2yy, _ptr(out))
    return out


def grad(chi: np.ndarray):
    chi = _c64(chi)
    ny, nx = chi.shape
    gx, gy = np.zeros_like(chi), np.zeros_like(chi)
    lib().orc_grad(nx, ny, _ptr(chi), _ptr(gx), _ptr(gy))
    return gx, gy


def lap(chi: np.ndarray):
    chi = _c64(chi)
    ny, nx = chi.shape
    out = np.zeros_like(chi)
    lib().orc_lap(nx, ny, _ptr(chi), _ptr(out))
    return out


def mu(params: dict, phi, phi0, psi):
    phi, phi0, psi = _c64(phi), _c64(phi0), _c64(psi)
    ny, nx = phi.shape
    p = dict(params, nx=nx, ny=ny)
    out = np.zeros_like(phi)
    op = make_params(p)
    lib().orc_mu(ctypes.byref(op), _ptr(phi), _ptr(phi0), _ptr(psi), _ptr(out))
    return out


def vox_dtau(D: float) -> float:
    return lib().orc_vox_dtau(D)


def smooth_solid(solid, D: float, iters: int = 20, dtau: float = 0.0, bounce_x: int = 0,
                 bounce_y: int = 0) -> np.ndarray:
    """phi0 from a voxel solid (R-VOX)."""
    s = _c64(solid)
    ny, nx = s.shape
    out = np.zeros_like(s)
    lib().orc_smooth_solid(nx, ny, int(bounce_x), int(bounce_y), D, int(iters), dtau, _ptr(s), _ptr(out))
    return out


def smooth_chi(chi, D: float, iters: int, dtau: float = 0.0, bounce_x: int = 0, bounce_y: int = 0):
    c = _c64(chi)
    ny, nx = c.shape
    out = np.zeros_like(c)
    lib().orc_smooth_chi(nx, ny, int(bounce_x), int(bounce_y), D, int(iters), dtau, _ptr(c), _ptr(out))
    return out


# ---------------------------------------------------------------- stepper
class Oracle:
    """FP64 CPU stepper.  Fields are numpy arrays of shape (ny, nx)."""

    def __init__(self, params: dict, phi, phi0, cos_theta=None, ux=None, uy=None, particles=None):
        """phi0, cos_theta: the stationary solid.  particles: (np, 8) array of
        x, y, ux, uy, omega, R, rho_p, cos_theta per free particle."""
        phi = _c64(phi)
        ny, nx = phi.shape
        assert params["nx"] == nx and params["ny"] == ny
        self.params = dict(params)
        self.shape = (ny, nx)
        self._keep = [phi, _c64(phi0)]
        ct = None if cos_theta is None else _c64(np.broadcast_to(cos_theta, phi.shape))
        uxa = None if ux is None else _c64(np.broadcast_to(ux, phi.shape))
        uya = None if uy is None else _c64(np.broadcast_to(uy, phi.shape))
        self._keep += [ct, uxa, uya]
        parts = np.zeros((0, 8)) if particles is None else _c64(np.reshape(particles, (-1, 8)))
        self._keep.append(parts)
        self.np = len(parts)
        op = make_params(self.params)
        h = ctypes.c_void_p()
        rc = lib().orc_create_particles(ctypes.byref(op), _ptr(self._keep[0]), _ptr(self._keep[1]),
                                        None if ct is None else _ptr(ct),
                                        None if uxa is None else _ptr(uxa),
                                        None if uya is None else _ptr(uya), self.np,
                                        _ptr(parts) if self.np else None, ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self._h = h
        names = [lib().orc_field_name(k).decode() for k in range(lib().orc_nfields())]
        self._fid = {n: k for k, n in enumerate(names)}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_destroy(h)
            self._h = None

    @property
    def steps(self) -> int:
        return lib().orc_steps_done(self._h)

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def field(self, name: str) -> np.ndarray:
        out = np.zeros(self.shape)
        rc = lib().orc_get_field(self._h, self._fid[name], _ptr(out))
        assert rc == 0
        return out

    def fields(self):
        return {n: self.field(n) for n in self._fid}

    def read(self):
        """phi, ux, uy, P at the current level."""
        return self.field("phi"), self.field("ux"), self.field("uy"), self.field("P")

    def pops(self):
        ny, nx = self.shape
        g = np.zeros((9, ny, nx))
        f = np.zeros((9, ny, nx))
        lib().orc_get_pops(self._h, _ptr(g), _ptr(f))
        return g, f

    def mass(self) -> float:
        return lib().orc_mass(self._h)

    def particles(self):
        """(state (np, 8), outputs of the last update (np, 7)); columns as in
        PARTICLE_IN and PARTICLE_OUT."""
        st = np.zeros((self.np, 8))
        out = np.zeros((self.np, 7))
        if self.np:
            lib().orc_get_particles(self._h, _ptr(st), _ptr(out))
        return st, out

    def energy(self):
        ef, ek = ctypes.c_double(), ctypes.c_double()
        lib().orc_energy(self._h, ctypes.byref(ef), ctypes.byref(ek))
        return ef.value, ek.value


def macro_node(params: dict, f, rho, muv, phi0, Fx, Fy, Sx, Sy, drx, dry, q_p,
               u0x=0.0, u0y=0.0, init=False, usolx=0.0, usoly=0.0):
    """Steps 5-6 at one node: returns dict u*, f dt, u, s2a, s2b, H, P."""
    L = lib()
    if not getattr(L, "_macro_node_set", False):
        L.orc_macro_node.argtypes = ([ctypes.POINTER(OrcParams), ctypes.c_int, _D]
                                     + [ctypes.c_double] * 14 + [_D])
        L._macro_node_set = True
    p = dict(params)
    p.setdefault("nx", 1)
    p.setdefault("ny", 1)
    op = make_params(p)
    f = _c64(f)
    out = np.zeros(10)
    L.orc_macro_node(ctypes.byref(op), int(init), _ptr(f), rho, muv, phi0, Fx, Fy, Sx, Sy,
                     drx, dry, q_p, u0x, u0y, usolx, usoly, _ptr(out))
    keys = ["usx", "usy", "ax", "ay", "ux", "uy", "s2a", "s2b", "H", "P"]
    return dict(zip(keys, out))


def repulsion(dx: float, dy: float, rsum: float, xi: float, eps: float) -> np.ndarray:
    """Short-range repulsion of Sec. 4.5 on a particle whose centre is (dx, dy)
    from the other centre (or from its mirror image across a wall)."""
    out = np.zeros(2)
    lib().orc_repulsion(dx, dy, rsum, xi, eps, _ptr(out))
    return out
