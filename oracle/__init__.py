"""FP64 CPU oracle for the SRT and SmrtLBM D2Q9 lattice Boltzmann updates.

TEST INFRASTRUCTURE ONLY.  Written from Zhou, "Single MRT-featured Lattice
Boltzmann Method" (arXiv:2409.01076) to check the GPU library; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the GPU path.

Arrays are numpy float64.  Lattice populations are node-major,
``f[y, x, a]`` with shape ``(ny, nx, 9)``; fields are ``(ny, nx)``.

Which passage each function follows:
  equilibrium      Eq. (feq-full)
  node_moments     Eq. (fea-0)
  node_collide     Eq. (lb.srt), Eq. (SmrtLBM-1), Eq. (SmrtLBM-lb.1.5)
  stream           left-hand side of those equations (f moves along e_a),
                   with the "standard bounce-back" walls and the moving lid of
                   the cavity section (readings: half-way walls, moving-wall
                   correction with rho_w = 1, lid owns the corner links; or
                   the second lid reading, an equilibrium lid on the top row)
  tau_from_re      Eq. (relation-chapman-viscosity) with Re = U N / nu
  reduce           sums for the steady-state residual (a reading; the paper
                   does not define its steady-state test)
"""
import ctypes
import os

import numpy as np

SRT, SMRT, TRT = 0, 1, 2
SCHEMES = {"srt": SRT, "smrt": SMRT, "trt": TRT}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsmrt_oracle.so")
_lib = None


class _Lattice(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("periodic_x", ctypes.c_int), ("periodic_y", ctypes.c_int),
        ("scheme", ctypes.c_int),
        ("tau", ctypes.c_double), ("tau_s", ctypes.c_double), ("u_lid", ctypes.c_double),
        ("lid", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(_Lattice)
    lib.oracle_constants.argtypes = [ip, ip, dp, ip]
    lib.oracle_constants.restype = None
    lib.oracle_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
    lib.oracle_equilibrium.restype = None
    lib.oracle_node_moments.argtypes = [dp, dp, dp, dp]
    lib.oracle_node_moments.restype = None
    lib.oracle_node_collide.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.oracle_node_collide.restype = ctypes.c_int
    lib.oracle_init_equilibrium.argtypes = [lp, dp, dp, dp, dp]
    lib.oracle_collide_lattice.argtypes = [lp, dp, dp]
    lib.oracle_stream_lattice.argtypes = [lp, dp, dp]
    lib.oracle_run.argtypes = [lp, dp, ctypes.c_long]
    lib.oracle_fields.argtypes = [lp, dp, dp, dp, dp]
    lib.oracle_reduce.argtypes = [ctypes.c_long, dp, dp, dp, dp, dp, dp]
    for name in ("oracle_init_equilibrium", "oracle_collide_lattice", "oracle_stream_lattice",
                 "oracle_run", "oracle_fields", "oracle_reduce"):
        getattr(lib, name).restype = ctypes.c_int
    lib.oracle_tau_from_re.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_tau_from_re.restype = ctypes.c_double
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_get_threads.argtypes = []
    lib.oracle_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments" % what)


def constants():
    """(ex, ey, w, opp) as numpy arrays, in the paper's D2Q9 order."""
    lib = _load()
    ex = (ctypes.c_int * 9)()
    ey = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    opp = (ctypes.c_int * 9)()
    lib.oracle_constants(ex, ey, w, opp)
    return (np.array(ex[:], dtype=np.int64), np.array(ey[:], dtype=np.int64),
            np.array(w[:], dtype=np.float64), np.array(opp[:], dtype=np.int64))


def equilibrium(rho, ux, uy):
    """f^eq of one node, Eq. (feq-full)."""
    out = np.empty(9)
    _load().oracle_equilibrium(float(rho), float(ux), float(uy), _ptr(out))
    return out


def node_moments(f):
    """(rho, ux, uy) of one node, Eq. (fea-0)."""
    f = _as_f64(f, (9,))
    r, x, y = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _load().oracle_node_moments(_ptr(f), ctypes.byref(r), ctypes.byref(x), ctypes.byref(y))
    return r.value, x.value, y.value


def node_collide(f, scheme, tau, tau_s=1.0):
    """Post-collision populations of one node for 'srt', 'smrt' or 'trt'."""
    f = _as_f64(f, (9,))
    out = np.empty(9)
    _check(_load().oracle_node_collide(SCHEMES[scheme], float(tau), float(tau_s), _ptr(f),
                                       _ptr(out)), "node_collide")
    return out


class Lattice:
    """Geometry and collision parameters of one oracle lattice.

    ``boundary`` is 'periodic' (both axes wrap), 'cavity' (walls on all four
    sides, the top one moving at ``u_lid``) or 'channel' (x wraps, walls at
    the bottom and top, the top moving at ``u_lid``).  ``lid`` is 'wall'
    (moving-wall bounce-back half a link above the top row) or 'equilibrium'
    (the top row is the lid, set each step to the equilibrium at (u_lid, 0)
    with the density its incoming populations give).
    """

    def __init__(self, nx, ny, scheme="smrt", tau=None, re=None, u_lid=0.0,
                 boundary="cavity", tau_s=1.0, lid="wall"):
        if tau is None:
            if re is None:
                raise ValueError("give tau or re")
            tau = tau_from_re(re, u_lid, nx)
        px, py = {"periodic": (1, 1), "cavity": (0, 0), "channel": (1, 0)}[boundary]
        self.nx, self.ny = int(nx), int(ny)
        self.scheme, self.tau, self.tau_s = scheme, float(tau), float(tau_s)
        self.u_lid, self.boundary = float(u_lid), boundary
        self.lid = lid
        self._c = _Lattice(self.nx, self.ny, px, py, SCHEMES[scheme], self.tau, self.tau_s,
                           self.u_lid, {"wall": 0, "equilibrium": 1}[lid])

    @property
    def shape(self):
        return (self.ny, self.nx, 9)

    def init_equilibrium(self, rho=None, ux=None, uy=None):
        """Populations f = f^eq(rho, u) at every node (defaults rho=1, u=0)."""
        s = (self.ny, self.nx)
        rho = np.ones(s) if rho is None else _as_f64(rho, s)
        ux = np.zeros(s) if ux is None else _as_f64(ux, s)
        uy = np.zeros(s) if uy is None else _as_f64(uy, s)
        f = np.empty(self.shape)
        _check(_load().oracle_init_equilibrium(ctypes.byref(self._c), _ptr(rho), _ptr(ux),
                                               _ptr(uy), _ptr(f)), "init_equilibrium")
        return f

    def collide(self, f):
        f = _as_f64(f, self.shape)
        out = np.empty(self.shape)
        _check(_load().oracle_collide_lattice(ctypes.byref(self._c), _ptr(f), _ptr(out)),
               "collide")
        return out

    def stream(self, fstar):
        fstar = _as_f64(fstar, self.shape)
        out = np.empty(self.shape)
        _check(_load().oracle_stream_lattice(ctypes.byref(self._c), _ptr(fstar), _ptr(out)),
               "stream")
        return out

    def run(self, f, nsteps):
        """Returns the populations after ``nsteps`` of collide-then-stream."""
        f = np.array(_as_f64(f, self.shape), copy=True)
        _check(_load().oracle_run(ctypes.byref(self._c), _ptr(f), int(nsteps)), "run")
        return f

    def fields(self, f):
        """(rho, ux, uy), each (ny, nx)."""
        f = _as_f64(f, self.shape)
        s = (self.ny, self.nx)
        rho, ux, uy = np.empty(s), np.empty(s), np.empty(s)
        _check(_load().oracle_fields(ctypes.byref(self._c), _ptr(f), _ptr(rho), _ptr(ux),
                                     _ptr(uy)), "fields")
        return rho, ux, uy


def reduce(rho, ux, uy, ux_snap, uy_snap):
    """Fixed-order FP64 sums: (sum|u-u_snap|^2, sum|u|^2, sum rho, #non-finite)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel()
            for a in (rho, ux, uy, ux_snap, uy_snap)]
    n = arrs[0].size
    if any(a.size != n for a in arrs):
        raise ValueError("reduce: size mismatch")
    out = np.empty(4)
    _check(_load().oracle_reduce(n, *[_ptr(a) for a in arrs], _ptr(out)), "reduce")
    return tuple(float(v) for v in out)


def residual(ux, uy, ux_snap, uy_snap, window):
    """R_K = ||u - u_snap||_2 / (K ||u||_2): the steady-state residual reading."""
    du2, u2, _, _ = reduce(np.ones_like(np.asarray(ux, dtype=np.float64)), ux, uy, ux_snap,
                           uy_snap)
    return float(np.sqrt(du2) / (window * np.sqrt(u2)))


def tau_from_re(re, u_lid, n):
    """tau for Re = U N / nu, Eq. (relation-chapman-viscosity) in lattice units."""
    return float(_load().oracle_tau_from_re(float(re), float(u_lid), int(n)))


def set_threads(n):
    return int(_load().oracle_set_threads(int(n)))


def get_threads():
    return int(_load().oracle_get_threads())
