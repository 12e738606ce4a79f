"""Python binding of the gfx950 D2Q9 SRT / SmrtLBM library (``include/smrt.h``).

Argument marshalling only: every step of the lattice update runs in the HIP
kernels of ``libsmrt.so``.  PyTorch provides device memory (the workspace and
the field/population tensors) and the stream.  There is no CPU fallback: on a
machine without the built library or without a GPU, creating a solver raises.
"""
import contextlib
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmrt.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
SCHEMES = {"srt": 0, "smrt": 1, "trt": 2}
BOUNDARIES = {"cavity": 0, "periodic": 1, "cavity_eqlid": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f32x": 4, "m64": 5, "m16": 6, "mbf16": 7}
_IO_DTYPES = {torch.float64: 0, torch.float32: 1}

EXPORTED = (
    "smrt_workspace_bytes", "smrt_create", "smrt_init_fields", "smrt_set_populations",
    "smrt_get_populations", "smrt_step", "smrt_moments", "smrt_residual", "smrt_mass",
    "smrt_mass_noalloc", "smrt_steps_done", "smrt_tau", "smrt_set_launch", "smrt_set_steps_per_launch",
    "smrt_get_steps_per_launch", "smrt_set_tile_order",
    "smrt_synchronize", "smrt_destroy",
    "smrt_last_error", "smrt_copy_kernel",
    "smrt_batch_workspace_bytes", "smrt_batch_create", "smrt_batch_step", "smrt_batch_run",
    "smrt_batch_autotune", "smrt_batch_moments", "smrt_batch_init_fields", "smrt_batch_steps_done",
    "smrt_batch_running", "smrt_batch_steps_per_launch", "smrt_batch_set_launch", "smrt_batch_destroy",
    "smrt_mlp_param_count", "smrt_mlp_workspace_bytes", "smrt_mlp_create", "smrt_mlp_set_params",
    "smrt_mlp_get_params", "smrt_mlp_forward", "smrt_mlp_gradient", "smrt_mlp_train_step",
    "smrt_mlp_destroy", "smrt_mlp_set_fused_forward", "smrt_mlp_uses_fused_forward", "smrt_gemm_bf16",
)
RUNNING, STEADY, UNSTABLE = 0, 1, 2


class SmrtError(RuntimeError):
    """A negative status returned by the library."""

    def __init__(self, code, message):
        super().__init__("%s (status %d)" % (message, code))
        self.code = code


class UnstableError(SmrtError):
    """The lattice holds a non-finite density or velocity."""


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("boundary", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("tau", ctypes.c_double), ("re", ctypes.c_double),
        ("u_lid", ctypes.c_double), ("tau_s", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("reserved", ctypes.c_int64 * 4),
    ]


class BatchParams(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("nx", ctypes.POINTER(ctypes.c_int32)), ("ny", ctypes.POINTER(ctypes.c_int32)),
        ("tau", ctypes.POINTER(ctypes.c_double)), ("re", ctypes.POINTER(ctypes.c_double)),
        ("u_lid", ctypes.c_double), ("tau_s", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("reserved", ctypes.c_int64 * 4),
    ]


class MlpParams(ctypes.Structure):
    _fields_ = [
        ("inputs", ctypes.c_int32), ("fourier", ctypes.c_int32), ("width", ctypes.c_int32),
        ("layers", ctypes.c_int32), ("outputs", ctypes.c_int32), ("max_batch", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("reserved", ctypes.c_int64 * 4),
    ]


_lib = None


def load():
    """Loads libsmrt.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(Params)
    sig = {
        "smrt_workspace_bytes": (ctypes.c_size_t, [pp]),
        "smrt_create": (ctypes.c_int, [pp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
        "smrt_init_fields": (ctypes.c_int, [vp, vp, vp, vp, i32]),
        "smrt_set_populations": (ctypes.c_int, [vp, vp, i32]),
        "smrt_get_populations": (ctypes.c_int, [vp, vp, i32]),
        "smrt_step": (ctypes.c_int, [vp, i64]),
        "smrt_moments": (ctypes.c_int, [vp, vp, vp, vp, i32]),
        "smrt_residual": (ctypes.c_int, [vp, dp]),
        "smrt_mass": (ctypes.c_int, [vp, dp]),
        "smrt_mass_noalloc": (ctypes.c_int, [vp, vp]),
        "smrt_steps_done": (i64, [vp]),
        "smrt_tau": (ctypes.c_double, [vp]),
        "smrt_set_launch": (ctypes.c_int, [vp, i32, i32, i32]),
        "smrt_set_steps_per_launch": (ctypes.c_int, [vp, i32, i32, i32]),
        "smrt_get_steps_per_launch": (i32, [vp]),
        "smrt_set_tile_order": (ctypes.c_int, [vp, i32]),
        "smrt_synchronize": (ctypes.c_int, [vp]),
        "smrt_destroy": (None, [vp]),
        "smrt_last_error": (ctypes.c_char_p, []),
        "smrt_copy_kernel": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "smrt_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(BatchParams)]),
        "smrt_batch_create": (ctypes.c_int, [ctypes.POINTER(BatchParams), vp, ctypes.c_size_t,
                                             ctypes.POINTER(vp)]),
        "smrt_batch_step": (ctypes.c_int, [vp, i64]),
        "smrt_batch_run": (ctypes.c_int, [vp, ctypes.c_double, i64, i64, ctypes.POINTER(i64),
                                          ctypes.POINTER(i32), dp]),
        "smrt_batch_autotune": (ctypes.c_int, [vp, i32, ctypes.POINTER(i32)]),
        "smrt_batch_moments": (ctypes.c_int, [vp, i32, vp, vp, vp, i32]),
        "smrt_batch_init_fields": (ctypes.c_int, [vp, i32, vp, vp, vp, i32]),
        "smrt_batch_steps_done": (i64, [vp]),
        "smrt_batch_running": (i32, [vp]),
        "smrt_batch_steps_per_launch": (i32, [vp]),
        "smrt_batch_set_launch": (ctypes.c_int, [vp, i32, i32, i32]),
        "smrt_batch_destroy": (None, [vp]),
        "smrt_mlp_param_count": (ctypes.c_size_t, [ctypes.POINTER(MlpParams)]),
        "smrt_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(MlpParams)]),
        "smrt_mlp_create": (ctypes.c_int, [ctypes.POINTER(MlpParams), vp, ctypes.c_size_t,
                                           ctypes.POINTER(vp)]),
        "smrt_mlp_set_params": (ctypes.c_int, [vp, vp, vp]),
        "smrt_mlp_get_params": (ctypes.c_int, [vp, vp]),
        "smrt_mlp_forward": (ctypes.c_int, [vp, vp, i32, vp]),
        "smrt_mlp_gradient": (ctypes.c_int, [vp, vp, vp, i32, vp, dp]),
        "smrt_mlp_train_step": (ctypes.c_int, [vp, vp, vp, i32, ctypes.c_float, dp]),
        "smrt_mlp_destroy": (None, [vp]),
        "smrt_mlp_set_fused_forward": (ctypes.c_int, [vp, i32]),
        "smrt_mlp_uses_fused_forward": (ctypes.c_int, [vp]),
        "smrt_gemm_bf16": (ctypes.c_int, [vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        msg = load().smrt_last_error().decode(errors="replace")
        raise (UnstableError if rc == EUNSTABLE else SmrtError)(rc, msg)
    return rc


def make_params(nx, ny, scheme="smrt", boundary="cavity", storage="f32", tau=None, re=None,
                u_lid=0.0, tau_s=1.0, stream=0):
    p = Params()
    p.nx, p.ny = int(nx), int(ny)
    p.scheme, p.boundary, p.storage = SCHEMES[scheme], BOUNDARIES[boundary], STORAGE[storage]
    p.tau = float(tau) if tau is not None else 0.0
    p.re = float(re) if re is not None else 0.0
    p.u_lid, p.tau_s = float(u_lid), float(tau_s)
    p.stream = int(stream) or None
    return p


def workspace_bytes(**kw):
    """Workspace bytes for the given parameters (0 if they are invalid)."""
    return int(load().smrt_workspace_bytes(ctypes.byref(make_params(**kw))))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@contextlib.contextmanager
def _caller_order(own, device):
    """For a call that reads or writes caller tensors on an object's own
    stream: the object's stream first waits for the caller's current stream
    (inputs written, memory free), and afterwards the caller's stream waits
    for the object's (results visible to the caller's next operations).  No
    effect when the two are the same stream."""
    cur = torch.cuda.current_stream(device)
    if cur.cuda_stream == own.cuda_stream:
        yield
        return
    own.wait_stream(cur)
    yield
    cur.wait_stream(own)


class Solver:
    """One lattice on one GPU.

    Parameters mirror ``smrt_params``: ``scheme`` in {'srt', 'smrt', 'trt'},
    ``boundary`` in {'cavity', 'periodic', 'cavity_eqlid'} ('cavity_eqlid': the
    cavity with the equilibrium lid on its top row, one step per launch),
    ``storage`` in {'f64', 'f32',
    'f16', 'bf16', 'f32x', 'm64', 'm16', 'mbf16'} ('f32x': FP32 storage with
    FP64 collision arithmetic; 'm*': SmrtLBM moment storage, binary32 (FP64)
    density and momentum with 16-bit (FP64) non-equilibrium amplitudes); give ``tau`` directly or ``re`` (then tau = 3 U N / Re + 1/2).
    The workspace is a torch uint8 tensor on ``device``; work goes to the
    current torch stream of that device at construction time.  Calls that take
    or return tensors are ordered against the caller's current stream, so the
    two streams may differ (e.g. a solver created on a side stream for graph
    capture).  The library launches on the current HIP device: with several
    devices, create and call a solver with its own device current
    (``torch.cuda.device``).
    """

    def __init__(self, nx, ny, scheme="smrt", boundary="cavity", storage="f32", tau=None,
                 re=None, u_lid=0.0, tau_s=1.0, device="cuda:0"):
        lib = load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a GPU device, got %s" % self.device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        self.nx, self.ny = int(nx), int(ny)
        self.scheme, self.boundary, self.storage = scheme, boundary, storage
        self._params = make_params(nx, ny, scheme, boundary, storage, tau, re, u_lid, tau_s,
                                   self.stream.cuda_stream)
        nbytes = lib.smrt_workspace_bytes(ctypes.byref(self._params))
        if nbytes == 0:
            _check(lib.smrt_create(ctypes.byref(self._params), None, 0,
                                   ctypes.byref(ctypes.c_void_p())))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check(lib.smrt_create(ctypes.byref(self._params), _ptr(self.workspace), nbytes,
                               ctypes.byref(ctx)))
        self._ctx = ctx

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            load().smrt_synchronize(self._ctx)
            load().smrt_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state --------------------------------------------------------------
    @property
    def tau(self):
        return float(load().smrt_tau(self._ctx))

    @property
    def steps_done(self):
        return int(load().smrt_steps_done(self._ctx))

    @property
    def steps_per_launch(self):
        return int(load().smrt_get_steps_per_launch(self._ctx))

    def _io(self, t, shape):
        if t is None:
            return None
        if t.device != self.device or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError("expected a contiguous %s tensor of shape %s on %s" %
                             (t.dtype, shape, self.device))
        if t.dtype not in _IO_DTYPES:
            raise ValueError("fields must be float32 or float64")
        return t

    def init_fields(self, rho=None, ux=None, uy=None):
        """f = f^eq(rho, u); tensors (ny, nx) float32/float64 on the device."""
        given = [t for t in (rho, ux, uy) if t is not None]
        dtype = given[0].dtype if given else torch.float32
        if any(t.dtype != dtype for t in given):
            raise ValueError("rho, ux, uy must share one dtype")
        s = (self.ny, self.nx)
        with _caller_order(self.stream, self.device):
            _check(load().smrt_init_fields(self._ctx, _ptr(self._io(rho, s)), _ptr(self._io(ux, s)),
                                           _ptr(self._io(uy, s)), _IO_DTYPES[dtype]))

    def set_populations(self, f):
        """Post-collision populations f, tensor (9, ny, nx) float32/float64."""
        f = self._io(f, (9, self.ny, self.nx))
        with _caller_order(self.stream, self.device):
            _check(load().smrt_set_populations(self._ctx, _ptr(f), _IO_DTYPES[f.dtype]))

    def populations(self, dtype=torch.float64):
        out = torch.empty((9, self.ny, self.nx), dtype=dtype, device=self.device)
        with _caller_order(self.stream, self.device):
            _check(load().smrt_get_populations(self._ctx, _ptr(out), _IO_DTYPES[dtype]))
        return out

    def step(self, n=1):
        _check(load().smrt_step(self._ctx, int(n)))

    def moments(self, dtype=torch.float64):
        """(rho, ux, uy) as new (ny, nx) tensors."""
        s = (self.ny, self.nx)
        rho, ux, uy = (torch.empty(s, dtype=dtype, device=self.device) for _ in range(3))
        return self.moments_into(rho, ux, uy)

    def moments_into(self, rho=None, ux=None, uy=None):
        """Writes (rho, ux, uy) into caller tensors (any may be None); returns them."""
        s = (self.ny, self.nx)
        given = [t for t in (rho, ux, uy) if t is not None]
        if not given:
            return rho, ux, uy
        dtype = given[0].dtype
        if any(t.dtype != dtype for t in given):
            raise ValueError("rho, ux, uy must share one dtype")
        with _caller_order(self.stream, self.device):
            _check(load().smrt_moments(self._ctx, _ptr(self._io(rho, s)), _ptr(self._io(ux, s)),
                                       _ptr(self._io(uy, s)), _IO_DTYPES[dtype]))
        return rho, ux, uy

    def residual(self):
        out = ctypes.c_double()
        _check(load().smrt_residual(self._ctx, ctypes.byref(out)))
        return out.value

    def mass(self):
        out = ctypes.c_double()
        _check(load().smrt_mass(self._ctx, ctypes.byref(out)))
        return out.value

    def mass_noalloc(self, out):
        """Enqueues (sum rho, non-finite node count) into a float64 device
        tensor of 2 elements, without allocation or synchronization."""
        if out.device != self.device or out.dtype != torch.float64 or out.numel() < 2 or not out.is_contiguous():
            raise ValueError("expected a contiguous float64 tensor of 2 elements on %s" % self.device)
        with _caller_order(self.stream, self.device):
            _check(load().smrt_mass_noalloc(self._ctx, _ptr(out)))
        return out

    def run_to_steady(self, tol=1e-7, window=1000, max_steps=10_000_000, callback=None):
        """Steps in windows of `window` until the windowed residual drops below
        `tol` or `max_steps` is reached.  Returns (steps, residuals, converged);
        raises UnstableError if the field blows up."""
        residuals = []
        steps = 0
        while steps < max_steps:
            n = min(window, max_steps - steps)
            self.step(n)
            steps += n
            r = self.residual()
            residuals.append(r)
            if callback is not None:
                callback(steps, r)
            if r < tol:
                return steps, residuals, True
        return steps, residuals, False

    def convert(self, storage):
        """A new solver with the same lattice and parameters in another storage
        type, holding this solver's current populations (rounded to the new
        type).  Its step counter and residual snapshot start afresh."""
        p = self._params
        other = Solver(self.nx, self.ny, scheme=self.scheme, boundary=self.boundary,
                       storage=storage, tau=self.tau, u_lid=p.u_lid, tau_s=p.tau_s,
                       device=self.device)
        # FP64 transfer: w + d and back is exact for every storage type's d
        f = self.populations(torch.float64)
        other.set_populations(f)
        del f
        return other

    def set_launch(self, bx, by, rows=1):
        _check(load().smrt_set_launch(self._ctx, int(bx), int(by), int(rows)))

    def set_steps_per_launch(self, steps, tile_rows=0, tile_cols=0):
        """1, or 2 .. 5 for the LDS-blocked kernels (FP64 storage: 2 .. 4);
        two-step tiles 64 x {4, 8, 16, 32} or 128 x {4, 8} (0 = 64 x 8),
        three- and four-step tiles 64 x {8, 16, 24, 26} (0 = 64 x 16),
        five-step tiles 64 x {16, 22} (0 = 64 x 16); FP64 storage 64 x 8
        (also 64 x 4 for two steps, 64 x 10 for four)."""
        _check(load().smrt_set_steps_per_launch(self._ctx, int(steps), int(tile_cols), int(tile_rows)))

    def set_tile_order(self, panel_cols):
        """Tile order of the multi-step kernels: 0 = row-major, P > 0 = XCD
        panels of P tile columns (same results, different L2 reuse)."""
        _check(load().smrt_set_tile_order(self._ctx, int(panel_cols)))

    def synchronize(self):
        _check(load().smrt_synchronize(self._ctx))


def copy_kernel(src, dst, nbytes=None, stream=None):
    """Launches the library's reference streaming copy (src -> dst, device tensors)."""
    nbytes = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    s = (stream or torch.cuda.current_stream(src.device)).cuda_stream
    _check(load().smrt_copy_kernel(_ptr(src), _ptr(dst), nbytes, ctypes.c_void_p(s or None)))


class Batch:
    """Many lid-driven cavities advanced together on one GPU (smrt_batch_*).

    ``nx``, ``ny``: side lengths per cavity; ``tau`` or ``re`` per cavity
    (sequence or None); one lid speed for all.  Workspace: a torch uint8
    tensor; work goes to the current torch stream at construction time.
    """

    def __init__(self, nx, ny, scheme="smrt", storage="f32", tau=None, re=None, u_lid=0.1,
                 tau_s=1.0, device="cuda:0"):
        lib = load()
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        self.nx = [int(v) for v in nx]
        self.ny = [int(v) for v in ny]
        self.count = len(self.nx)
        if len(self.ny) != self.count:
            raise ValueError("nx and ny must have the same length")
        c = self.count
        self._nx = (ctypes.c_int32 * c)(*self.nx)
        self._ny = (ctypes.c_int32 * c)(*self.ny)
        self._tau = (ctypes.c_double * c)(*[float(t) for t in tau]) if tau is not None else None
        self._re = (ctypes.c_double * c)(*[float(r) for r in re]) if re is not None else None
        p = BatchParams()
        p.count, p.scheme, p.storage = c, SCHEMES[scheme], STORAGE[storage]
        p.nx = ctypes.cast(self._nx, ctypes.POINTER(ctypes.c_int32))
        p.ny = ctypes.cast(self._ny, ctypes.POINTER(ctypes.c_int32))
        p.tau = ctypes.cast(self._tau, ctypes.POINTER(ctypes.c_double)) if self._tau else None
        p.re = ctypes.cast(self._re, ctypes.POINTER(ctypes.c_double)) if self._re else None
        p.u_lid, p.tau_s = float(u_lid), float(tau_s)
        p.stream = self.stream.cuda_stream or None
        self._params = p
        self.scheme, self.storage = scheme, storage
        nbytes = lib.smrt_batch_workspace_bytes(ctypes.byref(p))
        if nbytes == 0:
            _check(lib.smrt_batch_create(ctypes.byref(p), None, 0, ctypes.byref(ctypes.c_void_p())))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check(lib.smrt_batch_create(ctypes.byref(p), _ptr(self.workspace), nbytes, ctypes.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            load().smrt_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def steps_done(self):
        return int(load().smrt_batch_steps_done(self._ctx))

    @property
    def running(self):
        return int(load().smrt_batch_running(self._ctx))

    def step(self, n):
        _check(load().smrt_batch_step(self._ctx, int(n)))

    def run(self, tol=1e-7, window=1000, max_steps=500_000):
        """Runs until every cavity is steady/unstable or max_steps more steps.
        Returns (steps, status, residual) lists, one entry per cavity."""
        c = self.count
        steps = (ctypes.c_int64 * c)()
        status = (ctypes.c_int32 * c)()
        res = (ctypes.c_double * c)()
        _check(load().smrt_batch_run(self._ctx, float(tol), int(window), int(max_steps), steps,
                                     status, res))
        return list(steps), list(status), list(res)

    @property
    def steps_per_launch(self):
        return int(load().smrt_batch_steps_per_launch(self._ctx))

    def autotune(self, steps=20):
        """Times the candidate launch shapes; returns the chosen (bx, by, grid)
        (steps_per_launch tells the chosen kernel's steps per launch)."""
        chosen = (ctypes.c_int32 * 3)()
        _check(load().smrt_batch_autotune(self._ctx, int(steps), chosen))
        return tuple(chosen)

    def set_launch(self, bx, by, steps):
        """Launch shape by hand: `steps` time steps per launch on bx x by tiles."""
        _check(load().smrt_batch_set_launch(self._ctx, int(bx), int(by), int(steps)))

    def moments(self, index, dtype=torch.float64):
        s = (self.ny[index], self.nx[index])
        rho, ux, uy = (torch.empty(s, dtype=dtype, device=self.device) for _ in range(3))
        with _caller_order(self.stream, self.device):
            _check(load().smrt_batch_moments(self._ctx, int(index), _ptr(rho), _ptr(ux), _ptr(uy),
                                             _IO_DTYPES[dtype]))
        return rho, ux, uy

    def init_fields(self, index, rho=None, ux=None, uy=None):
        given = [t for t in (rho, ux, uy) if t is not None]
        dtype = given[0].dtype if given else torch.float32
        s = (self.ny[index], self.nx[index])
        for t in given:
            if t.dtype != dtype or tuple(t.shape) != s or not t.is_contiguous() or t.device != self.device:
                raise ValueError("fields must be contiguous %s tensors of shape %s" % (dtype, s))
        with _caller_order(self.stream, self.device):
            _check(load().smrt_batch_init_fields(self._ctx, int(index), _ptr(rho), _ptr(ux), _ptr(uy),
                                                 _IO_DTYPES[dtype]))


class MLP:
    """The warm-start coordinate network (smrt_mlp_*): points (x, y, s) ->
    outputs, bf16 matrix-core arithmetic with FP32 accumulation.  All tensors
    are float32 on the device; row counts must be multiples of 64."""

    def __init__(self, fourier=16, width=128, layers=5, outputs=3, max_batch=65536,
                 device="cuda:0"):
        lib = load()
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        p = MlpParams()
        p.inputs, p.fourier, p.width, p.layers, p.outputs = 3, fourier, width, layers, outputs
        p.max_batch = max_batch
        p.stream = self.stream.cuda_stream or None
        self._params = p
        self.fourier, self.width, self.layers, self.outputs = fourier, width, layers, outputs
        self.max_batch = max_batch
        self.param_count = int(lib.smrt_mlp_param_count(ctypes.byref(p)))
        nbytes = lib.smrt_mlp_workspace_bytes(ctypes.byref(p))
        if nbytes == 0:
            _check(lib.smrt_mlp_create(ctypes.byref(p), None, 0, ctypes.byref(ctypes.c_void_p())))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check(lib.smrt_mlp_create(ctypes.byref(p), _ptr(self.workspace), nbytes, ctypes.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            load().smrt_mlp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _f32(self, t, shape=None):
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous():
            raise ValueError("expected a contiguous float32 tensor on %s" % self.device)
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))
        return t

    def set_params(self, params, fourier_matrix):
        self._f32(params, (self.param_count,))
        self._f32(fourier_matrix, (self.fourier, 3))
        with _caller_order(self.stream, self.device):
            _check(load().smrt_mlp_set_params(self._ctx, _ptr(params), _ptr(fourier_matrix)))

    def get_params(self):
        out = torch.empty(self.param_count, dtype=torch.float32, device=self.device)
        with _caller_order(self.stream, self.device):
            _check(load().smrt_mlp_get_params(self._ctx, _ptr(out)))
        return out

    @property
    def fused_forward(self):
        """True when the forward pass runs as one launch (smrt_mlp_set_fused_forward)."""
        rc = load().smrt_mlp_uses_fused_forward(self._ctx)
        _check(min(rc, 0))
        return rc == 1

    @fused_forward.setter
    def fused_forward(self, enable):
        _check(load().smrt_mlp_set_fused_forward(self._ctx, int(bool(enable))))

    def forward(self, points, out=None):
        n = points.shape[0]
        self._f32(points, (n, 3))
        if out is None:
            out = torch.empty((n, self.outputs), dtype=torch.float32, device=self.device)
        with _caller_order(self.stream, self.device):
            _check(load().smrt_mlp_forward(self._ctx, _ptr(points), int(n),
                                           _ptr(self._f32(out, (n, self.outputs)))))
        return out

    def gradient(self, points, target):
        n = points.shape[0]
        grad = torch.empty(self.param_count, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        with _caller_order(self.stream, self.device):
            _check(load().smrt_mlp_gradient(self._ctx, _ptr(self._f32(points, (n, 3))),
                                            _ptr(self._f32(target, (n, self.outputs))), int(n), _ptr(grad),
                                            ctypes.byref(loss)))
        return loss.value, grad

    def train_step(self, points, target, lr, want_loss=False):
        n = points.shape[0]
        loss = ctypes.c_double() if want_loss else None
        with _caller_order(self.stream, self.device):
            _check(load().smrt_mlp_train_step(self._ctx, _ptr(self._f32(points, (n, 3))),
                                              _ptr(self._f32(target, (n, self.outputs))), int(n),
                                              float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


def gemm_bf16(a_bits, b_bits, m, n, k, lda, ldb, ldc, trans_a=False, trans_b=False, splits=1,
              out=None):
    """C (splits x m x ldc, float32) from bf16 bit patterns held in int16 tensors."""
    if out is None:
        out = torch.empty((splits, m, ldc), dtype=torch.float32, device=a_bits.device)
    s = torch.cuda.current_stream(a_bits.device).cuda_stream
    _check(load().smrt_gemm_bf16(_ptr(a_bits), _ptr(b_bits), _ptr(out), int(m), int(n), int(k),
                                 int(lda), int(ldb), int(ldc), int(bool(trans_a)), int(bool(trans_b)),
                                 int(splits), ctypes.c_void_p(s or None)))
    return out
