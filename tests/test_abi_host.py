"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol that include/smrt.h declares, lays out smrt_params as the header
says, and rejects invalid parameters before touching the device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

LIB = os.path.join(ROOT, "paper_2409_01076_amd", "libsmrt.so")
HEADER = os.path.join(ROOT, "include", "smrt.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsmrt.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smrt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2409_01076_amd import smrt
    lib = smrt.load()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(smrt.EXPORTED) == names


def test_params_layout_matches_header():
    from paper_2409_01076_amd import smrt
    P = smrt.Params
    assert ctypes.sizeof(P) == 96
    assert P.tau.offset == 24 and P.stream.offset == 56 and P.reserved.offset == 64


def _create(**kw):
    from paper_2409_01076_amd import smrt
    lib = smrt.load()
    p = smrt.make_params(**kw)
    ctx = ctypes.c_void_p(1234)
    rc = lib.smrt_create(ctypes.byref(p), None, 0, ctypes.byref(ctx))
    return rc, ctx.value, lib.smrt_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(nx=2, ny=64, tau=0.7), "nx and ny"),
    (dict(nx=64, ny=64, tau=0.5), "exceed 1/2"),
    (dict(nx=64, ny=64, re=100.0, u_lid=0.0), "non-zero lid"),
    (dict(nx=64, ny=64, re=-1.0, u_lid=0.1), "Reynolds"),
    (dict(nx=64, ny=64, tau=0.7, u_lid=0.6), "sound speed"),
    (dict(nx=64, ny=64, scheme="trt", tau=0.7, tau_s=0.4), "tau_s"),
    # Re so high that tau rounds to 1/2
    (dict(nx=64, ny=64, re=1e20, u_lid=0.1), "exceed 1/2"),
])
def test_create_rejects_invalid_parameters(kw, needle):
    from paper_2409_01076_amd import smrt
    rc, ctx, msg = _create(**kw)
    assert rc == smrt.EINVAL and ctx is None and needle in msg


def test_workspace_bytes_host_only():
    from paper_2409_01076_amd import smrt
    nb32 = smrt.workspace_bytes(nx=4096, ny=4096, storage="f32", tau=0.6)
    nb64 = smrt.workspace_bytes(nx=4096, ny=4096, storage="f64", tau=0.6)
    nb16 = smrt.workspace_bytes(nx=4096, ny=4096, storage="f16", tau=0.6)
    cells = 4096 * 4096
    # two population buffers dominate: 2 x 9 x 4 bytes per node, plus the FP64 snapshot
    assert 72 * cells <= nb32 < 72 * cells + 16 * cells + (1 << 22)
    assert 144 * cells <= nb64 and 36 * cells <= nb16 < nb32
    assert smrt.workspace_bytes(nx=4096, ny=4096, storage="f32", tau=0.4) == 0


@pytest.mark.parametrize("storage,widest", [("f64", 262_144), ("f32", 524_288), ("f16", 1_048_576),
                                             ("bf16", 1_048_576)])
def test_row_width_limit(storage, widest):
    # a lattice row holds at most 2 MiB of stored values (32-bit offsets inside a tile)
    from paper_2409_01076_amd import smrt
    assert smrt.workspace_bytes(nx=widest, ny=3, storage=storage, tau=0.6) > 0
    assert smrt.workspace_bytes(nx=widest + 1, ny=3, storage=storage, tau=0.6) == 0
    rc, ctx, msg = _create(nx=widest + 1, ny=3, storage=storage, tau=0.6)
    assert rc == smrt.EINVAL and ctx is None and "bytes of stored values" in msg
    # nodes are capped at 2^34 whatever the width
    assert smrt.workspace_bytes(nx=4096, ny=(1 << 22) + 1, storage=storage, tau=0.6) == 0


def _batch_bytes(nx, ny, storage="f32"):
    from paper_2409_01076_amd import smrt
    c = len(nx)
    p = smrt.BatchParams()
    p.count, p.scheme, p.storage = c, smrt.SCHEMES["smrt"], smrt.STORAGE[storage]
    anx, any_ = (ctypes.c_int32 * c)(*nx), (ctypes.c_int32 * c)(*ny)
    tau = (ctypes.c_double * c)(*([0.6] * c))
    p.nx = ctypes.cast(anx, ctypes.POINTER(ctypes.c_int32))
    p.ny = ctypes.cast(any_, ctypes.POINTER(ctypes.c_int32))
    p.tau = ctypes.cast(tau, ctypes.POINTER(ctypes.c_double))
    p.u_lid = 0.1
    lib = smrt.load()
    n = lib.smrt_batch_workspace_bytes(ctypes.byref(p))
    return n, lib.smrt_last_error().decode()


def test_batch_row_width_and_size_limits():
    n, _ = _batch_bytes([64, 524_288], [64, 3])
    assert n > 0
    n, msg = _batch_bytes([64, 524_289], [64, 3])
    assert n == 0 and "cavity 1" in msg and "bytes of stored values" in msg
    n, msg = _batch_bytes([4096], [(1 << 22) + 1])
    assert n == 0 and "too large" in msg


def test_null_context_calls_fail_cleanly():
    from paper_2409_01076_amd import smrt
    lib = smrt.load()
    lib.smrt_destroy(None)
    assert lib.smrt_step(None, 1) == smrt.EINVAL
    assert lib.smrt_steps_done(None) == -1
    out = ctypes.c_double()
    assert lib.smrt_residual(None, ctypes.byref(out)) == smrt.EINVAL
    assert lib.smrt_set_launch(None, 64, 4, 1) == smrt.EINVAL
    assert lib.smrt_set_tile_order(None, 8) == smrt.EINVAL
    assert lib.smrt_copy_kernel(None, None, 16, None) == smrt.EINVAL
    assert "NULL" in lib.smrt_last_error().decode()


def test_header_cites_the_paper_for_each_scheme():
    text = open(HEADER).read()
    for eq in ("lb.srt", "SmrtLBM-1", "SmrtLBM-lb.1.5", "feq-full", "fea-0", "relation-chapman-viscosity"):
        assert eq in text
