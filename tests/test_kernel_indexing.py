"""CPU replay of the stream-collide kernels' index arithmetic (no GPU needed).

The kernels in paper_2409_01076_amd/csrc/lbm_kernels.hpp trust their grid:
an address outside its buffer faults the GPU, and an LDS read of a frame cell
that the previous step did not write gives wrong values without any error.
This file walks every workgroup of every launch shape the library offers, the
way the kernels index, on lattices from 3 x 3 up with ragged tiles, and checks:

* every global load and store address lies in its buffer, with the workspace
  layout of smrt_api.hip (rows padded to 256 bytes, direction planes rounded
  to 64 KiB plus a 4 KiB pad) and the kernels' addressing: a uniform 64-bit
  base per direction plus a 32-bit unsigned per-lane byte offset, so a
  negative offset shows up as a wrapped one;
* every LDS read of a multi-step launch lies in the frame and sees the value
  written by the step before (the frame holds the tile plus S - 1 rings; the
  step on ring r sits at offset S - 1 - r);
* a tile that takes the check-free inner path has its widest region inside
  the lattice and off its outer ring;
* the XCD panel tile order visits every tile exactly once.

Launch shapes and thread counts mirror smrt_set_steps_per_launch and
multi_threads in smrt_api.hip, and the batch shapes and per-cavity layout of
smrt_batch.hip.
"""
import itertools

import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
U32 = (1 << 32) - 1


def layout(nx, ny, e, batch=False):
    """(pitch, plane) in elements; a batch packs each cavity's planes tighter."""
    per_row = 256 // e
    pitch = -(-nx // per_row) * per_row
    if batch:
        return pitch, -(-pitch * ny // per_row) * per_row
    plane_bytes = -(-pitch * ny * e // 65536) * 65536 + 4096
    return pitch, plane_bytes // e


def threads(steps, tx, ty):
    if (steps >= 4 and tx * ty >= 512) or (steps == 2 and tx * ty >= 2048):
        return 768
    return 512 if tx * ty >= 1024 else 256


# (steps, tile_cols, tile_rows) offered per storage class
TILES_32 = ([(2, 64, r) for r in (4, 8, 16, 32)] + [(2, 128, 4), (2, 128, 8)] +
            [(s, 64, r) for s in (3, 4) for r in (8, 16, 24, 26)] + [(5, 64, 16), (5, 64, 22)])
TILES_64 = [(2, 64, 4), (2, 64, 8), (3, 64, 8), (4, 64, 8), (4, 64, 10)]


class Buffer:
    def __init__(self, nx, ny, e, batch=False):
        self.nx, self.ny, self.e = nx, ny, e
        self.pitch, self.plane = layout(nx, ny, e, batch)
        self.limit = 9 * self.plane * e

    def check(self, addr, what):
        addr = np.asarray(addr)
        if addr.size:
            assert addr.min() >= 0 and addr.max() < self.limit, (
                "%s address out of bounds on %dx%d (e=%d): [%d, %d] of %d"
                % (what, self.nx, self.ny, self.e, addr.min(), addr.max(), self.limit))

    def pull_interior(self, row0, x, y):
        """Interior pull: plane base at row row0 (shifted by -e_a) + offset."""
        off = (((y - 1 - row0) * self.pitch + (x - 1)) * self.e) & U32
        bases = (np.arange(9) * self.plane + (row0 + 1 - EY) * self.pitch + (1 - EX)) * self.e
        return (bases[:, None] + off[None, :]).ravel()

    def pull_edge(self, periodic, x, y):
        sx = x[None, :] - EX[:, None]
        sy = y[None, :] - EY[:, None]
        a = np.arange(9)[:, None]
        if periodic:
            sx = np.where(sx < 0, sx + self.nx, np.where(sx >= self.nx, sx - self.nx, sx))
            sy = np.where(sy < 0, sy + self.ny, np.where(sy >= self.ny, sy - self.ny, sy))
            return ((a * self.plane + sy * self.pitch + sx) * self.e).ravel()
        inside = (sx >= 0) & (sx < self.nx) & (sy >= 0) & (sy < self.ny)
        own = OPP[:, None] * self.plane + y[None, :] * self.pitch + x[None, :]
        return (np.where(inside, a * self.plane + sy * self.pitch + sx, own) * self.e).ravel()

    def store(self, row0, x, y):
        off = (((y - row0) * self.pitch + x) * self.e) & U32
        bases = (np.arange(9) * self.plane + row0 * self.pitch) * self.e
        return (bases[:, None] + off[None, :]).ravel()

    def pull(self, periodic, row0, x, y, wrapped=None):
        edge = (x == 0) | (x == self.nx - 1) | (y == 0) | (y == self.ny - 1)
        if wrapped is not None:
            edge |= wrapped
        self.check(self.pull_edge(periodic, x[edge], y[edge]), "edge pull")
        self.check(self.pull_interior(row0, x[~edge], y[~edge]), "interior pull")


def one_step(nx, ny, e, periodic, bx, by, rows, batch=False):
    """stream_collide: block (bx, by), each thread `rows` nodes by rows apart
    (batch_stream_collide: rows = 1, per cavity)."""
    buf = Buffer(nx, ny, e, batch)
    tiles_x, tiles_y = -(-nx // bx), -(-ny // (by * rows))
    tix, tiy = (a.ravel() for a in np.meshgrid(np.arange(bx), np.arange(by)))
    for ty, tx in itertools.product(range(tiles_y), range(tiles_x)):
        ytile = ty * by * rows
        x = tx * bx + tix
        for r in range(rows):
            y = ytile + tiy + r * by
            m = (x < nx) & (y < ny)
            buf.pull(periodic, max(ytile - 1, 0), x[m], y[m])
            buf.check(buf.store(ytile, x[m], y[m]), "store")


def multi_step(nx, ny, e, periodic, S, TX, TY, batch=False):
    """stream_collide_xS (batch_stream_collide_xS: per cavity) on every
    TX x TY tile: HBM phase, LDS frame, store."""
    buf = Buffer(nx, ny, e, batch)
    NT = threads(S, TX, TY)
    R = S - 1
    FX, FY = TX + 2 * R, TY + 2 * R
    i = np.arange(-(-FX * FY // NT) * NT)
    lx, ly = i % FX, i // FX
    for ty, tx in itertools.product(range(-(-ny // TY)), range(-(-nx // TX))):
        X0, Y0 = tx * TX, ty * TY
        inner = X0 - R >= 1 and X0 + TX + R <= nx - 1 and Y0 - R >= 1 and Y0 + TY + R <= ny - 1
        xu, yu = X0 - R + lx, Y0 - R + ly
        if inner:
            live = i < FX * FY
            x, y = xu[live], yu[live]
            assert ((x >= 1) & (x <= nx - 2) & (y >= 1) & (y <= ny - 2)).all(), "inner tile touches the edge"
            buf.check(buf.pull_interior(Y0 - R - 1, x, y), "inner pull")
        else:
            if periodic:
                live = (i < FX * FY) & (xu <= nx + R - 1) & (yu <= ny + R - 1)
                x = np.where(xu < 0, xu + nx, np.where(xu >= nx, xu - nx, xu))
                y = np.where(yu < 0, yu + ny, np.where(yu >= ny, yu - ny, yu))
            else:
                live = (i < FX * FY) & (xu >= 0) & (xu < nx) & (yu >= 0) & (yu < ny)
                x, y = xu, yu
            wrapped = (x != xu) | (y != yu)
            buf.pull(periodic, Y0 - R - 1 if Y0 > R else 0, x[live], y[live], wrapped[live])
        # LDS frame: version of the step each cell holds (-1: never written)
        ver = np.full((FY, FX), -1)
        ver[ly[live], lx[live]] = 1
        for step, r in enumerate(range(R - 1, -1, -1), start=2):
            BX, BY, OFF = TX + 2 * r, TY + 2 * r, R - r
            j = np.arange(-(-BX * BY // NT) * NT) if r > 0 else np.arange(TX * TY)
            jx, jy = j % BX, j // BX
            mx, my = X0 - r + jx, Y0 - r + jy
            if inner:
                ok = j < BX * BY
            elif periodic:
                ok = (j < BX * BY) & (mx <= nx + r - 1) & (my <= ny + r - 1)
            else:
                ok = (j < BX * BY) & (mx >= 0) & (mx < nx) & (my >= 0) & (my < ny)
            if r == 0:  # last step: the tile's nodes inside the lattice
                ok = (mx < nx) & (my < ny)
            fx, fy, mx, my = jx[ok] + OFF, jy[ok] + OFF, mx[ok], my[ok]
            for a in range(9):
                sx, sy = mx - EX[a], my - EY[a]
                need = np.ones_like(sx, bool) if periodic or inner else (
                    (sx >= 0) & (sx < nx) & (sy >= 0) & (sy < ny))
                ax, ay = fx[need] - EX[a], fy[need] - EY[a]
                assert ((ax >= 0) & (ax < FX) & (ay >= 0) & (ay < FY)).all(), ("frame read outside", S, tx, ty, a)
                assert (ver[ay, ax] == step - 1).all(), ("stale frame read", nx, ny, S, TX, TY, step, tx, ty, a)
                if not periodic and not inner:  # bounce-back reads the node's own cell
                    assert (ver[fy[~need], fx[~need]] == step - 1).all()
            if r > 0:
                ver[fy, fx] = step
            else:
                buf.check(buf.store(Y0, mx, my), "store")


SIZES_ONE = [3, 5, 7, 17, 63, 64, 65, 67, 129, 157, 300]


@pytest.mark.parametrize("e", [8, 4, 2])
@pytest.mark.parametrize("periodic", [True, False])
def test_one_step_kernel_addresses(e, periodic):
    for nx, ny in itertools.product(SIZES_ONE, SIZES_ONE):
        for bx, by, rows in ((512, 1, 1), (256, 1, 1), (128, 2, 1), (64, 4, 1), (256, 1, 2), (64, 2, 8)):
            one_step(nx, ny, e, periodic, bx, by, rows)


def multi_cases(tiles):
    for S, TX, TY in tiles:
        R = S - 1
        for nx, ny in [(TX + 2 * R, TY + 2 * R), (TX + 2 * R + 3, TY + 2 * R + 1), (200, 97), (131, 131),
                       (257, 300), (300, 157), (64, 64), (5, 7), (3, 3)]:
            for periodic in (True, False):
                # a periodic ring wraps once: the lattice must hold the tile and its rings
                if periodic and (nx < TX + 2 * R or ny < TY + 2 * R):
                    continue
                yield S, TX, TY, nx, ny, periodic


@pytest.mark.parametrize("S,TX,TY", TILES_32)
def test_multi_step_kernels_fp32_and_16bit(S, TX, TY):
    for S_, TX_, TY_, nx, ny, periodic in multi_cases([(S, TX, TY)]):
        for e in (4, 2):
            multi_step(nx, ny, e, periodic, S_, TX_, TY_)


@pytest.mark.parametrize("S,TX,TY", TILES_64)
def test_multi_step_kernels_fp64(S, TX, TY):
    for S_, TX_, TY_, nx, ny, periodic in multi_cases([(S, TX, TY)]):
        multi_step(nx, ny, 8, periodic, S_, TX_, TY_)


# batch launch shapes (smrt_batch.hip): one-step blocks, multi-step tiles (no FP64)
BATCH_BLOCKS = [(64, 4), (128, 2), (256, 1), (32, 8), (64, 8), (128, 4), (256, 2), (512, 1),
                (64, 16), (64, 22)]   # one-step remainders on multi-step tables (64 x 22: two row passes)
BATCH_TILES = [(2, 64, 4), (2, 64, 8), (2, 64, 16), (3, 64, 8), (3, 64, 16), (4, 64, 8), (4, 64, 16), (5, 64, 16),
               (2, 64, 22), (3, 64, 22), (4, 64, 22), (5, 64, 22)]
BATCH_SIZES = [3, 17, 64, 65, 100, 157, 300]


@pytest.mark.parametrize("e", [8, 4, 2])
def test_batch_kernels_stay_in_their_cavity(e):
    # an address past a cavity's own planes lands in the next cavity: no
    # fault, silent corruption, so each cavity is checked against its region
    for nx, ny in itertools.product(BATCH_SIZES, BATCH_SIZES):
        for bx, by in BATCH_BLOCKS:
            one_step(nx, ny, e, False, bx, by, 1, batch=True)
        if e == 8:
            continue
        for S, TX, TY in BATCH_TILES:
            multi_step(nx, ny, e, False, S, TX, TY, batch=True)


def test_replay_catches_a_negative_row_offset():
    """The replay itself: an interior pull based one row too low wraps its
    32-bit offset and must be caught."""
    buf = Buffer(300, 157, 4)
    x, y = np.array([5]), np.array([1])
    with pytest.raises(AssertionError):
        buf.check(buf.pull_interior(1, x, y), "interior pull")  # y - 1 - row0 = -1


def xcd_contiguous(bid, n):
    xcd, local = bid % 8, bid // 8
    per, rem = n // 8, n % 8
    return np.where(xcd < rem, xcd * (per + 1) + local, rem * (per + 1) + (xcd - rem) * per + local)


def panel_tile(pos, tiles_x, tiles_y, P):
    if P <= 0:
        return pos % tiles_x, pos // tiles_x
    full, per_panel = tiles_x // P, P * tiles_y
    panel = pos // per_panel
    w = pos - panel * per_panel
    tx_full, ty_full = panel * P + w % P, w // P
    pw = max(tiles_x - full * P, 1)
    w2 = pos - full * per_panel
    return np.where(panel < full, tx_full, full * P + w2 % pw), np.where(panel < full, ty_full, w2 // pw)


@pytest.mark.parametrize("tiles_x,tiles_y", [(1, 1), (3, 5), (8, 8), (64, 187), (17, 33), (9, 1)])
@pytest.mark.parametrize("P", [0, 8, 16, 32])
def test_tile_order_visits_every_tile_once(tiles_x, tiles_y, P):
    n = tiles_x * tiles_y
    pos = xcd_contiguous(np.arange(n), n)
    assert sorted(pos.tolist()) == list(range(n))
    tx, ty = panel_tile(pos, tiles_x, tiles_y, min(P, tiles_x))
    assert ((tx >= 0) & (tx < tiles_x) & (ty >= 0) & (ty < tiles_y)).all()
    assert len(set(zip(tx.tolist(), ty.tolist()))) == n


# --- moment storage (stream_collide_mom, paper_2409_01076_amd/csrc/moment_kernels.hpp) -----

MOM_TX = 64


@pytest.mark.parametrize("grid", [8, 16, 24, 12456, 16960])
def test_batch_xcd_order_visits_every_tile_once(grid):
    """batch_multi's workgroup-to-tile map: with n tiles listed and
    c = ceil(n / 8), workgroup b takes tile (b mod 8) c + b / 8 (none when
    b / 8 >= c), for a grid that is a multiple of 8 and at least n: every
    listed tile exactly once, each XCD (b mod 8) one contiguous run, and the
    runs spread over all 8 XCDs however far the table has shrunk."""
    assert grid % 8 == 0
    b = np.arange(grid)
    for ntiles in sorted(n for n in {1, 5, 9, grid // 3, grid - 7, grid} if 1 <= n <= grid):
        c = (ntiles + 7) // 8
        t = np.where(b // 8 < c, (b % 8) * c + b // 8, ntiles)
        got = t[t < ntiles]
        assert np.array_equal(np.sort(got), np.arange(ntiles))
        per_xcd = [t[(b % 8 == x) & (t < ntiles)] for x in range(8)]
        for run in per_xcd:
            assert np.all(np.diff(run) == 1)
        assert max(len(r) for r in per_xcd) <= c
        busy = sum(len(r) > 0 for r in per_xcd)
        assert busy == min(8, -(-ntiles // c))


@pytest.mark.parametrize("mom_ty", [8, 16])
@pytest.mark.parametrize("e_moment,e_amp", [(8, 8), (4, 2)])
@pytest.mark.parametrize("boundary", ["cavity", "periodic"])
@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 70), (65, 9), (64, 8), (129, 17), (300, 157)])
def test_moment_kernel_indexing(mom_ty, e_moment, e_amp, boundary, nx, ny):
    MOM_TY = mom_ty
    """Every workgroup of the moment-storage launch: the LDS cells a node reads
    were staged by the same workgroup, with the value of the node its pull
    names (wrapped for a periodic lattice); every global access lies in its
    plane (three moment planes, then two amplitude planes of the same element
    count, as smrt_api.hip lays them out)."""
    pitch, plane = layout(nx, ny, e_moment)
    buffer_bytes = -(-(3 * plane * e_moment + 2 * plane * e_amp) // 256) * 256
    fx, fy = MOM_TX + 2, MOM_TY + 2
    tiles_x = -(-nx // MOM_TX)
    tiles = tiles_x * -(-ny // MOM_TY)
    per = boundary == "periodic"
    for tile in range(tiles):
        x0, y0 = (tile % tiles_x) * MOM_TX, (tile // tiles_x) * MOM_TY
        staged = {}
        for i in range(fx * fy):
            lx, ly = i % fx, i // fx
            x, y = x0 - 1 + lx, y0 - 1 + ly
            if per:   # the kernel's wrap: once, then a remainder if still outside
                x = x + nx if x < 0 else (x - nx if x >= nx else x)
                y = y + ny if y < 0 else (y - ny if y >= ny else y)
                x, y = (x if 0 <= x < nx else x % nx), (y if 0 <= y < ny else y % ny)
            elif not (0 <= x < nx and 0 <= y < ny):
                continue
            off = y * pitch + x
            assert 0 <= off < plane
            for k in range(3):   # moment planes
                assert 0 <= (k * plane + off) * e_moment < 3 * plane * e_moment
            for k in range(2):   # amplitude planes after them
                b = 3 * plane * e_moment + (k * plane + off) * e_amp
                assert 3 * plane * e_moment <= b and b + e_amp <= buffer_bytes
            staged[(lx, ly)] = (x, y)
        for t in range(MOM_TX * MOM_TY):
            lx, ly = t % MOM_TX + 1, t // MOM_TX + 1
            x, y = x0 + lx - 1, y0 + ly - 1
            if x >= nx or y >= ny:
                continue
            assert staged[(lx, ly)] == (x, y)
            edge = not per and (x in (0, nx - 1) or y in (0, ny - 1))
            for a in range(1, 9):
                sx, sy = x - EX[a], y - EY[a]
                if not edge or (0 <= sx < nx and 0 <= sy < ny):
                    cell = (lx - EX[a], ly - EY[a])
                    assert 0 <= cell[0] < fx and 0 <= cell[1] < fy
                    assert staged[cell] == ((sx % nx, sy % ny) if per else (sx, sy))


@pytest.mark.parametrize("nb,ng", [(256, 256), (512, 256), (256, 64), (1, 1), (7, 300), (300, 7), (1024, 1)])
def test_backward_and_grad_roles_cover_each_workgroup_once(nb, ng):
    """backward_and_grad's role spread over a grid of T = nb + ng workgroups:
    workgroup b is a gradient block when floor((b + 1) ng / T) steps up, block
    floor(b ng / T), else input-gradient workgroup b - floor(b ng / T).  Every
    index of each role is taken exactly once, and the gradient blocks are
    spread evenly (at most one more in any prefix than its share)."""
    T = nb + ng
    b = np.arange(T, dtype=np.int64)
    before = b * ng // T
    is_grad = (b + 1) * ng // T > before
    back = (b - before)[~is_grad]
    grad = before[is_grad]
    assert np.array_equal(np.sort(back), np.arange(nb))
    assert np.array_equal(np.sort(grad), np.arange(ng))
    prefix = np.cumsum(is_grad)
    share = (b + 1) * ng / T
    assert np.all(np.abs(prefix - share) < 1.0)
