"""The pipelined schedule's plan image, on the CPU (jacobi_pipelined_plan
only writes host memory): every (pass, block) appears once, and every block
an item waits on comes earlier in the item order -- the condition that keeps
relaxed-mode waits from deadlocking, since persistent workgroups take items
in order and every earlier item is held by a running workgroup.  The waits
are those of the batched kernel: the 27 neighbours of the previous pass, and
for pipelined runs the two conditions of Eq. 3 (the previous pass's chunk
tk + dl, plus the team delay dt at a segment's front; the next pass's chunk
tk - du - 2, except at a segment's rear).  The pass-by-pass order of a
one-grid batch is checked too."""
import ctypes
import struct

import pytest

from paper_0912_4506_amd import _lib
from paper_0912_4506_amd._lib import Grid, Pipeline, Tile, JAC_EARG


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


HDR = struct.Struct("<I9i5q")           # magic, dtype .. team, grids_off .. max_shell
GRID = struct.Struct("<QQqq16i")        # a, b, sy, sz, nx .. counter_off, team, dl, du, dt


def parse(buf):
    raw = bytes(buf)
    h = HDR.unpack_from(raw, 0)
    nitems, order, team = h[3], h[8], h[9]
    grids_off, items_off = h[10], h[11]
    g = GRID.unpack_from(raw, grids_off)
    nti, ntj, nkc, passes = g[7], g[8], g[9], g[13]
    gteam, dl, du, dt = g[16], g[17], g[18], g[19]
    items = [struct.unpack_from("<4i", raw, items_off + 16 * n)[:3] for n in range(nitems)]
    return dict(order=order, team=team, nti=nti, ntj=ntj, nkc=nkc, passes=passes, items=items,
                gteam=gteam, dl=dl, du=du, dt=dt)


def plan(lib, shape, T, team, t, kchunk, bx=64, by=72, waves=12, dtype=1, sync=None):
    nx, ny, nz = shape
    g = Grid(nx, ny, nz, 0, 0)
    tile = Tile(t, bx, by, kchunk, waves)
    n = lib.jacobi_pipelined_plan_bytes(dtype, ctypes.byref(g), T, ctypes.byref(tile))
    assert n > 0, lib.jacobi_last_error()
    buf = (ctypes.c_ubyte * n)()
    out = (ctypes.c_int * 1)()
    sy = ctypes.byref(Pipeline(*sync)) if sync else None
    rc = lib.jacobi_pipelined_plan(dtype, ctypes.byref(g), ctypes.c_void_p(1 << 20),
                                   ctypes.c_void_p(1 << 34), T, team, sy, ctypes.byref(tile), buf, n,
                                   out)
    assert rc == 0, lib.jacobi_last_error()
    return parse(buf), out[0], buf


def waits(p, pas, tile):
    """(pass, tile) pairs the batched kernel makes item (pas, tile) wait on."""
    nti, ntj, nkc, team = p["nti"], p["ntj"], p["nkc"], p["gteam"]
    ti, tj, tk = tile % nti, tile // nti % ntj, tile // (nti * ntj)
    out = []
    if pas > 0:
        for dk in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    a, b, c = ti + di, tj + dj, tk + dk
                    if 0 <= a < nti and 0 <= b < ntj and 0 <= c < nkc:
                        out.append((pas - 1, (c * ntj + b) * nti + a))
    if team > 0 and pas > 0:
        c = min(tk + p["dl"] + (p["dt"] if pas % team == 0 else 0), nkc - 1)
        out.append((pas - 1, (c * ntj + tj) * nti + ti))
    if team > 0 and p["du"] > 0 and pas % team != team - 1 and pas + 1 < p["passes"]:
        c = tk - p["du"] - 2
        if c >= 0:
            out.append((pas + 1, (c * ntj + tj) * nti + ti))
    return out


def check_order(p):
    pos = {}
    for n, (grid, pas, tile) in enumerate(p["items"]):
        assert grid == 0
        assert (pas, tile) not in pos
        pos[(pas, tile)] = n
    nti, ntj, nkc = p["nti"], p["ntj"], p["nkc"]
    assert len(pos) == p["passes"] * nti * ntj * nkc
    for (pas, tile), n in pos.items():
        for dep in waits(p, pas, tile):
            assert pos[dep] < n, ((pas, tile), dep)


@pytest.mark.parametrize("shape,T,team,t,kchunk", [
    ((200, 150, 120), 13, 4, 1, 16),
    ((200, 150, 120), 13, 1, 2, 8),
    ((130, 70, 64), 20, 7, 1, 4),
    ((64, 64, 33), 9, 3, 3, 5),
    ((64, 64, 33), 9, 100, 1, 16),
])
def test_pipelined_order_respects_dependencies(lib, shape, T, team, t, kchunk):
    p, out_idx, _ = plan(lib, shape, T, team, t, kchunk)
    assert p["order"] == 1 and p["team"] == team
    assert p["passes"] == -(-T // t) and out_idx == p["passes"] % 2
    assert p["nkc"] == -(-shape[2] // kchunk)
    check_order(p)
    # within a segment, pass seg+s runs 2s chunks behind pass seg (dl = 1): the first
    # item of a later pass of the segment comes after its predecessor's item
    # on the next chunk
    firsts = {}
    for n, (_, pas, tile) in enumerate(p["items"]):
        firsts.setdefault(pas, n)
    assert all(firsts[q] < firsts[q + 1] for q in range(p["passes"] - 1))


def test_batch_order_respects_dependencies(lib):
    g = Grid(130, 70, 64, 0, 0)
    tile = Tile(2, 64, 72, 16, 12)
    T = (ctypes.c_int * 1)(7)
    n = lib.jacobi_batched_plan_bytes(1, 1, ctypes.byref(g), T, ctypes.byref(tile))
    buf = (ctypes.c_ubyte * n)()
    out = (ctypes.c_int * 1)()
    A = (ctypes.c_void_p * 1)(1 << 20)
    B = (ctypes.c_void_p * 1)(1 << 34)
    assert lib.jacobi_batched_plan(1, 1, ctypes.byref(g), A, B, T, ctypes.byref(tile), buf, n,
                                   out) == 0
    p = parse(buf)
    assert p["order"] == 0
    check_order(p)


def test_pipelined_argument_checks(lib):
    g = Grid(40, 40, 40, 0, 0)
    tile = Tile(1, 64, 72, 8, 12)
    n = lib.jacobi_pipelined_plan_bytes(1, ctypes.byref(g), 10, ctypes.byref(tile))
    buf = (ctypes.c_ubyte * n)()
    out = (ctypes.c_int * 1)()
    for team in (0, -3, 2000):
        assert lib.jacobi_pipelined_plan(1, ctypes.byref(g), ctypes.c_void_p(1 << 20),
                                         ctypes.c_void_p(1 << 34), 10, team, None,
                                         ctypes.byref(tile), buf, n, out) == JAC_EARG
    assert lib.jacobi_pipelined_plan(1, ctypes.byref(g), ctypes.c_void_p(1 << 20),
                                     ctypes.c_void_p(1 << 34), 10, 2, None, ctypes.byref(tile), buf,
                                     n - 16, out) != 0
    # a pipelined plan refuses lockstep runs before any HIP call
    p, _, buf = plan(lib, (40, 40, 40), 10, 2, 1, 8)
    ws = lib.jacobi_batched_workspace(buf)
    assert ws > 0
    rc = lib.jacobi_batched_run(buf, ctypes.c_void_p(1 << 36), ctypes.c_void_p(1 << 38), ws,
                                _lib.JAC_BATCH_LOCKSTEP, None)
    assert rc == JAC_EARG and "relaxed" in lib.jacobi_last_error().decode()


@pytest.mark.parametrize("sync", [(1, 1, 0), (1, 2, 0), (1, 4, 0), (1, 0, 0), (2, 2, 0), (2, 5, 3),
                                  (1, 1, 8), (3, 0, 8)])
@pytest.mark.parametrize("shape,T,team,t,kchunk", [
    ((200, 150, 120), 13, 4, 1, 16),
    ((130, 70, 64), 20, 7, 1, 4),
    ((64, 64, 33), 9, 3, 3, 5),
    ((130, 70, 300), 24, 6, 2, 8),
])
def test_relaxed_sync_waits_can_end(lib, shape, T, team, t, kchunk, sync):
    """Both conditions of Eq. 3 (lower distance dl, upper distance du, team
    delay dt): every counter an item waits on belongs to an earlier item, so
    every wait ends; the wavefront lag between consecutive passes of a
    segment is dl + 1 chunks."""
    p, _, _ = plan(lib, shape, T, team, t, kchunk, sync=sync)
    assert (p["dl"], p["du"], p["dt"], p["gteam"]) == (*sync, team)
    check_order(p)
    nij = p["nti"] * p["ntj"]
    first = {}
    for n, (_, pas, tile) in enumerate(p["items"]):
        first.setdefault((pas, tile // nij), n)
    lag = sync[0] + 1
    for pas in range(1, p["passes"]):
        if pas % team == 0:
            continue
        for q in range(p["nkc"] - lag):
            # pass pas on chunk q goes out with pass pas-1 on chunk q + lag
            assert first[(pas - 1, q + lag)] < first[(pas, q)]


def test_relaxed_sync_argument_checks(lib):
    g = Grid(40, 40, 40, 0, 0)
    tile = Tile(1, 64, 72, 8, 12)
    n = lib.jacobi_pipelined_plan_bytes(1, ctypes.byref(g), 10, ctypes.byref(tile))
    buf = (ctypes.c_ubyte * n)()
    out = (ctypes.c_int * 1)()
    for bad in [(0, 0, 0), (2, 1, 0), (1, 0, -1), (-1, 3, 0)]:
        rc = lib.jacobi_pipelined_plan(1, ctypes.byref(g), ctypes.c_void_p(1 << 20),
                                       ctypes.c_void_p(1 << 34), 10, 2,
                                       ctypes.byref(Pipeline(*bad)), ctypes.byref(tile), buf, n, out)
        assert rc == JAC_EARG, bad
    # a plain batch carries no pipeline distances
    T = (ctypes.c_int * 1)(7)
    nb = lib.jacobi_batched_plan_bytes(1, 1, ctypes.byref(g), T, ctypes.byref(tile))
    bb = (ctypes.c_ubyte * nb)()
    A = (ctypes.c_void_p * 1)(1 << 20)
    B = (ctypes.c_void_p * 1)(1 << 34)
    assert lib.jacobi_batched_plan(1, 1, ctypes.byref(g), A, B, T, ctypes.byref(tile), bb, nb,
                                   out) == 0
    p = parse(bb)
    assert (p["gteam"], p["du"], p["dt"]) == (0, 0, 0)


def batch_buf(lib, shapes, Ts, t=2, bx=64, by=72, waves=12, kchunk=16):
    n = len(shapes)
    G = (Grid * n)(*[Grid(*s, 0, 0) for s in shapes])
    T = (ctypes.c_int * n)(*Ts)
    tile = Tile(t, bx, by, kchunk, waves)
    nb = lib.jacobi_batched_plan_bytes(1, n, G, T, ctypes.byref(tile))
    buf = (ctypes.c_ubyte * nb)()
    A = (ctypes.c_void_p * n)(*[(2 * m + 1) << 32 for m in range(n)])
    B = (ctypes.c_void_p * n)(*[(2 * m + 2) << 32 for m in range(n)])
    assert lib.jacobi_batched_plan(1, n, G, A, B, T, ctypes.byref(tile), buf, nb,
                                   (ctypes.c_int * n)()) == 0, lib.jacobi_last_error()
    return buf


def all_items(buf):
    raw = bytes(buf)
    h = HDR.unpack_from(raw, 0)
    return [struct.unpack_from("<4i", raw, h[11] + 16 * n) for n in range(h[3])]


def test_stress_shuffles_within_passes_and_delays(lib):
    """jacobi_batched_stress: each pass keeps its item set and its place in
    the queue (so every wait still points to an earlier item), the order
    inside passes changes, about a quarter of the items get a delay in
    1..max_delay, and the same seed gives the same image."""
    buf = batch_buf(lib, [(130, 70, 64), (40, 30, 20), (90, 90, 33)], [7, 4, 6])
    before = all_items(buf)
    assert all(d == 0 for *_, d in before)
    keep = bytes(buf)
    assert lib.jacobi_batched_stress(buf, len(buf), 12345, 8) == 0
    after = all_items(buf)
    assert [x[:3] for x in after] != [x[:3] for x in before]
    passes_before = [x[1] for x in before]
    assert [x[1] for x in after] == passes_before          # pass boundaries unchanged
    for pas in set(passes_before):
        assert sorted(x[:3] for x in after if x[1] == pas) == \
            sorted(x[:3] for x in before if x[1] == pas)
    delays = [x[3] for x in after]
    assert all(0 <= d <= 8 for d in delays)
    frac = sum(d > 0 for d in delays) / len(delays)
    assert 0.15 < frac < 0.35, frac
    assert set(d for d in delays if d) == set(range(1, 9))
    # the same seed on the original image gives the same stressed image
    again = (ctypes.c_ubyte * len(buf)).from_buffer_copy(keep)
    assert lib.jacobi_batched_stress(again, len(again), 12345, 8) == 0
    assert bytes(again) == bytes(buf)
    # the header, grids and pass table are untouched
    h = HDR.unpack_from(keep, 0)
    assert bytes(buf)[:h[11]] == keep[:h[11]] and bytes(buf)[h[12]:] == keep[h[12]:]
    # max_delay 0: shuffle only
    only = (ctypes.c_ubyte * len(buf)).from_buffer_copy(keep)
    assert lib.jacobi_batched_stress(only, len(only), 7, 0) == 0
    assert all(x[3] == 0 for x in all_items(only))


def test_stress_keeps_the_pipelined_order(lib):
    p, _, buf = plan(lib, (130, 70, 64), 20, 7, 1, 4, sync=(1, 2, 1))
    before = all_items(buf)
    assert lib.jacobi_batched_stress(buf, len(buf), 99, 16) == 0
    after = all_items(buf)
    assert [x[:3] for x in after] == [x[:3] for x in before]
    assert any(x[3] for x in after) and max(x[3] for x in after) <= 16
    check_order(parse(buf))


def test_stress_argument_checks(lib):
    buf = batch_buf(lib, [(40, 30, 20)], [4])
    assert lib.jacobi_batched_stress(buf, len(buf), 1, 65) == JAC_EARG
    assert lib.jacobi_batched_stress(buf, len(buf), 1, -1) == JAC_EARG
    assert lib.jacobi_batched_stress(buf, len(buf) - 16, 1, 4) == JAC_EARG
    assert "plan_bytes" in lib.jacobi_last_error().decode()
    assert lib.jacobi_batched_stress(None, 0, 1, 4) == JAC_EARG
    junk = (ctypes.c_ubyte * 256)()
    assert lib.jacobi_batched_stress(junk, 256, 1, 4) == JAC_EARG


def test_damaged_plan_images_are_refused(lib):
    """An image whose offsets or pass table do not match the layout the plan
    builder writes is refused before anything reads past it."""
    buf = batch_buf(lib, [(40, 30, 20), (33, 17, 9)], [6, 4])
    good = bytes(buf)
    assert lib.jacobi_batched_workspace(buf) > 0
    h = list(HDR.unpack_from(good, 0))

    def damaged(field, value=None, pass_last=None):
        img = (ctypes.c_ubyte * len(good)).from_buffer_copy(good)
        if field is not None:
            hh = list(h)
            hh[field] = value
            HDR.pack_into(img, 0, *hh)
        if pass_last is not None:
            struct.pack_into("<i", img, h[12] + 4 * h[7], pass_last)
        return img

    for img in (damaged(11, h[12] + 16),            # items past the pass table
                damaged(3, h[3] + 1000),             # more items than the image holds
                damaged(12, h[13]),                  # pass table past the end
                damaged(7, h[7] + 50),               # more passes than the table holds
                damaged(None, pass_last=h[3] - 1)):  # pass table does not end at nitems
        assert lib.jacobi_batched_workspace(img) == 0
        assert "not a batch plan" in lib.jacobi_last_error().decode()
        assert lib.jacobi_batched_stress(img, len(img), 1, 4) == JAC_EARG
        assert lib.jacobi_batched_run(img, ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 34),
                                      1 << 20, 0, None) == JAC_EARG


def test_batch_argument_checks(lib):
    """Empty and oversized batches, missing arrays, a grid with T = 0 among
    others (it keeps its input: no items, out_idx 0) and overlapping grids."""
    g = (Grid * 2)(Grid(40, 30, 20, 0, 0), Grid(33, 17, 9, 0, 0))
    T = (ctypes.c_int * 2)(6, 0)
    tile = Tile(2, 64, 72, 16, 12)
    assert lib.jacobi_batched_plan_bytes(1, 0, g, T, ctypes.byref(tile)) == 0
    assert "batch size" in lib.jacobi_last_error().decode()
    assert lib.jacobi_batched_plan_bytes(1, 70000, g, T, ctypes.byref(tile)) == 0
    assert lib.jacobi_batched_plan_bytes(1, 2, None, T, ctypes.byref(tile)) == 0
    nb = lib.jacobi_batched_plan_bytes(1, 2, g, T, ctypes.byref(tile))
    assert nb > 0
    buf = (ctypes.c_ubyte * nb)()
    out = (ctypes.c_int * 2)(7, 7)
    A = (ctypes.c_void_p * 2)(1 << 32, 3 << 32)
    B = (ctypes.c_void_p * 2)(2 << 32, 4 << 32)
    assert lib.jacobi_batched_plan(1, 2, g, A, B, T, ctypes.byref(tile), buf, nb, out) == 0
    assert out[1] == 0
    items = all_items(buf)
    assert items and all(m == 0 for m, *_ in items)        # the T = 0 grid has no items
    assert lib.jacobi_batched_plan(1, 2, g, A, B, T, ctypes.byref(tile), buf, nb - 16,
                                   out) != 0
    Bo = (ctypes.c_void_p * 2)(2 << 32, (1 << 32) + 4096)  # grid 1's b inside grid 0's a
    assert lib.jacobi_batched_plan(1, 2, g, A, Bo, T, ctypes.byref(tile), buf, nb, out) == JAC_EARG
    assert "overlap" in lib.jacobi_last_error().decode()
