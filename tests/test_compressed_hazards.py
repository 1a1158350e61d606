"""Host-side check of the compressed single grid's hazard analysis (no GPU).

Block placement as the library documents it (include/jacobi.h, tblock.h):
along an axis of n interior cells, blocks w cells wide with halo h; block 0
starts at the shell cell and is valid on [1, w - h), block b >= 1 on w - 2h
more cells.  A block reads its whole extended extent (clamped into the grid)
of the input frame, over its own k chunk's planes and the shell planes (other
chunks' planes come from copies), and writes its valid cells into the output
frame, shifted by S against the input (array index = cell + S in frame 0).

Checked by box intersection on many geometries: whenever a block's output
box meets another block's input box, that other block is one of the three
it waits for (same k chunk, neighbour at -1 along i, j or both for the pass
that writes frame 1, at +1 for the pass back), and no two blocks write the
same cell.  Geometries where a valid width is below depth + S are the ones
the library refuses.
"""
import itertools

import pytest


def axis_tile(blk, n, w, h):
    first, mid = w - h, w - 2 * h
    if blk == 0:
        e, a, b = 0, 1, first
    else:
        a = first + (blk - 1) * mid
        e, b = a - h, a + mid
    return e, a, min(b, n + 1)


def axis_blocks(n, w, h):
    first, mid = w - h, w - 2 * h
    return 1 if first >= n + 1 else 1 + (n + 1 - first + mid - 1) // mid


def meets(a, b):
    return a[0] <= b[1] and b[0] <= a[1]


def violations(nx, ny, nz, bx, by, d, S, kchunk, direction):
    nti, ntj = axis_blocks(nx, bx, d), axis_blocks(ny, by, d)
    nkc = -(-nz // kchunk)
    src, dst = (S, 0) if direction > 0 else (0, S)
    items = []
    for tk, tj, ti in itertools.product(range(nkc), range(ntj), range(nti)):
        ei, ai, bi = axis_tile(ti, nx, bx, d)
        ej, aj, bj = axis_tile(tj, ny, by, d)
        k0 = 1 + tk * kchunk
        k1 = min(k0 + kchunk, nz + 1)
        kstart = max(k0 - d, 0)
        reads_k = [(max(kstart, k0), min(k1 + d, k1 - 1))]
        if kstart == 0:
            reads_k.append((0, 0))
        if k1 + d >= nz + 1:
            reads_k.append((nz + 1, nz + 1))
        r = ((max(ei, 0) + src, min(ei + bx - 1, nx + 1) + src),
             (max(ej, 0) + src, min(ej + by - 1, ny + 1) + src), reads_k)
        wbox = ((ai + dst, bi - 1 + dst), (aj + dst, bj - 1 + dst), (k0, k1 - 1))
        step = -1 if direction > 0 else 1
        deps = {(ti + step, tj, tk), (ti, tj + step, tk), (ti + step, tj + step, tk)}
        items.append(((ti, tj, tk), r, wbox, deps))
    bad = []
    for (zid, _, zw, zdeps), (yid, yr, yw, _) in itertools.permutations(items, 2):
        if meets(yr[0], zw[0]) and meets(yr[1], zw[1]) and any(meets(k, zw[2]) for k in yr[2]):
            if yid not in zdeps:
                bad.append(("missing wait", zid, yid))
        if all(meets(yw[a], zw[a]) for a in range(3)):
            bad.append(("double write", zid, yid))
    return bad


GEOMETRIES = [(150, 100, 40), (64, 70, 17), (129, 130, 31), (5, 3, 9)]
SHAPES = [(64, 72), (64, 48), (64, 32), (64, 56)]


@pytest.mark.parametrize("grid", GEOMETRIES)
def test_only_three_neighbours_are_overwritten(grid):
    nx, ny, nz = grid
    checked = 0
    for (bx, by), d in itertools.product(SHAPES, range(1, 9)):
        for S in (d, d + 1):                    # pass depths t and t - 1 share S = t
            if bx - 2 * d < d + S or by - 2 * d < d + S:
                continue                        # refused by the library
            for kchunk in sorted({S, S + 3, 16, nz}):
                kchunk = max(kchunk, S)
                for direction in (1, -1):
                    assert violations(nx, ny, nz, bx, by, d, S, kchunk, direction) == []
                    checked += 1
    assert checked > 50


def test_narrow_blocks_would_need_more_waits():
    """The width condition is needed: a 32-row block at depth 8 with S = 9
    (valid width 16 < d + S) overwrites inputs of the block two rows away."""
    bad = violations(150, 100, 40, 64, 32, 8, 9, 9, 1)
    assert any(kind == "missing wait" for kind, _, _ in bad)
