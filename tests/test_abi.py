"""The C ABI on the CPU: libjacobi.so loads, exports every function
include/jacobi.h declares, and rejects bad arguments before any HIP call
(so no GPU is needed)."""
import ctypes

import pytest

from paper_0912_4506_amd import _lib
from paper_0912_4506_amd._lib import Grid, Tile, JAC_EARG, JAC_EUNSUPPORTED, JAC_EWORKSPACE


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _lib.declared_symbols()
    assert len(declared) >= 12
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared) == set(_lib.SIGNATURES), "binding and header disagree"
    assert lib.jacobi_version() == 3


P = ctypes.c_void_p
A = P(1 << 20)
B = P(1 << 30)
OUT = ctypes.c_int()


def err(lib):
    return lib.jacobi_last_error().decode()


def call_plain(lib, g, a=A, b=B, T=3, dtype=1):
    return lib.jacobi_plain(dtype, ctypes.byref(g) if g is not None else None, a, b, T, None,
                            ctypes.byref(OUT))


def test_grid_checks(lib):
    assert call_plain(lib, Grid(0, 4, 4, 0, 0)) == JAC_EARG and "extents" in err(lib)
    assert call_plain(lib, Grid(4, 4, 4, 5, 0)) == JAC_EARG and "sy" in err(lib)
    assert call_plain(lib, Grid(4, 4, 4, 6, 30)) == JAC_EARG and "sz" in err(lib)
    assert call_plain(lib, None) == JAC_EARG and "NULL" in err(lib)


def test_pointer_and_dtype_checks(lib):
    g = Grid(4, 4, 4, 0, 0)
    assert call_plain(lib, g, a=None) == JAC_EARG and "a is NULL" in err(lib)
    assert call_plain(lib, g, a=P((1 << 20) + 4)) == JAC_EARG and "aligned" in err(lib)
    assert call_plain(lib, g, b=P((1 << 20) + 8 * 10)) == JAC_EARG and "overlap" in err(lib)
    assert call_plain(lib, g, dtype=7) == JAC_EARG and "dtype" in err(lib)
    assert call_plain(lib, g, T=-1) == JAC_EARG and "negative" in err(lib)


def test_zero_sweeps_enqueue_nothing(lib):
    OUT.value = 5
    assert call_plain(lib, Grid(4, 4, 4, 0, 0), T=0) == 0 and OUT.value == 0
    assert err(lib) == ""


def test_tile_checks(lib):
    g = Grid(8, 8, 8, 0, 0)

    def tb(tile):
        return lib.jacobi_tblock(1, ctypes.byref(g), A, B, 5, ctypes.byref(tile), None, None,
                                 ctypes.byref(OUT))

    assert tb(Tile(9, 0, 0, 0, 0)) == JAC_EARG and "depth" in err(lib)
    assert tb(Tile(4, 100, 0, 0, 0)) == JAC_EARG
    assert tb(Tile(4, 100, 100, 0, 0)) == JAC_EUNSUPPORTED and "menu" in err(lib)
    assert tb(Tile(4, 64, 48, 0, 5)) == JAC_EUNSUPPORTED and "waves" in err(lib)
    assert tb(Tile(2, 0, 0, -1, 0)) == JAC_EARG and "kchunk" in err(lib)


def test_menu_and_default_tile(lib):
    buf = (ctypes.c_int * 192)()
    n = lib.jacobi_tile_menu(1, buf, 64)
    assert n >= 2
    shapes = [(buf[3 * m], buf[3 * m + 1], buf[3 * m + 2]) for m in range(n)]
    assert all(bx % 64 == 0 and by > 0 and w in (4, 8, 12, 16) for bx, by, w in shapes)
    assert len(set(shapes)) == len(shapes)
    t = Tile()
    for kind in (0, 1, 2):
        assert lib.jacobi_default_tile(1, ctypes.byref(Grid(512, 512, 512, 0, 0)), 100, 0, kind,
                                       ctypes.byref(t)) == 0
        assert 1 <= t.t <= 8 and (t.bx, t.by, t.waves) in shapes
    for kind in (-1, 3):
        assert lib.jacobi_default_tile(1, ctypes.byref(Grid(512, 512, 512, 0, 0)), 100, 0, kind,
                                       ctypes.byref(t)) == -1
        assert b"kind" in lib.jacobi_last_error()
    # depth never exceeds the sweep count
    assert lib.jacobi_default_tile(1, ctypes.byref(Grid(9, 9, 9, 0, 0)), 3, 8, 0,
                                   ctypes.byref(t)) == 0
    assert t.t == 3


def test_adjoint_workspace_checks(lib):
    g = Grid(10, 11, 12, 0, 0)
    need = lib.jacobi_adjoint_workspace(1, ctypes.byref(g), 4)
    faces = 2 * (11 * 12 + 10 * 12 + 10 * 11)
    assert need == (2 + 4) * faces * 8
    tile = Tile(4, 0, 0, 0, 0)
    rc = lib.jacobi_adjoint(1, ctypes.byref(g), A, B, 5, ctypes.byref(tile), None, 0, None,
                            ctypes.byref(OUT))
    assert rc == JAC_EWORKSPACE
    rc = lib.jacobi_adjoint(1, ctypes.byref(g), A, B, 5, ctypes.byref(tile), P(1 << 34), need - 8,
                            None, ctypes.byref(OUT))
    assert rc == JAC_EWORKSPACE and "needed" in err(lib)


def test_adjoint_refuses_faces_beyond_2gib(lib):
    """The trace pass addresses one level of shell faces with 32-bit byte
    offsets: a grid whose faces take 2 GiB or more per level is refused
    before anything is enqueued (here 2 (ny nz + nx nz + nx ny) > 2^28)."""
    g = Grid(8, 1 << 14, 1 << 14, 0, 0)
    tile = Tile(4, 0, 0, 0, 0)
    rc = lib.jacobi_adjoint(1, ctypes.byref(g), P(1 << 40), P(1 << 44), 5, ctypes.byref(tile),
                            None, 0, None, ctypes.byref(OUT))
    assert rc == JAC_EUNSUPPORTED and "2 GiB" in err(lib)
    # FP32 halves the bytes: 2^29 values * 4 B is still 2 GiB
    rc = lib.jacobi_adjoint(0, ctypes.byref(g), P(1 << 40), P(1 << 44), 5, ctypes.byref(tile),
                            None, 0, None, ctypes.byref(OUT))
    assert rc == JAC_EUNSUPPORTED
    # T = 0 is the identity and needs no trace
    assert lib.jacobi_adjoint(1, ctypes.byref(g), P(1 << 40), P(1 << 44), 0, ctypes.byref(tile),
                              None, 0, None, ctypes.byref(OUT)) == 0


def test_residual_and_copy_checks(lib):
    g = Grid(10, 10, 10, 0, 0)
    n2 = P(1 << 36)
    need = lib.jacobi_residual_workspace(ctypes.byref(g))
    assert need > 0
    assert lib.jacobi_residual_f64(ctypes.byref(g), A, B, n2, None, 0, None) == JAC_EWORKSPACE
    assert lib.jacobi_residual_f64(ctypes.byref(g), A, P((1 << 20) + 16), n2, P(1 << 38), need,
                                   None) == JAC_EARG
    # the fused update-residual: missing workspace, then overlapping buffers
    bufs = [P(1 << k) for k in (20, 22, 24, 26, 28)]   # x, e32, x_new, r32, zero32
    assert lib.jacobi_update_residual_f64(ctypes.byref(g), *bufs, n2, None, 0,
                                          None) == JAC_EWORKSPACE
    assert lib.jacobi_update_residual_f64(ctypes.byref(g), *bufs, n2, P(1 << 38), need - 8,
                                          None) == JAC_EWORKSPACE
    for u in range(5):
        bad = list(bufs)
        bad[u] = P(bufs[(u + 1) % 5].value + 64)       # inside the next buffer
        assert lib.jacobi_update_residual_f64(ctypes.byref(g), *bad, n2, P(1 << 38), need,
                                              None) == JAC_EARG, u
        assert "overlap" in err(lib)
    assert lib.jacobi_update_residual_f64(ctypes.byref(g), bufs[0], bufs[1], bufs[2], bufs[3],
                                          bufs[4], P(bufs[3].value + 8), P(1 << 38), need,
                                          None) == JAC_EARG             # norm2 inside r32
    assert lib.jacobi_copy(A, P((1 << 20) + 16), 64, None) == JAC_EARG   # overlap
    assert lib.jacobi_copy(A, B, 12, None) == JAC_EARG                   # not a multiple of 16


def test_compressed_checks(lib):
    """jacobi_compressed: the frame shift is t, so t is required; the array
    strides must leave room for both frames; 64-wide blocks only."""
    g = Grid(40, 30, 20, 0, 0)
    ws_need = lib.jacobi_compressed_workspace(1, ctypes.byref(g), 10, ctypes.byref(Tile(4, 0, 0, 0, 0)))
    assert ws_need > 0
    # the saved shell and the per-pass counters are always there; plane copies
    # only with several k chunks
    one_chunk = lib.jacobi_compressed_workspace(1, ctypes.byref(g), 10,
                                                ctypes.byref(Tile(4, 0, 0, 20, 0)))
    two_chunks = lib.jacobi_compressed_workspace(1, ctypes.byref(g), 10,
                                                 ctypes.byref(Tile(4, 0, 0, 10, 0)))
    assert two_chunks - one_chunk >= 9 * 46 * 36 * 8   # 2t+1 planes of the padded array
    WS = P(1 << 34)
    out = ctypes.c_int(7)

    def call(g=g, u=A, T=10, tile=Tile(4, 0, 0, 0, 0), ws=WS, nbytes=ws_need, dtype=1, outp=True):
        return lib.jacobi_compressed(dtype, ctypes.byref(g), u, T, ctypes.byref(tile), ws, nbytes,
                                     None, ctypes.byref(out) if outp else None)

    assert lib.jacobi_compressed_workspace(1, ctypes.byref(g), 10, ctypes.byref(Tile())) == 0
    assert "tile->t" in err(lib)
    assert call(tile=Tile(0, 0, 0, 0, 0)) == JAC_EARG and "t in 1.." in err(lib)
    assert call(tile=Tile(9, 0, 0, 0, 0)) == JAC_EARG
    assert call(g=Grid(40, 30, 20, 43, 0)) == JAC_EARG and "nx+2+t" in err(lib)
    assert call(g=Grid(40, 30, 20, 46, 46 * 35)) == JAC_EARG and "ny+2+t" in err(lib)
    assert call(tile=Tile(4, 128, 32, 0, 0)) == JAC_EUNSUPPORTED and "64-wide" in err(lib)
    assert call(tile=Tile(4, 0, 0, 3, 0)) == JAC_EARG and "kchunk" in err(lib)
    assert call(T=-1) == JAC_EARG
    assert call(u=None) == JAC_EARG and "u is NULL" in err(lib)
    assert call(ws=None) == JAC_EWORKSPACE
    assert call(nbytes=ws_need - 1) == JAC_EWORKSPACE
    assert call(ws=P((1 << 34) + 8)) == JAC_EARG and "256-byte" in err(lib)
    assert call(ws=P((1 << 20) + 256)) == JAC_EARG and "overlaps" in err(lib)
    assert call(outp=False) == JAC_EARG and "out_frame" in err(lib)
    assert call(T=0) == 0 and out.value == 0          # nothing enqueued


def test_lbm_argument_checks(lib):
    from paper_0912_4506_amd._lib import LbmGrid
    g = LbmGrid(8, 8, 8)
    n = 19 * 8 * 8 * 8 * 8

    def call(grid=g, f=A, ft=P((1 << 20) + n), omega=1.0, T=2, dtype=1):
        return lib.lbm_d3q19_steps(dtype, ctypes.byref(grid) if grid is not None else None, f, ft,
                                   omega, T, None, ctypes.byref(OUT))

    assert call(grid=None) == JAC_EARG and "NULL" in err(lib)
    assert call(grid=LbmGrid(0, 8, 8)) == JAC_EARG and "extents" in err(lib)
    assert call(grid=LbmGrid(8, 8, 70000)) == JAC_EARG and "large" in err(lib)
    assert call(ft=P((1 << 20) + n - 8)) == JAC_EARG and "overlap" in err(lib)
    assert call(f=None) == JAC_EARG
    assert call(omega=float("nan")) == JAC_EARG and "omega" in err(lib)
    assert call(T=-1) == JAC_EARG
    assert call(dtype=3) == JAC_EARG
    OUT.value = 5
    assert call(T=0) == 0 and OUT.value == 0

    def blocked(grid=g, T=2, kchunk=0, ft=P((1 << 20) + n)):
        return lib.lbm_d3q19_blocked(1, ctypes.byref(grid), A, ft, 1.0, T, kchunk, None,
                                     ctypes.byref(OUT))

    assert blocked(kchunk=-1) == JAC_EARG and "kchunk" in err(lib)
    assert blocked(kchunk=70000) == JAC_EARG
    assert blocked(grid=LbmGrid(8, 400000, 2), ft=P(1 << 40)) == JAC_EARG and "ny/6" in err(lib)
    assert blocked(ft=P((1 << 20) + n - 8)) == JAC_EARG and "overlap" in err(lib)
    OUT.value = 5
    assert blocked(T=0) == 0 and OUT.value == 0


def test_noalloc_residual_refuses_large_grids(lib):
    """More partial sums than the fixed array holds: refused before any HIP call."""
    g = Grid(16384, 2048, 4096, 0, 0)       # 64 * 256 * 64 partial sums > 2^17
    rc = lib.jacobi_residual_f64_noalloc(ctypes.byref(g), P(1 << 44), P(1 << 46), P(1 << 20), None)
    assert rc == JAC_EUNSUPPORTED and "partial sums" in err(lib)
    rc = lib.jacobi_residual_f64_noalloc(ctypes.byref(Grid(8, 8, 8, 0, 0)), P(1 << 20), P(1 << 20),
                                         P(1 << 30), None)
    assert rc == JAC_EARG and "overlap" in err(lib)


def test_grid_add_checks(lib):
    g = Grid(6, 6, 6, 0, 0)
    span = 8 * 8 * 8 * 8
    assert lib.jacobi_grid_add(1, ctypes.byref(g), A, P((1 << 20) + span - 8), None) == JAC_EARG
    assert "overlap" in err(lib)
    assert lib.jacobi_grid_add(1, ctypes.byref(g), A, P((1 << 20) + 4), None) == JAC_EARG
    assert lib.jacobi_grid_add(1, ctypes.byref(g), None, B, None) == JAC_EARG and "dst" in err(lib)
    assert lib.jacobi_grid_add(5, ctypes.byref(g), A, B, None) == JAC_EARG
    assert lib.jacobi_grid_add(1, ctypes.byref(Grid(6, 6, 6, 7, 0)), A, B, None) == JAC_EARG


def test_size_limits(lib):
    """Extents above 2^28 and planes of 2 GiB or more are refused before any
    HIP call (the kernels index planes and rows with 32-bit values)."""
    big = Grid(1 << 28 | 1, 4, 4, 0, 0)
    assert call_plain(lib, big) == JAC_EARG and "2^28" in err(lib)
    wide = Grid(16384, 16384, 2, 0, 0)                 # 16386^2 doubles = 2.15 GB per plane
    assert call_plain(lib, wide, a=P(1 << 40), b=P(1 << 44)) == JAC_EUNSUPPORTED
    assert "2 GiB" in err(lib)
    rc = lib.jacobi_tblock(1, ctypes.byref(wide), P(1 << 40), P(1 << 44), 4, None, None, None,
                           ctypes.byref(OUT))
    assert rc == JAC_EUNSUPPORTED and "2 GiB" in err(lib)
    fits = Grid(16382, 16382, 2, 0, 0)                 # 16384^2 doubles: 2 GiB exactly
    assert call_plain(lib, fits, a=P(1 << 40), b=P(1 << 44)) == JAC_EUNSUPPORTED
