"""The tuning cache on the CPU: choices written to a text file, read back,
keyed by (architecture, dtype, geometry, T), consulted by the library's
default blocking, and loaded from JACOBI_TUNE_CACHE in a fresh process.
With no device visible the library takes the architecture to be gfx950."""
import ctypes
import os
import subprocess
import sys

import pytest

from paper_0912_4506_amd import _lib
from paper_0912_4506_amd._lib import Grid, Tile, JAC_EARG, JAC_EUNSUPPORTED

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = "# arch dtype nx ny nz sy sz T t bx by waves kchunk ms\n"
GOOD = ("gfx950 f64 40 30 20 42 1344 10 3 64 64 8 0 0.25\n"
        "gfx942 f64 40 30 20 42 1344 10 2 128 32 8 0 0.5\n"
        "gfx950 f32 512 512 512 514 264196 100 5 64 64 16 0 3.5\n")


@pytest.fixture
def lib():
    lib = _lib.load()
    assert lib.jacobi_tune_forget() == 0
    yield lib
    lib.jacobi_tune_forget()


def lookup(lib, arch, dtype, g, T):
    t = Tile()
    rc = lib.jacobi_tune_lookup(arch.encode() if arch else None, dtype, ctypes.byref(g), T,
                                ctypes.byref(t))
    return rc, (t.t, t.bx, t.by, t.waves, t.kchunk)


def test_load_lookup_save_roundtrip(lib, tmp_path):
    src = tmp_path / "tune.txt"
    src.write_text(HEADER + "\n   # indented comment\n" + GOOD)
    n = ctypes.c_int(-1)
    assert lib.jacobi_tune_load(str(src).encode(), ctypes.byref(n)) == 0 and n.value == 3
    g = Grid(40, 30, 20, 0, 0)          # sy, sz resolved to 42, 1344
    assert lookup(lib, "gfx950", 1, g, 10) == (0, (3, 64, 64, 8, 0))
    assert lookup(lib, "gfx942", 1, g, 10) == (0, (2, 128, 32, 8, 0))
    assert lookup(lib, None, 1, g, 10) == (0, (3, 64, 64, 8, 0))     # this process: gfx950
    assert lookup(lib, "gfx950", 1, g, 11)[0] == JAC_EUNSUPPORTED    # another T
    assert lookup(lib, "gfx950", 0, g, 10)[0] == JAC_EUNSUPPORTED    # another dtype
    assert lookup(lib, "gfx950", 1, Grid(40, 30, 20, 48, 0), 10)[0] == JAC_EUNSUPPORTED
    assert lookup(lib, "gfx950", 0, Grid(512, 512, 512, 0, 0), 100) == (0, (5, 64, 64, 16, 0))
    out = tmp_path / "saved.txt"
    assert lib.jacobi_tune_save(str(out).encode()) == 0
    text = out.read_text()
    assert sum(1 for l in text.splitlines() if l and not l.startswith("#")) == 3
    assert lib.jacobi_tune_forget() == 0
    assert lookup(lib, "gfx950", 1, g, 10)[0] == JAC_EUNSUPPORTED
    assert lib.jacobi_tune_load(str(out).encode(), ctypes.byref(n)) == 0 and n.value == 3
    assert lookup(lib, "gfx942", 1, g, 10) == (0, (2, 128, 32, 8, 0))
    again = tmp_path / "again.txt"
    assert lib.jacobi_tune_save(str(again).encode()) == 0
    assert again.read_text() == text
    assert not [p for p in os.listdir(tmp_path) if ".tmp." in p]


def test_default_tile_uses_the_cache(lib, tmp_path):
    g = Grid(40, 30, 20, 0, 0)
    before, before12 = Tile(), Tile()
    assert lib.jacobi_default_tile(1, ctypes.byref(g), 10, 0, 0, ctypes.byref(before)) == 0
    assert lib.jacobi_default_tile(1, ctypes.byref(g), 12, 0, 0, ctypes.byref(before12)) == 0
    src = tmp_path / "tune.txt"
    src.write_text("gfx950 f64 40 30 20 42 1344 10 2 128 32 8 0 0.1\n")
    assert lib.jacobi_tune_load(str(src).encode(), None) == 0
    t = Tile()
    assert lib.jacobi_default_tile(1, ctypes.byref(g), 10, 0, 0, ctypes.byref(t)) == 0
    assert (t.t, t.bx, t.by, t.waves) == (2, 128, 32, 8)
    assert (t.t, t.bx, t.by) != (before.t, before.bx, before.by)
    # another T: the library's own choice, as before the load
    assert lib.jacobi_default_tile(1, ctypes.byref(g), 12, 0, 0, ctypes.byref(t)) == 0
    assert (t.t, t.bx, t.by, t.waves) == (before12.t, before12.bx, before12.by, before12.waves)
    # a caller's own depth: the block shape is not taken from the cache either
    assert lib.jacobi_default_tile(1, ctypes.byref(g), 10, 3, 0, ctypes.byref(t)) == 0
    assert t.t == 3 and (t.bx, t.by) != (128, 32)


@pytest.mark.parametrize("line,why", [
    ("gfx950 f16 40 30 20 42 1344 10 3 64 64 8 0 0.25", "dtype"),
    ("gfx950 f64 40 30 20 42 1344 10 9 64 64 8 0 0.25", "range"),
    ("gfx950 f64 40 30 20 42 1344 10 3 96 64 8 0 0.25", "range"),       # not on the menu
    ("gfx950 f64 40 30 20 42 1344 10 3 64 64 0 0 0.25", "range"),       # waves must be given
    ("gfx950 f64 40 30 20 41 1344 10 3 64 64 8 0 0.25", "geometry"),    # sy < nx+2
    ("gfx950 f64 40 30 20 42 1344 2 3 64 64 8 0 0.25", "range"),        # t > T
    ("gfx950 f64 40 30 20 42 1344 10 3 64 64 8 0", "expected"),         # a field short
    ("gfx950 f64 40 30 20 42 1344 10 3 64 64 8 0 0.25 7", "expected"),  # a field more
    ("gfx/950 f64 40 30 20 42 1344 10 3 64 64 8 0 0.25", "architecture"),
    ("gfx950 f64 40 30 20 42 1344 10 3 64 64 8 -1 0.25", "range"),
    ("gfx950 f64 40 30 20 42 1344 10 3 64 64 8 0 nan", "range"),
])
def test_bad_lines_are_refused_whole(lib, tmp_path, line, why):
    src = tmp_path / "bad.txt"
    src.write_text(GOOD + line + "\n")
    assert lib.jacobi_tune_load(str(src).encode(), None) == JAC_EARG
    msg = lib.jacobi_last_error().decode()
    assert f"bad.txt:4:" in msg and why in msg, msg
    # nothing of the file is kept, not even its good lines
    assert lookup(lib, "gfx950", 1, Grid(40, 30, 20, 0, 0), 10)[0] == JAC_EUNSUPPORTED


def test_file_errors(lib, tmp_path):
    assert lib.jacobi_tune_load(str(tmp_path / "missing.txt").encode(), None) == JAC_EARG
    assert "cannot open" in lib.jacobi_last_error().decode()
    assert lib.jacobi_tune_save(str(tmp_path / "no" / "dir.txt").encode()) == JAC_EARG
    assert lib.jacobi_tune_load(None, None) == JAC_EARG
    assert lib.jacobi_tune_save(b"") == JAC_EARG
    long = tmp_path / "long.txt"
    long.write_text("#" * 2000 + "\n")
    assert lib.jacobi_tune_load(str(long).encode(), None) == JAC_EARG
    assert "too long" in lib.jacobi_last_error().decode()


CHILD = """
import ctypes, sys
sys.path.insert(0, {root!r})
from paper_0912_4506_amd import _lib
from paper_0912_4506_amd._lib import Grid, Tile
t = Tile()
assert _lib.load().jacobi_default_tile(1, ctypes.byref(Grid(40, 30, 20, 0, 0)), 10, 0, 0,
                                       ctypes.byref(t)) == 0
print(t.t, t.bx, t.by, t.waves)
"""


def child_default(env_path):
    env = dict(os.environ, JACOBI_TUNE_CACHE=str(env_path))
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return tuple(int(v) for v in r.stdout.split()), r.stderr


def test_environment_file_persists_across_processes(tmp_path):
    path = tmp_path / "env_tune.txt"
    path.write_text("gfx950 f64 40 30 20 42 1344 10 2 128 32 8 0 0.1\n")
    got, _ = child_default(path)
    assert got == (2, 128, 32, 8)
    # a file that does not parse: reported, ignored, the library's own default used
    path.write_text("garbage\n")
    got_bad, err = child_default(path)
    assert "ignoring the tuning cache" in err and "env_tune.txt:1" in err
    assert got_bad != (2, 128, 32, 8)
    # no file yet: no error
    got_none, err = child_default(tmp_path / "not_yet.txt")
    assert got_none == got_bad and err == ""
