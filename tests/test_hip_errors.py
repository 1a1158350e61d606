"""HIP error paths, forced from the host: in a process with no GPU visible,
every entry point that enqueues work gets past its argument checks (valid
grids, aligned, disjoint device addresses) and then meets a real HIP error
at its first HIP call.  Each must return JAC_EHIP, name the step and the HIP
error in jacobi_last_error(), and leave the library usable: the next call's
own argument error or success replaces the message.  (On a machine with a
GPU these calls would run kernels on the fake addresses, so the test is
skipped there.)"""
import ctypes

import pytest

from paper_0912_4506_amd import _lib
from paper_0912_4506_amd._lib import (Grid, Tile, LbmGrid, Pipeline, JAC_EARG, JAC_EHIP)

P = ctypes.c_void_p


def _gpu_visible():
    import torch
    return torch.cuda.is_available()


pytestmark = pytest.mark.skipif(_gpu_visible(), reason="needs a process with no GPU visible")

OUT = ctypes.c_int()
G = Grid(40, 30, 20, 0, 0)
SPAN = 42 * 32 * 22


def addr(k):
    """Disjoint, 256-byte aligned fake device addresses, 1 GiB apart."""
    return P((k + 1) << 30)


def batched_plan(lib, pipelined):
    a = (P * 1)(addr(0))
    b = (P * 1)(addr(1))
    T = (ctypes.c_int * 1)(8)
    tile = Tile(4, 0, 0, 0, 0)
    idx = (ctypes.c_int * 1)()
    if pipelined:
        n = lib.jacobi_pipelined_plan_bytes(1, ctypes.byref(G), 8, ctypes.byref(tile))
        buf = ctypes.create_string_buffer(n)
        rc = lib.jacobi_pipelined_plan(1, ctypes.byref(G), addr(0), addr(1), 8, 2,
                                       ctypes.byref(Pipeline(1, 2, 0)), ctypes.byref(tile),
                                       buf, n, idx)
    else:
        n = lib.jacobi_batched_plan_bytes(1, 1, ctypes.byref(G), T, ctypes.byref(tile))
        buf = ctypes.create_string_buffer(n)
        rc = lib.jacobi_batched_plan(1, 1, ctypes.byref(G), a, b, T, ctypes.byref(tile), buf, n,
                                     idx)
    assert rc == 0, lib.jacobi_last_error()
    return buf, lib.jacobi_batched_workspace(buf)


def calls(lib):
    g = ctypes.byref(G)
    t4 = ctypes.byref(Tile(4, 0, 0, 0, 0))
    ws = addr(8)
    res_ws = lib.jacobi_residual_workspace(g)
    adj_ws = lib.jacobi_adjoint_workspace(1, g, 4)
    comp_ws = lib.jacobi_compressed_workspace(1, ctypes.byref(Grid(40, 30, 20, 46, 46 * 36)), 8, t4)
    bplan, bws = batched_plan(lib, False)
    pplan, pws = batched_plan(lib, True)
    best = Tile()
    ms = ctypes.c_float()
    return {
        "plain": lambda: lib.jacobi_plain(1, g, addr(0), addr(1), 3, None, ctypes.byref(OUT)),
        "tblock": lambda: lib.jacobi_tblock(1, g, addr(0), addr(1), 8, t4, None, None,
                                            ctypes.byref(OUT)),
        "tblock_rhs": lambda: lib.jacobi_tblock(0, g, addr(0), addr(1), 8, t4, addr(2), None,
                                                ctypes.byref(OUT)),
        "adjoint": lambda: lib.jacobi_adjoint(1, g, addr(0), addr(1), 8, t4, ws, adj_ws, None,
                                              ctypes.byref(OUT)),
        "residual": lambda: lib.jacobi_residual_f64(g, addr(0), addr(1), addr(2), ws, res_ws, None),
        "residual_noalloc": lambda: lib.jacobi_residual_f64_noalloc(g, addr(0), addr(1), addr(2),
                                                                    None),
        "update": lambda: lib.jacobi_update_f64(g, addr(0), addr(1), None),
        "update_residual": lambda: lib.jacobi_update_residual_f64(
            g, addr(0), addr(1), addr(2), addr(3), addr(4), addr(5), ws, res_ws, None),
        "fill": lambda: lib.jacobi_fill(1, g, addr(0), 1.0, None),
        "grid_add": lambda: lib.jacobi_grid_add(1, g, addr(0), addr(1), None),
        "copy": lambda: lib.jacobi_copy(addr(0), addr(1), 1 << 20, None),
        "batched_relaxed": lambda: lib.jacobi_batched_run(bplan, addr(6), ws, bws, 0, None),
        "batched_lockstep": lambda: lib.jacobi_batched_run(bplan, addr(6), ws, bws, 1, None),
        "pipelined": lambda: lib.jacobi_batched_run(pplan, addr(6), ws, pws, 0, None),
        "compressed": lambda: lib.jacobi_compressed(1, ctypes.byref(Grid(40, 30, 20, 46, 46 * 36)),
                                                    addr(0), 8, t4, ws, comp_ws, None,
                                                    ctypes.byref(OUT)),
        "lbm": lambda: lib.lbm_d3q19_steps(1, ctypes.byref(LbmGrid(16, 8, 8)), addr(0), addr(1),
                                           1.2, 2, None, ctypes.byref(OUT)),
        "lbm_blocked": lambda: lib.lbm_d3q19_blocked(1, ctypes.byref(LbmGrid(16, 8, 8)), addr(0),
                                                     addr(1), 1.2, 2, 0, None, ctypes.byref(OUT)),
        "autotune": lambda: lib.jacobi_autotune(1, g, addr(0), addr(1), 4, 2, 1, ctypes.byref(best),
                                                ctypes.byref(ms), None),
    }


def test_every_enqueuing_entry_point_reports_the_hip_error():
    lib = _lib.load()
    table = calls(lib)
    assert set(table) >= {"plain", "tblock", "adjoint", "residual", "residual_noalloc", "update",
                          "update_residual", "fill", "grid_add", "copy", "batched_relaxed",
                          "pipelined", "compressed", "lbm", "lbm_blocked", "autotune"}
    for name, call in table.items():
        rc = call()
        msg = lib.jacobi_last_error().decode()
        assert rc == JAC_EHIP, (name, rc, msg)
        assert "HIP error" in msg and ":" in msg.split("HIP error")[0], (name, msg)
        # the library is still usable: an argument error replaces the message...
        assert lib.jacobi_plain(1, ctypes.byref(Grid(0, 4, 4, 0, 0)), addr(0), addr(1), 1, None,
                                ctypes.byref(OUT)) == JAC_EARG
        assert "extents" in lib.jacobi_last_error().decode()
        # ...and a call with nothing to enqueue succeeds and clears it
        assert lib.jacobi_plain(1, ctypes.byref(G), addr(0), addr(1), 0, None,
                                ctypes.byref(OUT)) == 0
        assert lib.jacobi_last_error().decode() == ""


def test_python_binding_raises_with_the_code():
    from paper_0912_4506_amd._lib import check, JacobiError
    lib = _lib.load()
    rc = lib.jacobi_fill(1, ctypes.byref(G), addr(0), 0.0, None)
    with pytest.raises(JacobiError) as e:
        check(rc)
    assert e.value.code == JAC_EHIP and "fill launch" in str(e.value)
