"""PyTorch-facing wrappers of libjacobi.so.

Grids are torch tensors on the GPU of shape (nz+2, ny+2, nx+2), dtype float32
or float64, with unit stride along the last axis (i); the other two strides
may be padded.  PyTorch provides the device memory and the stream (the
current stream of the tensor's device); every step runs in the library's
kernels.  The wrappers only marshal arguments.
"""
import ctypes
import os

import torch

from . import _lib
from ._lib import Grid, Tile, check

_DTYPES = {torch.float32: _lib.JAC_F32, torch.float64: _lib.JAC_F64}


def dtype_code(x):
    try:
        return _DTYPES[x.dtype]
    except KeyError:
        raise TypeError(f"grids must be float32 or float64, got {x.dtype}") from None


def grid_of(x):
    """jac_grid_t of a (nz+2, ny+2, nx+2) tensor (strides in elements)."""
    if x.dim() != 3:
        raise ValueError(f"grid must be 3-D (nz+2, ny+2, nx+2), got shape {tuple(x.shape)}")
    if x.stride(2) != 1:
        raise ValueError("grid must be contiguous along i (last axis)")
    nz, ny, nx = (s - 2 for s in x.shape)
    return Grid(nx, ny, nz, x.stride(1), x.stride(0))


def _same(a, b):
    if a.shape != b.shape or a.dtype != b.dtype or a.device != b.device:
        raise ValueError("grids must share shape, dtype and device")
    if a.stride() != b.stride():
        raise ValueError("grids must share strides")


def _stream(x):
    if not x.is_cuda:
        raise ValueError("grids must live on the GPU")
    return ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _tile(t=None, bx=0, by=0, kchunk=0, waves=0):
    return Tile(int(t or 0), int(bx or 0), int(by or 0), int(kchunk or 0), int(waves or 0))


def plain(a, b, T):
    """T plain sweeps; a holds level 0.  Returns the tensor (a or b) holding
    level T."""
    _same(a, b)
    out = ctypes.c_int(0)
    lib = _lib.load()
    with torch.cuda.device(a.device):
        check(lib.jacobi_plain(dtype_code(a), ctypes.byref(grid_of(a)), _ptr(a), _ptr(b), int(T),
                               _stream(a), ctypes.byref(out)))
    return b if out.value else a


def tblock(a, b, T, t=None, bx=0, by=0, kchunk=0, rhs=None, waves=0):
    """T sweeps fused t per pass (t=None: library choice).  With rhs, each
    sweep computes (six neighbours + rhs) / 6.  Returns the tensor holding
    level T."""
    _same(a, b)
    if rhs is not None:
        _same(a, rhs)
    out = ctypes.c_int(0)
    lib = _lib.load()
    tile = _tile(t, bx, by, kchunk, waves)
    with torch.cuda.device(a.device):
        check(lib.jacobi_tblock(dtype_code(a), ctypes.byref(grid_of(a)), _ptr(a), _ptr(b), int(T),
                                ctypes.byref(tile), _ptr(rhs), _stream(a), ctypes.byref(out)))
    return b if out.value else a


def copy(dst, src):
    """dst <- src with the library's copy kernel (the M_s probe)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("copy needs two contiguous tensors of the same byte size")
    with torch.cuda.device(src.device):
        check(_lib.load().jacobi_copy(_ptr(dst), _ptr(src), nbytes, _stream(src)))
    return dst


def tile_menu(dtype=torch.float64):
    """Compiled block shapes: (bx, by, waves) triples."""
    lib = _lib.load()
    buf = (ctypes.c_int * 192)()
    n = lib.jacobi_tile_menu(_DTYPES[dtype], buf, 64)
    check(0 if n >= 0 else n)
    return [(buf[3 * m], buf[3 * m + 1], buf[3 * m + 2]) for m in range(min(n, 64))]


def default_tile(shape, T, t=0, dtype=torch.float64, rhs=False, adjoint=False):
    """Library choice of (t, bx, by, kchunk, waves) for a (nz+2, ny+2, nx+2)
    grid (rhs: for sweeps with a right-hand side; adjoint: for adjoint())."""
    nz, ny, nx = (s - 2 for s in shape)
    tile = Tile()
    kind = 2 if adjoint else int(bool(rhs))
    check(_lib.load().jacobi_default_tile(_DTYPES[dtype], ctypes.byref(Grid(nx, ny, nz, 0, 0)),
                                          int(T), int(t or 0), kind, ctypes.byref(tile)))
    return tile.t, tile.bx, tile.by, tile.kchunk, tile.waves


def adjoint_workspace(like, t=0):
    """Device workspace (uint8 tensor) for adjoint() on grids shaped like ``like``."""
    n = _lib.load().jacobi_adjoint_workspace(dtype_code(like), ctypes.byref(grid_of(like)), int(t or 0))
    if n == 0:
        check(_lib.JAC_EARG)
    return torch.empty(n, dtype=torch.uint8, device=like.device)


def adjoint(lam_a, lam_b, T, t=None, bx=0, by=0, kchunk=0, ws=None, waves=0):
    """Adjoint of T sweeps.  lam_a holds dL/d(level T) (whole grid); returns the
    tensor (lam_a or lam_b) holding dL/d(level 0): interior and shell."""
    _same(lam_a, lam_b)
    if ws is None:
        ws = adjoint_workspace(lam_a, t or 0)
    out = ctypes.c_int(0)
    tile = _tile(t, bx, by, kchunk, waves)
    with torch.cuda.device(lam_a.device):
        check(_lib.load().jacobi_adjoint(dtype_code(lam_a), ctypes.byref(grid_of(lam_a)),
                                         _ptr(lam_a), _ptr(lam_b), int(T), ctypes.byref(tile),
                                         _ptr(ws), ws.numel(), _stream(lam_a), ctypes.byref(out)))
    return lam_b if out.value else lam_a


def fill(x, value):
    """Every element of grid x (shell included) set to value."""
    with torch.cuda.device(x.device):
        check(_lib.load().jacobi_fill(dtype_code(x), ctypes.byref(grid_of(x)), _ptr(x),
                                      float(value), _stream(x)))
    return x


def grid_add(dst, src):
    """dst += src on every element of a grid, shell included (in place;
    returns dst).  dst and src: same dtype, shape and strides."""
    if src.dtype != dst.dtype or src.shape != dst.shape or src.stride() != dst.stride() \
            or src.device != dst.device:
        raise ValueError("dst and src must have the same dtype, shape, strides and device")
    with torch.cuda.device(dst.device):
        check(_lib.load().jacobi_grid_add(dtype_code(dst), ctypes.byref(grid_of(dst)), _ptr(dst),
                                          _ptr(src), _stream(dst)))
    return dst


def residual_workspace(x):
    n = _lib.load().jacobi_residual_workspace(ctypes.byref(grid_of(x)))
    if n == 0:
        check(_lib.JAC_EARG)
    return torch.empty(n, dtype=torch.uint8, device=x.device)


def residual_f64(x, r32, norm2, ws=None):
    """r32 <- (float)(b - A x) on the interior (FP64 arithmetic); norm2[0] <-
    |b - A x|^2 (device float64 tensor of one element)."""
    if x.dtype != torch.float64 or r32.dtype != torch.float32 or norm2.dtype != torch.float64:
        raise TypeError("residual_f64 needs float64 x, float32 r32 and a float64 norm2")
    if x.shape != r32.shape or x.stride() != r32.stride():
        raise ValueError("x and r32 must share shape and strides")
    if ws is None:
        ws = residual_workspace(x)
    with torch.cuda.device(x.device):
        check(_lib.load().jacobi_residual_f64(ctypes.byref(grid_of(x)), _ptr(x), _ptr(r32),
                                              _ptr(norm2), _ptr(ws), ws.numel(), _stream(x)))
    return norm2


def residual_f64_noalloc(x, r32, norm2):
    """residual_f64 with no workspace (jacobi_residual_f64_noalloc): the
    library's fixed per-GPU array holds the partial sums; nothing is
    allocated.  Calls that overlap in time on one GPU race."""
    if x.dtype != torch.float64 or r32.dtype != torch.float32 or norm2.dtype != torch.float64:
        raise TypeError("residual_f64_noalloc needs float64 x, float32 r32 and a float64 norm2")
    if x.shape != r32.shape or x.stride() != r32.stride():
        raise ValueError("x and r32 must share shape and strides")
    with torch.cuda.device(x.device):
        check(_lib.load().jacobi_residual_f64_noalloc(ctypes.byref(grid_of(x)), _ptr(x), _ptr(r32),
                                                      _ptr(norm2), _stream(x)))
    return norm2


def update_f64(x, e32):
    """x += (double)e32 on the interior."""
    if x.dtype != torch.float64 or e32.dtype != torch.float32:
        raise TypeError("update_f64 needs float64 x and float32 e32")
    if x.shape != e32.shape or x.stride() != e32.stride():
        raise ValueError("x and e32 must share shape and strides")
    with torch.cuda.device(x.device):
        check(_lib.load().jacobi_update_f64(ctypes.byref(grid_of(x)), _ptr(x), _ptr(e32),
                                            _stream(x)))
    return x


def update_residual_f64(x, e32, x_new, r32, zero32, norm2, ws=None):
    """x_new <- x + (double)e32 and zero32 <- 0 on the interior; r32 and
    norm2 as residual_f64 gives them for x_new.  All six tensors distinct."""
    if (x.dtype != torch.float64 or x_new.dtype != torch.float64 or norm2.dtype != torch.float64
            or e32.dtype != torch.float32 or r32.dtype != torch.float32
            or zero32.dtype != torch.float32):
        raise TypeError("update_residual_f64 needs float64 x, x_new, norm2 and float32 e32, r32, "
                        "zero32")
    for other in (e32, x_new, r32, zero32):
        if other.shape != x.shape or other.stride() != x.stride():
            raise ValueError("the grids must share shape and strides")
    if ws is None:
        ws = residual_workspace(x)
    with torch.cuda.device(x.device):
        check(_lib.load().jacobi_update_residual_f64(
            ctypes.byref(grid_of(x)), _ptr(x), _ptr(e32), _ptr(x_new), _ptr(r32), _ptr(zero32),
            _ptr(norm2), _ptr(ws), ws.numel(), _stream(x)))
    return x_new


class BatchPlan:
    """A batched run over independent grids (one blocking choice for all).

    Builds the plan image on the host (jacobi_batched_plan), keeps a device
    copy and the counter workspace, and enqueues the run with run(); run()
    makes no host copies and allocates nothing, so it can be captured in a
    CUDA/HIP graph and replayed.  results() names, per grid, the tensor that
    holds level T after a run."""

    MODES = {"relaxed": _lib.JAC_BATCH_RELAXED, "lockstep": _lib.JAC_BATCH_LOCKSTEP}

    def __init__(self, grids_a, grids_b, Ts, t=None, bx=0, by=0, kchunk=0, waves=0):
        n = len(grids_a)
        if n != len(grids_b) or n != len(Ts) or n == 0:
            raise ValueError("need equal, non-empty lists of a grids, b grids and sweep counts")
        for a, b in zip(grids_a, grids_b):
            _same(a, b)
        self.a, self.b = list(grids_a), list(grids_b)
        self.dtype = grids_a[0].dtype
        if any(x.dtype != self.dtype for x in grids_a):
            raise TypeError("all grids of a batch share one dtype")
        lib = _lib.load()
        code = dtype_code(grids_a[0])
        G = (Grid * n)(*[grid_of(x) for x in grids_a])
        T = (ctypes.c_int * n)(*[int(v) for v in Ts])
        A = (ctypes.c_void_p * n)(*[x.data_ptr() for x in grids_a])
        B = (ctypes.c_void_p * n)(*[x.data_ptr() for x in grids_b])
        tile = _tile(t, bx, by, kchunk, waves)
        nbytes = lib.jacobi_batched_plan_bytes(code, n, G, T, ctypes.byref(tile))
        self.out_idx = (ctypes.c_int * n)()
        if nbytes == 0:     # the plan call repeats the failed check and returns its code
            check(lib.jacobi_batched_plan(code, n, G, A, B, T, ctypes.byref(tile), None, 0,
                                          self.out_idx) or _lib.JAC_EARG)
        self._host = (ctypes.c_ubyte * nbytes)()
        check(lib.jacobi_batched_plan(code, n, G, A, B, T, ctypes.byref(tile), self._host, nbytes,
                                      self.out_idx))
        dev = grids_a[0].device
        self.plan_dev = torch.frombuffer(bytearray(self._host), dtype=torch.uint8).to(dev)
        ws = lib.jacobi_batched_workspace(self._host)
        self.ws = torch.zeros(max(ws, 8), dtype=torch.uint8, device=dev)
        self.device = dev

    def run(self, mode="relaxed"):
        with torch.cuda.device(self.device):
            check(_lib.load().jacobi_batched_run(self._host, _ptr(self.plan_dev), _ptr(self.ws),
                                                 self.ws.numel(), self.MODES[mode],
                                                 _stream(self.plan_dev)))
        return self

    def stress(self, seed, max_delay=8):
        """Shuffle the items of each pass and delay some of them
        (jacobi_batched_stress), then refresh the device copy: a test of the
        relaxed synchronisation, whose results must not change."""
        check(_lib.load().jacobi_batched_stress(self._host, len(self._host), int(seed),
                                                int(max_delay)))
        self.plan_dev.copy_(torch.frombuffer(bytearray(self._host), dtype=torch.uint8))
        return self

    def items(self):
        """The plan's work items (grid, pass, block, delay) in queue order,
        read back from the host image (layout in csrc/kernels.h)."""
        import struct
        raw = bytes(self._host)
        hdr = struct.unpack_from("<I9i5q", raw, 0)
        nitems, items_off = hdr[3], hdr[11]
        return [struct.unpack_from("<4i", raw, items_off + 16 * i) for i in range(nitems)]

    def results(self):
        return [b if o else a for a, b, o in zip(self.a, self.b, self.out_idx)]

    def wait_error(self):
        """True if a relaxed-mode wait gave up (read after synchronising)."""
        return bool(self.ws[-4:].view(torch.int32).item())

    def geometry(self):
        """Per grid, the plan's block geometry read back from the host image
        (layout of the plan header and per-grid records in csrc/kernels.h):
        dicts of nx, ny, nz, block columns nti x ntj, k chunks nkc of kchunk
        planes, i-halo hi, T, passes and the plan's depth t."""
        import struct
        raw = bytes(self._host)
        hdr = struct.unpack_from("<I9i5q", raw, 0)
        n, cfg_t, grids_off = hdr[2], hdr[6], hdr[10]
        out = []
        for m in range(n):
            g = struct.unpack_from("<QQqq16i", raw, grids_off + 96 * m)
            nx, ny, nz, nti, ntj, nkc, hi, kchunk, T, passes = g[4:14]
            out.append(dict(nx=nx, ny=ny, nz=nz, nti=nti, ntj=ntj, nkc=nkc, hi=hi, kchunk=kchunk,
                            T=T, passes=passes, t=cfg_t))
        return out


class PipelinePlan(BatchPlan):
    """Pipelined temporal blocking of one grid (jacobi_pipelined_plan): T
    sweeps as passes of t sweeps per block, segments of `team` passes
    streaming through k chunks of `kchunk` planes a few chunks apart, with
    the relaxed synchronisation of Eq. 3: lower distance dl, upper distance
    du (0: none; dl = du = 1 is lock-step) and team delay dt, in chunks
    beyond the one-chunk halo.  Runs in relaxed mode only; results()[0]
    holds level T."""

    def __init__(self, a, b, T, team=4, t=1, bx=0, by=0, kchunk=0, waves=0, dl=1, du=0, dt=0):
        _same(a, b)
        self.a, self.b = [a], [b]
        self.dtype = a.dtype
        lib = _lib.load()
        code = dtype_code(a)
        g = grid_of(a)
        tile = _tile(t, bx, by, kchunk, waves)
        sync = _lib.Pipeline(int(dl), int(du), int(dt))
        nbytes = lib.jacobi_pipelined_plan_bytes(code, ctypes.byref(g), int(T), ctypes.byref(tile))
        self.out_idx = (ctypes.c_int * 1)()
        if nbytes == 0:     # the plan call repeats the failed check and returns its code
            check(lib.jacobi_pipelined_plan(code, ctypes.byref(g), _ptr(a), _ptr(b), int(T),
                                            int(team), ctypes.byref(sync), ctypes.byref(tile), None,
                                            0, self.out_idx) or _lib.JAC_EARG)
        self._host = (ctypes.c_ubyte * nbytes)()
        check(lib.jacobi_pipelined_plan(code, ctypes.byref(g), _ptr(a), _ptr(b), int(T), int(team),
                                        ctypes.byref(sync), ctypes.byref(tile), self._host, nbytes,
                                        self.out_idx))
        self.plan_dev = torch.frombuffer(bytearray(self._host), dtype=torch.uint8).to(a.device)
        ws = lib.jacobi_batched_workspace(self._host)
        self.ws = torch.zeros(max(ws, 8), dtype=torch.uint8, device=a.device)
        self.device = a.device


def pipelined(a, b, T, team=4, t=1, bx=0, by=0, kchunk=0, waves=0, dl=1, du=0, dt=0):
    """Level T of grid a by pipelined temporal blocking; returns the tensor
    (a or b) that holds it."""
    return PipelinePlan(a, b, T, team, t, bx, by, kchunk, waves, dl, du, dt).run("relaxed").results()[0]


def compressed_shape(nx, ny, nz, t):
    """Shape (nz+2, ny+2+t, nx+2+t) of a compressed-grid array for depth t."""
    return (nz + 2, ny + 2 + t, nx + 2 + t)


def compressed_frame(u, t, frame):
    """View of frame 0 (cell (i, j, k) at u[k, j+t, i+t]) or frame 1 (at
    u[k, j, i]) of a compressed-grid array u, shaped like a grid."""
    if u.dim() != 3:
        raise ValueError("a compressed-grid array is 3-D")
    ny, nx = u.shape[1] - 2 - t, u.shape[2] - 2 - t
    if ny < 1 or nx < 1:
        raise ValueError(f"array {tuple(u.shape)} is too small for depth t = {t}")
    return u[:, t:, t:] if frame == 0 else u[:, :ny + 2, :nx + 2]


def compressed_grid(u, t):
    """jac_grid_t of a compressed-grid array (interior and array strides)."""
    if u.dim() != 3 or u.stride(2) != 1:
        raise ValueError("a compressed-grid array is 3-D and contiguous along i")
    nz, ny, nx = u.shape[0] - 2, u.shape[1] - 2 - t, u.shape[2] - 2 - t
    return Grid(nx, ny, nz, u.stride(1), u.stride(0))


class Compressed:
    """T sweeps in one array (jacobi_compressed): u has compressed_shape()
    and holds level 0 in frame 0.  run() enqueues the passes (no host copies,
    no allocation); result() is the view of the frame holding level T."""

    def __init__(self, u, T, t, bx=0, by=0, kchunk=0, waves=0):
        if u.dtype not in _DTYPES:
            raise TypeError(f"grids must be float32 or float64, got {u.dtype}")
        self.u, self.T, self.t = u, int(T), int(t)
        self.g = compressed_grid(u, self.t)
        self.tile = _tile(t, bx, by, kchunk, waves)
        lib = _lib.load()
        nbytes = lib.jacobi_compressed_workspace(_DTYPES[u.dtype], ctypes.byref(self.g), self.T,
                                                 ctypes.byref(self.tile))
        if nbytes == 0:
            check(_lib.JAC_EARG)
        self.ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device=u.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + nbytes]
        self.frame = 0

    def run(self):
        out = ctypes.c_int(0)
        with torch.cuda.device(self.u.device):
            check(_lib.load().jacobi_compressed(
                _DTYPES[self.u.dtype], ctypes.byref(self.g), _ptr(self.u), self.T,
                ctypes.byref(self.tile), _ptr(self.ws_view), self.ws_view.numel(), _stream(self.u),
                ctypes.byref(out)))
        self.frame = out.value
        return self

    def result(self):
        return compressed_frame(self.u, self.t, self.frame)

    def wait_error(self):
        """True if a wait gave up (read after synchronising)."""
        return bool(self.ws_view[:4].view(torch.int32).item())


def compressed(u, T, t, bx=0, by=0, kchunk=0, waves=0):
    """Level T of the grid in frame 0 of u, computed in place; returns the
    view of the frame that holds it."""
    return Compressed(u, T, t, bx, by, kchunk, waves).run().result()


def batched(grids_a, grids_b, Ts, t=None, bx=0, by=0, kchunk=0, mode="relaxed", waves=0):
    """Level T[m] of every grid m (one launch); returns the result tensors."""
    return BatchPlan(grids_a, grids_b, Ts, t, bx, by, kchunk, waves).run(mode).results()


def autotune(a, b, T, tmax=0, reps=2):
    """Time every block shape and depth for T sweeps on grids a, b (their
    contents are overwritten); returns ((t, bx, by, waves), ms) of the fastest
    and makes it the library's choice for this geometry and T."""
    _same(a, b)
    best = Tile()
    ms = ctypes.c_float(0)
    with torch.cuda.device(a.device):
        check(_lib.load().jacobi_autotune(dtype_code(a), ctypes.byref(grid_of(a)), _ptr(a), _ptr(b),
                                          int(T), int(tmax), int(reps), ctypes.byref(best),
                                          ctypes.byref(ms), _stream(a)))
    return (best.t, best.bx, best.by, best.waves), ms.value


def tune_save(path):
    """Write the library's tuning choices (every architecture) to a text file."""
    check(_lib.load().jacobi_tune_save(os.fsencode(path)))


def tune_load(path):
    """Add the tuning choices of a file written by tune_save (or named by
    JACOBI_TUNE_CACHE); returns how many it held."""
    n = ctypes.c_int(0)
    check(_lib.load().jacobi_tune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_lookup(grid, T, dtype=torch.float64, arch=None):
    """The remembered choice (t, bx, by, kchunk, waves) for a grid (a tensor,
    or (nx, ny, nz)) and T on `arch` (None: the current device's), or None."""
    g = grid_of(grid) if isinstance(grid, torch.Tensor) else Grid(*grid, 0, 0)
    code = dtype_code(grid) if isinstance(grid, torch.Tensor) else (1 if dtype == torch.float64 else 0)
    tile = Tile()
    rc = _lib.load().jacobi_tune_lookup(arch.encode() if arch else None, code, ctypes.byref(g),
                                         int(T), ctypes.byref(tile))
    if rc == _lib.JAC_EUNSUPPORTED:
        return None
    check(rc)
    return tile.t, tile.bx, tile.by, tile.kchunk, tile.waves


def tune_forget():
    """Forget every tuning choice of this process."""
    check(_lib.load().jacobi_tune_forget())


def autotune_batch(grids_a, grids_b, Ts, candidates=None, mode="relaxed", reps=2):
    """Pick the (t, bx, by) of a batched run by timing the whole batch for
    each candidate (the grids' contents are overwritten).  Returns
    ((t, bx, by, waves), ms)."""
    if candidates is None:
        candidates = [(t, bx, by, w) for (bx, by, w) in tile_menu(grids_a[0].dtype)
                      for t in range(2, 7)]
    best, best_ms = None, float("inf")
    st = torch.cuda.current_stream(grids_a[0].device)
    for (t, bx, by, w) in candidates:
        try:
            plan = BatchPlan(grids_a, grids_b, Ts, t=t, bx=bx, by=by, waves=w)
            plan.run(mode)
        except _lib.JacobiError:
            continue
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            plan.run(mode)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if ms < best_ms:
            best, best_ms = (t, bx, by, w), ms
    return best, best_ms


def lbm_d3q19(f, f_tmp, omega, T, blocked=False, kchunk=0):
    """T D3Q19 lattice Boltzmann steps (BGK, periodic box) on populations f of
    shape (19, nz, ny, nx) (contiguous, float32 or float64); f_tmp is a second
    buffer like f.  blocked: two steps per pass over memory
    (lbm_d3q19_blocked; kchunk z planes per workgroup, 0 = library choice),
    bitwise the same results.  Returns the tensor (f or f_tmp) holding step T."""
    if f.shape != f_tmp.shape or f.dtype != f_tmp.dtype or f.device != f_tmp.device:
        raise ValueError("f and f_tmp must share shape, dtype and device")
    if f.dim() != 4 or f.shape[0] != 19 or not (f.is_contiguous() and f_tmp.is_contiguous()):
        raise ValueError("populations must be contiguous tensors of shape (19, nz, ny, nx)")
    _, nz, ny, nx = f.shape
    out = ctypes.c_int(0)
    with torch.cuda.device(f.device):
        lib = _lib.load()
        if blocked:
            check(lib.lbm_d3q19_blocked(dtype_code(f), ctypes.byref(_lib.LbmGrid(nx, ny, nz)),
                                        _ptr(f), _ptr(f_tmp), float(omega), int(T), int(kchunk),
                                        _stream(f), ctypes.byref(out)))
        else:
            check(lib.lbm_d3q19_steps(dtype_code(f), ctypes.byref(_lib.LbmGrid(nx, ny, nz)),
                                      _ptr(f), _ptr(f_tmp), float(omega), int(T), _stream(f),
                                      ctypes.byref(out)))
    return f_tmp if out.value else f
