"""ctypes binding of libjacobi.so (argument marshalling only).

The library is loaded after PyTorch, so it shares the HIP runtime PyTorch
already loaded.  There is no fallback: if the library is missing, loading
fails with an error that says how to build it.
"""
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjacobi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "jacobi.h")

JAC_F32, JAC_F64 = 0, 1
JAC_OK, JAC_EARG, JAC_EHIP, JAC_EWORKSPACE, JAC_EUNSUPPORTED = 0, -1, -2, -3, -4
MAX_DEPTH = 8
ABI_VERSION = 3
JAC_BATCH_RELAXED, JAC_BATCH_LOCKSTEP = 0, 1


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("sy", ctypes.c_int64), ("sz", ctypes.c_int64)]


class Tile(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("bx", ctypes.c_int32), ("by", ctypes.c_int32),
                ("kchunk", ctypes.c_int32), ("waves", ctypes.c_int32)]


class LbmGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Pipeline(ctypes.Structure):
    _fields_ = [("dl", ctypes.c_int32), ("du", ctypes.c_int32), ("dt", ctypes.c_int32)]


class JacobiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libjacobi error {code}: {msg}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_GP = ctypes.POINTER(Grid)
_TP = ctypes.POINTER(Tile)
_IP = ctypes.POINTER(ctypes.c_int)

SIGNATURES = {
    "jacobi_version": ([], ctypes.c_int),
    "jacobi_last_error": ([], ctypes.c_char_p),
    "jacobi_plain": ([ctypes.c_int, _GP, _P, _P, ctypes.c_int, _P, _IP], ctypes.c_int),
    "jacobi_tblock": ([ctypes.c_int, _GP, _P, _P, ctypes.c_int, _TP, _P, _P, _IP], ctypes.c_int),
    "jacobi_adjoint_workspace": ([ctypes.c_int, _GP, ctypes.c_int], ctypes.c_size_t),
    "jacobi_adjoint": ([ctypes.c_int, _GP, _P, _P, ctypes.c_int, _TP, _P, ctypes.c_size_t, _P,
                        _IP], ctypes.c_int),
    "jacobi_residual_workspace": ([_GP], ctypes.c_size_t),
    "jacobi_residual_f64": ([_GP, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "jacobi_update_f64": ([_GP, _P, _P, _P], ctypes.c_int),
    "jacobi_residual_f64_noalloc": ([_GP, _P, _P, _P, _P], ctypes.c_int),
    "jacobi_update_residual_f64": ([_GP, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
                                   ctypes.c_int),
    "jacobi_fill": ([ctypes.c_int, _GP, _P, ctypes.c_double, _P], ctypes.c_int),
    "jacobi_grid_add": ([ctypes.c_int, _GP, _P, _P, _P], ctypes.c_int),
    "jacobi_copy": ([_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "jacobi_tune_save": ([ctypes.c_char_p], ctypes.c_int),
    "jacobi_tune_load": ([ctypes.c_char_p, _IP], ctypes.c_int),
    "jacobi_tune_lookup": ([ctypes.c_char_p, ctypes.c_int, _GP, ctypes.c_int, _TP], ctypes.c_int),
    "jacobi_tune_forget": ([], ctypes.c_int),
    "jacobi_batched_plan_bytes": ([ctypes.c_int, ctypes.c_int, _GP, _IP, _TP], ctypes.c_size_t),
    "jacobi_batched_plan": ([ctypes.c_int, ctypes.c_int, _GP, ctypes.POINTER(_P),
                             ctypes.POINTER(_P), _IP, _TP, _P, ctypes.c_size_t, _IP], ctypes.c_int),
    "jacobi_batched_workspace": ([_P], ctypes.c_size_t),
    "jacobi_batched_stress": ([_P, ctypes.c_size_t, ctypes.c_uint, ctypes.c_int], ctypes.c_int),
    "jacobi_batched_run": ([_P, _P, _P, ctypes.c_size_t, ctypes.c_int, _P], ctypes.c_int),
    "jacobi_pipelined_plan_bytes": ([ctypes.c_int, _GP, ctypes.c_int, _TP], ctypes.c_size_t),
    "jacobi_pipelined_plan": ([ctypes.c_int, _GP, _P, _P, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(Pipeline), _TP, _P, ctypes.c_size_t, _IP],
                              ctypes.c_int),
    "jacobi_compressed_workspace": ([ctypes.c_int, _GP, ctypes.c_int, _TP], ctypes.c_size_t),
    "jacobi_compressed": ([ctypes.c_int, _GP, _P, ctypes.c_int, _TP, _P, ctypes.c_size_t, _P, _IP],
                          ctypes.c_int),
    "jacobi_tile_menu": ([ctypes.c_int, _IP, ctypes.c_int], ctypes.c_int),
    "lbm_d3q19_steps": ([ctypes.c_int, ctypes.POINTER(LbmGrid), _P, _P, ctypes.c_double,
                         ctypes.c_int, _P, _IP], ctypes.c_int),
    "lbm_d3q19_blocked": ([ctypes.c_int, ctypes.POINTER(LbmGrid), _P, _P, ctypes.c_double,
                           ctypes.c_int, ctypes.c_int, _P, _IP], ctypes.c_int),
    "jacobi_autotune": ([ctypes.c_int, _GP, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _TP,
                         ctypes.POINTER(ctypes.c_float), _P], ctypes.c_int),
    "jacobi_default_tile": ([ctypes.c_int, _GP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _TP],
                            ctypes.c_int),
}


HEADERS = [HEADER, os.path.join(os.path.dirname(_HERE), "include", "lbm.h")]


def declared_symbols():
    """Function names the public headers (include/jacobi.h, include/lbm.h) declare."""
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:jacobi|lbm)_\w+)\s*\(", text))
    return sorted(names)


def load():
    """Load libjacobi.so (after torch, to share its HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library links against)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python paper_0912_4506_amd/csrc/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [name for name in SIGNATURES if not hasattr(lib, name)]
    if missing:
        raise RuntimeError(f"{LIB_PATH} lacks {', '.join(missing)}: it is older than this "
                           "binding; rebuild it")
    for name, (args, res) in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if lib.jacobi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {lib.jacobi_version()}, this binding "
                           f"needs {ABI_VERSION}; rebuild it")
    _lib = lib
    return lib


def last_error():
    return load().jacobi_last_error().decode()


def check(rc):
    if rc != JAC_OK:
        raise JacobiError(rc, last_error())
    return rc
