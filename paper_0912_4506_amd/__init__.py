"""MI355X-native temporally blocked 3D Jacobi sweeps (libjacobi.so + binding).

Submodules load lazily: ``inputs`` and ``perf_model`` are plain Python;
``jacobi`` (and everything that runs on the GPU) loads libjacobi.so, which
must have been built (``__graft_entry__.build()``).
"""
import importlib

__all__ = ["inputs", "perf_model", "jacobi"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
