"""MI355X-native curvilinear steepest-descent micromagnetic energy minimizer.

The HIP library and its ctypes binding load on first use (``binding``);
importing the package itself loads no native code.
"""
import importlib

__all__ = ["meshgen", "binding"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
