"""MI355X (gfx950) near-field XL-MIMO Gram, beamforming rates and capacity saturation.

The compute path is the HIP library ``libxlmimo.so`` (C ABI in include/xlmimo.h);
``paper_2503_18118_amd.xlmimo`` is its ctypes binding.  The binding is imported
lazily so that ``paper_2503_18118_amd.build`` works before the library exists.
"""
import importlib

__all__ = ["xlmimo", "build"]


def __getattr__(name):
    if name in ("xlmimo", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
