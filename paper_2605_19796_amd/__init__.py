"""MI355X-native filtering, Favre filtering, SGS tensors and closures on periodic grids.

The compute path is the HIP library ``libkcf.so`` (C ABI declared in include/kcf.h);
``kcf`` is its ctypes binding, ``synth`` produces seeded synthetic input fields, and
``build`` compiles the library for gfx950. Importing the package loads nothing.
"""
__all__ = ["kcf", "synth", "build"]
