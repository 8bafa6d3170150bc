"""MI355X-native fully discrete Active Flux (RB-TAI) step for the 2-D Euler equations.

The compute path is libaf.so (hand-written HIP for gfx950, C ABI in include/af.h);
this package only binds it.  Importing the package loads nothing; the library is
loaded on first use and a missing build raises ImportError.
"""
__all__ = ["inputs", "stepper", "build"]
