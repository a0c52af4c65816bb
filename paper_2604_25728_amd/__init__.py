"""MI355X (gfx950) implementation of the SQNGD hot path (arXiv 2604.25728).

The compute lives in ``libsqngd.so`` (hand-written HIP, C ABI declared in
``include/sqngd.h``); :mod:`paper_2604_25728_amd.native` is the thin ctypes
binding, :mod:`paper_2604_25728_amd.autograd` the autograd.Function and
:mod:`paper_2604_25728_amd.optim` the driver of the alternating iteration.
Importing the package loads nothing; the binding loads the library on first use
and raises if it has not been built.
"""

__all__ = ["inputs", "native", "autograd", "optim"]
