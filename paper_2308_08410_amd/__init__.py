"""Geodesic-BP hot path on AMD Instinct MI355X (gfx950).

The compute lives in ``libgbp.so`` (HIP kernels behind the C ABI of
``include/gbp.h``); ``paper_2308_08410_amd.binding`` marshals PyTorch tensors
into it.  Importing the binding requires the built library.
"""

__all__ = ["binding", "build"]
