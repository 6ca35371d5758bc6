"""Euler characteristic curves of 2D/3D images on MI355X (gfx950).

The computation lives in the HIP library ``libecc_hip.so`` behind the C ABI of
``include/ecc.h``; ``paper_2203_09087_amd.ecc`` is its Python binding.  Importing
this package loads nothing; the library is loaded on first use and an error is
raised if it has not been built.
"""
__all__ = ["ecc", "synth", "build"]
