"""MI355X (gfx950) block-wise two-source extractor.

Per block pair, the inner product over F_{2^m} of Def. 3.2, over consecutive
equal blocks (Algorithm 1) of two raw sample streams, computed by hand-written
HIP kernels behind the C ABI in include/qrng_ext.h.

Submodules:
  binding -- ctypes binding of libqrngext.so (Extractor, Stream)
  inputs  -- seeded synthetic ADC-style raw data and workloads
  build   -- compile libqrngext.so for gfx950
"""
__all__ = ["binding", "inputs", "build"]
