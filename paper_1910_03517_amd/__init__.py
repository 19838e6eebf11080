"""MI355X-native seam-matched exposure / white-balance correction for camera rings.

Submodules are imported on demand so that the input generator can be used
without the compiled library:

  rt        -- ctypes binding of the C-ABI library (libringcorr.so)
  synth     -- seeded synthetic rigs (inputs only)
  build     -- hipcc build of the library for gfx950
"""
__all__ = ["rt", "synth", "build"]
