"""MI355X (gfx950) inaccessibility measure field (IMF) library.

The compute path is the HIP library ``libimf.so`` (C interface in
``include/imf.h``); this package only marshals arguments to it.  PyTorch
provides device memory and streams.
"""
from .imf import (Context, Stats, IMFError, TOOL_FLAT, TOOL_BALL, TOOL_RECT2D, TOOL_VOXEL,
                  DIR_F64, DIR_LATTICE, DIR_ROTATION, SHARP_ALL, SHARP_BOUNDARY, SHARP_TIP, METHOD_AUTO, METHOD_FFT,
                  METHOD_DIRECT, FLAG_PLAIN, FLAG_MASK_SWEEP, FLAG_NO_CACHE, FLAG_PROFILE,
                  FLAG_NO_BOUND, FLAG_NO_GRAPH,
                  KERNEL_CLASSES, library_path,
                  fft_size)

__all__ = ["Context", "Stats", "IMFError", "TOOL_FLAT", "TOOL_BALL", "TOOL_RECT2D", "TOOL_VOXEL",
           "DIR_F64", "DIR_LATTICE", "DIR_ROTATION", "SHARP_ALL", "SHARP_BOUNDARY", "SHARP_TIP", "METHOD_AUTO",
           "METHOD_FFT", "METHOD_DIRECT", "FLAG_PLAIN", "FLAG_MASK_SWEEP", "FLAG_NO_CACHE",
           "FLAG_PROFILE", "FLAG_NO_BOUND", "FLAG_NO_GRAPH", "KERNEL_CLASSES",
           "library_path", "fft_size"]
