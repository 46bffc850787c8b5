"""MI355X-native k-space time-reversal FWI gradient (arXiv 2102.00755).

The compute path is the HIP library ``libfwi.so`` (C-ABI in include/fwi.h);
this package only marshals arguments.  Importing ``paper_2102_00755_amd.fwi``
requires the built library; there is no CPU fallback.
"""

__all__ = ["fwi", "build"]
