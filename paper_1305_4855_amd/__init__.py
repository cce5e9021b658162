"""MI355X-native Hough-transform track finding (vote, peaks, assign) for gfx950.

The GPU path lives in the C-ABI library ``libhough.so`` (``include/hough.h``);
``paper_1305_4855_amd.hough`` is its thin ctypes binding.  The binding is not
imported here, so that the synthetic-event generator and the workload
definitions can be used on machines without the library.
"""
__all__ = ["configs", "synth"]
