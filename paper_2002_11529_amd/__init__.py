"""UT raw-bank decoding and Compass upstream tracking on AMD MI355X (gfx950).

The computation lives in libutcompass.so (hand-written HIP, C ABI in include/ut_compass.h); this
package is its thin ctypes binding.  See api.py.
"""
from .api import (Geometry, compass_params, ut_decode, ut_decode_noalloc, compass_find, compass_fit_grad,
                  compass_fit_freeze, compass_fit_grad_frozen, CompassChi2Function, library, version, autotune, ut_global_event_cut,
                  compass_consolidate,
                  FLAG_BANK_ORDER, FLAG_CAPACITY, FLAG_LAYER_OVERFLOW, FLAG_BANK_SIZE, MAX_BANK_WORDS,
                  NOALLOC_MAX_EVENTS)

__all__ = ["Geometry", "compass_params", "ut_decode", "ut_decode_noalloc", "compass_find", "compass_fit_grad",
           "compass_fit_freeze", "compass_fit_grad_frozen", "CompassChi2Function", "library", "version", "autotune", "ut_global_event_cut",
           "compass_consolidate", "FLAG_BANK_ORDER", "FLAG_CAPACITY",
           "FLAG_LAYER_OVERFLOW", "FLAG_BANK_SIZE", "MAX_BANK_WORDS", "NOALLOC_MAX_EVENTS"]
