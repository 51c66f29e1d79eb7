"""Chromatic Gibbs sampling of Gaussian Markov random fields on MI355X (gfx950).

The sampler itself lives in the HIP library ``libgmrf.so`` (sources under
``csrc/``, C ABI in ``include/gmrf.h``); :mod:`.gmrf` is its thin ctypes
binding and :mod:`.inputs` builds seeded synthetic workloads.  Importing the
package loads nothing: the library is opened on first use and a missing
library is an error, never a fallback.
"""
__all__ = ["gmrf", "inputs"]
