"""MI355X (gfx950) implementation of the SETD pseudo-spectral step for stochastic
field theories (Johnsrud & Rana, arXiv 2511.22510).

The compute path lives in the HIP library ``libsetd.so`` behind the C ABI
declared in ``include/setd.h``; :mod:`paper_2511_22510_amd.setd` is the thin
ctypes binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
