"""MI355X-native solver for the nonlocal obstacle-potential phase-field model and
its multifidelity Monte Carlo estimator (arXiv 2310.10750).

The compute path is the HIP library ``libnlch.so`` (C ABI declared in
``include/nlch.h``); :mod:`paper_2310_10750_amd.nlch` is its thin ctypes
binding.  :mod:`paper_2310_10750_amd.synth` draws the seeded synthetic inputs.
Importing the package loads nothing; the binding loads the library on first use
and raises if it is missing.
"""
__all__ = ["nlch", "synth"]
