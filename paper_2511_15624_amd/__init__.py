"""MI355X-native interval bound propagation for security-constrained DCOPF.

The compute path is the HIP library ``libibp.so`` (C ABI declared in
``include/ibp.h``); :mod:`paper_2511_15624_amd.ibp` is its thin ctypes binding
and :mod:`paper_2511_15624_amd.synth` draws seeded synthetic instances.
Importing the package loads nothing; the library is loaded on first use.
"""

__all__ = ["synth", "ibp"]
