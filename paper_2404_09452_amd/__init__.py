"""MI355X-native density-fitted Coulomb/exchange (DF-J/K) build.

The compute path is the HIP library libdfjk.so (C ABI in include/dfjk.h);
importing :mod:`paper_2404_09452_amd.dfjk` loads it and fails loudly when it
is missing.  There is no CPU fallback.
"""


def __getattr__(name):
    if name in ("Plan", "boys", "DFJKError", "PRECISION"):
        from . import dfjk
        return getattr(dfjk, name)
    raise AttributeError(name)
