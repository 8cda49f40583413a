"""MI355X-native spectral Gauss-quadrature electron density (Lanczos-Gauss LSSGQ).

The compute path lives in the HIP library ``libsgq.so`` (``csrc/``), reached through
the C ABI declared in ``include/sgq.h``; :mod:`.sgq` is the thin ctypes binding.
"""
