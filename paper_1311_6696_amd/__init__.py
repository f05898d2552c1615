"""MI355X-native boundary-MPS environments of finite PEPS (arXiv:1311.6696).

The compute path is the HIP library ``libpepsenv.so`` behind the C ABI of
``include/peps_env.h``; ``paper_1311_6696_amd.binding`` is a thin ctypes
wrapper over it.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
