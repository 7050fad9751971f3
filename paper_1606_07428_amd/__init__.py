"""MI355X-native (gfx950) rigid-body Stokes mobility solver.

The compute path lives in the HIP/C++ library ``librbm.so`` built from
``csrc/`` (C-ABI declared in ``include/rbm.h``); ``rbm`` is its thin ctypes
binding.  Importing this package loads nothing; ``rbm.load()`` loads the library
and raises if it is missing.
"""
