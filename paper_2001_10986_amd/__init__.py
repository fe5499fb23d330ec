"""MI355X-native entropic domain decomposition for W2 optimal transport.

The compute path is the HIP library built from ``csrc/`` (C-ABI declared in
``include/dd.h``); ``dd`` is its thin ctypes binding.  Importing the package
does not load the library; ``paper_2001_10986_amd.dd`` does, and raises if it
is missing.
"""
