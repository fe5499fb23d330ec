"""Oracle of entropic domain decomposition for W2 optimal transport.

TEST INFRASTRUCTURE ONLY.  Only tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from here; the
product path (the HIP library and its Python binding) never does.

- ``ddo``:   ctypes binding of the FP64 C oracle (sparse Algorithm 2 with the
             multi-scale driver), same call shapes as the GPU C-ABI.
- ``dense``: NumPy FP64 dense references (full-grid entropic OT, dense
             Algorithm 1 with exact cell solves, 1D monotone rearrangement)
             that pin the C oracle.
"""
