"""Test infrastructure only: the plain CPU oracle for the Jacobi eigensolver/SVD.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it, and it
imports nothing from the GPU library.
"""
