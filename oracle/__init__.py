"""TEST INFRASTRUCTURE ONLY: the sequential CPU oracle for hash-blocked TSDF fusion.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.
"""
