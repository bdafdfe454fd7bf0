"""FP64 CPU oracle for the PoVar hot path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package.  It shares no code with the HIP library.
"""
