"""CPU oracle for the IMEX-TR Landau-Brazovskii hot path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The GPU library shares no code with it.
"""
