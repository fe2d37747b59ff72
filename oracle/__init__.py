"""FP64 CPU oracle of the higher-order charge-conserving EM-FEMPIC method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
under ``oracle/``.  The product path (the ``paper_2111_12411_amd`` package and
its HIP library) shares no code with it and never calls it.
"""
