"""CPU oracle for the PP-STAT hot path: textbook RNS-CKKS plus the statistics
circuits, written from the definitions.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
under ``oracle/``.  The product library never does, and nothing here imports
the product library.
"""
