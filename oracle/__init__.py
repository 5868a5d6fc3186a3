"""Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

May be imported only by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``. The product path never touches it.
"""
