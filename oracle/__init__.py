"""Plain FP64 CPU oracle of the adaptive wavelet TRiSK method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``, never by the product path.  It shares no code with the
HIP library; both receive their inputs from ``paper_1404_0405_amd.inputs``.
"""
