"""CPU FP64 oracle for tensor-kernel l_p regression over the packed layout.

TEST INFRASTRUCTURE ONLY: this package may be imported only by ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``.  It
shares no code with the GPU library (``paper_2003_10482_amd``) and neither
imports the other.  Inputs come from ``synth`` (seeded generators, no method
arithmetic).

Modules
-------
layout     packed sizes, ranks and the nested-loop order (Section 5)
tensor     packed build / contraction / derivative via the C oracle, the full
           tensor and closed forms (Section 4)
dual       dual objective, damped-Newton dual solve, primal recovery,
           prediction, support and model-selection derivatives (Sections 4, 6)
precision  round-to-nearest-even storage rounding (FP32, BF16)

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` except the figure-level feature-selection counts of
Section 6.3, which are unseeded in the paper ("parity unpinned"; only the
threshold rule itself is pinned).
"""
