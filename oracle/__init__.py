"""CPU FP64 oracle for the SSN kernel-OT hot path.  TEST INFRASTRUCTURE ONLY: imported by ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``, never by the product package."""
from . import kot_oracle  # noqa: F401
