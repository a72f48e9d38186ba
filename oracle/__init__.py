"""CPU FP64 oracle of the angular-momentum-conserving Cartesian FMM.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The GPU solver never imports it.
"""
