"""FP64 CPU oracle of the splatting rasterizer with the entropy constraint.

Test infrastructure only: tests/, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of bench.py may use it; the product path never does.
"""
