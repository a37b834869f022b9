"""FP64 CPU oracle of the ternary free-energy entropic LBM update.

Test infrastructure only: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the GPU library.
"""
