"""FP64 CPU oracle of the parallel pooled pCN sampler -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  It shares no code with
the GPU library.
"""
