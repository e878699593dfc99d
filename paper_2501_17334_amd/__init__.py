"""MI355X (gfx950) pooled-pCN Bayesian quantum state tomography.

The compute path is libqst.so (HIP kernels behind the C ABI in include/qst.h);
``paper_2501_17334_amd.qst`` is its thin ctypes binding and
``paper_2501_17334_amd.synth`` the seeded synthetic-data generator.
"""
__all__ = ["qst", "synth"]
