"""MI355X-native neural texture compression hot path (arXiv 2305.17105).

The compute lives in the HIP library ``libntc.so`` (C ABI declared in include/ntc.h);
``paper_2305_17105_amd.ntc`` is the thin ctypes binding over it and ``synth`` holds
the seeded synthetic input generators.
"""
