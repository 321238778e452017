"""MI355X-native ProbMinHash signatures (Ertl, IEEE TKDE 2020, arXiv 1911.00675).

The compute path is the HIP library ``libpmh.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/pmh.h``; ``paper_1911_00675_amd.pmh`` is its
Python binding and ``paper_1911_00675_amd.workloads`` holds the seeded input
generators.  Submodules are imported explicitly by their users.
"""
