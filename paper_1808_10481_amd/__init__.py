"""Hermite-leapfrog time stepping for first-order acoustic systems on MI355X.

The compute path is the HIP library ``libhermite_lf.so`` (C ABI declared in
``include/hl.h``); ``paper_1808_10481_amd.hl`` is its thin Python binding.
``paper_1808_10481_amd.inputs`` holds seeded synthetic inputs.
"""
