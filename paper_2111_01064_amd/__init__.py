"""MI355X-native heterodyned (relative-binning) and full-grid likelihoods for
massive-black-hole-binary signals with the LISA A/E/T response (Katz 2021,
arXiv:2111.01064).

The compute path is the HIP library ``libmbh.so`` (``csrc/``) behind a C ABI
(``include/mbh.h``); :mod:`paper_2111_01064_amd.mbh` is its thin ctypes binding.
:mod:`paper_2111_01064_amd.inputs` holds the seeded synthetic-input generators.
"""
__all__ = ["inputs", "mbh"]
