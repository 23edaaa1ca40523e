"""Wavelet-adaptive block ACM solver hot path for MI355X (gfx950).

The compute path is the C-ABI library ``libwacm.so`` (HIP kernels); import
:mod:`paper_1912_05371_amd.wacm` for the binding.  ``inputs`` and ``cases``
only generate synthetic workloads and do not need the library.
"""
