"""MI355X-native (gfx950 HIP) RNS-CKKS inverse-square-root hot path.

The arithmetic runs in the C-ABI library ``libckks_hip.so`` (HIP kernels +
C++ host orchestration); ``paper_2606_10477_amd.ckks`` is the thin ctypes
binding with the same names.
"""
