"""MI355X-native SN-like dynamic low-rank thermal radiative transfer.

The computation lives in the HIP library libdlrtrt.so (C-ABI in include/dlrtrt.h);
``paper_2601_18705_amd.dlrtrt`` is its ctypes binding.
"""
