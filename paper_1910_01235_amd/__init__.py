"""MI355X-native mean-field EAM + master-equation hot path of the MXE method
(arXiv:1910.01235): HIP kernels behind a C ABI, with a thin ctypes binding."""
