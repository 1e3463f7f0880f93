"""MI355X-native encrypted Argmax of SecPE (arXiv 2502.00847).

The product is libsecpe.so (HIP kernels for gfx950 behind the C ABI of
include/secpe.h); ``secpe`` is its thin Python binding.
"""
