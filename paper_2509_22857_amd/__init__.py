"""MI355X-native leveled RNS-CKKS evaluator for private CNN inference with
quadratic activations (arXiv 2509.22857).

The compute path is the HIP library `_build/libckkscnn.so` (C-ABI in
include/ckkscnn.h); `ckks` is its thin Python binding.
"""
