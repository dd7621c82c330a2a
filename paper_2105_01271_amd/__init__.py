"""MI355X-native deterministic-sketch low-rank SVD / row ID (arXiv 2105.01271).

The compute path is libdsketch.so (HIP kernels for gfx950 behind the C ABI of
include/dsketch.h); `dsketch` is its thin Python binding and `synth` draws the
seeded synthetic snapshot matrices.
"""
