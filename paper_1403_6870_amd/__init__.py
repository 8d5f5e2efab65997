"""MI355X (gfx950) implementation of McFarland's modified ziggurat sampler
(arXiv:1403.6870) for exponential and normal pseudorandom numbers.

The product is libzig.so (C ABI in include/zig.h, HIP kernels in csrc/);
`paper_1403_6870_amd.zig` is its Python binding.
"""
