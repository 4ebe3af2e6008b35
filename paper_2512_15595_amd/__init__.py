"""MI355X-native blocked / sectorized Bloom filter (bulk add and contains).

The compute path is hand-written HIP for gfx950 in ``csrc/`` behind the C ABI
declared in ``include/bf.h``; ``paper_2512_15595_amd.bf`` is its thin Python
binding.  Importing this package does not load the native library; importing
``paper_2512_15595_amd.bf`` does, and fails loudly if it is not built.
"""

__all__ = ["bf", "workloads"]
