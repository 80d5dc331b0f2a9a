"""MI355X-native parallel block-based Viterbi decoder (arXiv 1608.00066).

The decoder runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libpbvd.so`` (declared in ``include/pbvd.h``).
``paper_1608_00066_amd.pbvd`` is the thin ctypes binding with the same
entry-point names; ``paper_1608_00066_amd.datagen`` makes seeded channel
inputs; ``paper_1608_00066_amd.build`` compiles the library in-tree.
"""
