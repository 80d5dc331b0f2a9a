"""MI355X-native parallel block-based Viterbi decoder (arXiv 1608.00066).

The decoder runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libpbvd.so`` (declared in ``include/pbvd.h``).  ``pbvd`` is the thin
ctypes binding with the same entry-point names; it is imported lazily so that
``datagen`` stays usable without the GPU library.
"""


def __getattr__(name):
    if name == "pbvd":
        from . import pbvd
        return pbvd
    raise AttributeError(name)
