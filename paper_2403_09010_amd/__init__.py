"""MI355X-native symmetric-deletion Levenshtein neighbour search.

The search runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/symdel.h`` (``libsymdel.so``, built in-tree by ``build.py``);
``symdel`` is the thin ctypes binding.
"""
from .symdel import Context, Index, Pairs, Server, SymdelError, load_library, LIB_PATH  # noqa: F401
from .symdel import (OPT_TIMING, OPT_PATH, OPT_GROUP_CAP, OPT_GROUP_BITS, OPT_SORT_ITEMS,  # noqa: F401
                     OPT_BATCH_TILE, OPT_PROBE, OPT_GROUP_BATCHES, MLP_PARAMS)
