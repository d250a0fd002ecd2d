"""MI355X-native symmetric-deletion Levenshtein neighbour search.

The search runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/symdel.h`` (``libsymdel.so``, built in-tree by ``build.py``);
``symdel`` is the thin ctypes binding.
"""
from .symdel import Context, Pairs, SymdelError, load_library, LIB_PATH  # noqa: F401
