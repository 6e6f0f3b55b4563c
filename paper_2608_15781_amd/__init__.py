"""MI355X-native reactive colour-gradient lattice Boltzmann step (hand-written HIP for gfx950).

The compute path is the C-ABI library ``liblbm.so`` built from ``csrc/``; ``core`` is a thin
ctypes binding over it (argument marshalling only). Importing this package loads nothing;
``core.Lbm`` loads the library on first use and raises if it has not been built.
"""
__all__ = ["inputs", "core"]
