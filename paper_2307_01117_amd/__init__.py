"""MI355X-native periodic 1D heat stencil (explicit Euler, 3-point Laplacian).

The compute path is the C-ABI library ``libheat.so`` built from ``csrc/``
(hand-written HIP for gfx950).  ``heat`` binds it with ctypes; importing this
package does not load it, so ``inputs`` can be used without a GPU.
"""
__all__ = ["inputs", "heat"]
