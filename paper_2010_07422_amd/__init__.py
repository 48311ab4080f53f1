"""IRCUR (Iterated Robust CUR) for robust PCA on AMD Instinct MI355X (gfx950).

The compute path is a C-ABI shared library (``libircur.so``, declared in
``include/ircur.h``) built from hand-written HIP kernels; ``ircur`` in this
package is a thin ctypes binding to it.  Importing the package does not load
the library: the first call does, and it raises if the library is missing.
"""
__all__ = ["ircur", "synth"]
