"""FliX flipped-index batch operations on MI355X (gfx950).

The compute path is the HIP library ``libflix.so`` behind the C ABI declared
in ``include/flix.h``; ``flix.py`` is a thin ctypes binding over it.
"""
