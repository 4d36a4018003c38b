"""MI355X (gfx950) sparse general matrix-matrix product by row-wise Gustavson.

The product runs in the HIP library ``libmsp.so`` (C ABI in include/msp.h);
``binding`` is its thin ctypes layer and ``gen`` holds the seeded synthetic
input generators.  Importing the package does not load the library.
"""
__all__ = ["binding", "gen"]
