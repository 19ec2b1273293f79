"""MI355X-native multiple-right-hand-side setup for DD-alpha-AMG.

The GPU library (HIP, gfx950) sits behind the C-ABI declared in include/mrhs.h;
paper_1601_03184_amd.mrhs is its Python binding.  Importing this package loads
nothing: the binding loads the shared library on first use and raises if it is
missing.
"""
