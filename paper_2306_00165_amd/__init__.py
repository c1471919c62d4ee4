"""pcfv: adjoint-descent equilibria of plane Couette flow on MI355X (gfx950).

The compute path is the HIP library ``libpcfv.so`` behind the C ABI declared
in ``include/pcfv.h``; ``paper_2306_00165_amd.pcfv`` is its thin ctypes
binding.  Importing the package loads nothing; ``inputs`` holds the seeded
input generators.
"""
